"""Pins of the oracle's iterative methods: Lanczos against dense
diagonalization and its breakdown rule; the cTPQ propagator against the
exact exponential within the Taylor truncation bound, its beta = 0 and large
beta limits and the canonical energy at small size; D(z) by direct solves
against the spectral sum, the Lanczos continued fraction and its analytic
properties; SplitMix64 against its published outputs."""
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import core as O
from paper_2307_13222_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def spin_setup(m, two_sz=0):
    s = O.basis_list(m.n_sites, O.sector_popcount_spin(m.n_sites, two_sz))
    return s, (lambda v: O.spin_hv(m, s, v))


# ---------------------------------------------------------------- Lanczos --

@pytest.mark.parametrize("model", ["chain12", "ladder12", "xxz10"])
def test_lanczos_matches_dense(model):
    m = {"chain12": W.random_heisenberg(12, "chain", 1),
         "ladder12": W.random_heisenberg(12, "ladder", 2),
         "xxz10": W.xxz_chain_j2(10)}[model]
    s, hv = spin_setup(m)
    Ed = np.linalg.eigvalsh(O.spin_sparse(m, s).toarray())
    r = O.lanczos(hv, O.splitmix_uniform(1, 0, len(s)), 200)
    assert abs(O.tridiag_lowest(r["alpha"], r["beta"])[0] - Ed[0]) < 1e-10


def test_lanczos_hubbard_matches_dense():
    m = W.hubbard_square(2, 3, 1.0, 4.0)
    ups, dns = O.hubbard_basis(6, 3, 3)
    Ed = np.linalg.eigvalsh(O.hubbard_sparse(m, ups, dns).toarray())
    r = O.lanczos(lambda v: O.hubbard_hv(m, ups, dns, v), W.random_vector(400, 3), 150)
    assert abs(O.tridiag_lowest(r["alpha"], r["beta"])[0] - Ed[0]) < 1e-10


def test_lanczos_breakdown_on_eigenvector():
    # Ising chain: every basis state is an eigenvector -> breakdown at k = 1
    m = W._spin(8, W.chain_pairs(8), [(1.0, 0.0)] * 8, "ising")
    s, hv = spin_setup(m)
    v0 = np.zeros(len(s)); v0[5] = 1.0
    r = O.lanczos(hv, v0, 50)
    assert r["steps"] == 1
    assert abs(r["alpha"][0] - O.spin_sparse(m, s).diagonal()[5]) < 1e-14


def test_lanczos_ground_vector_is_eigenvector():
    m = W.heisenberg_chain(12)
    s, hv = spin_setup(m)
    v0 = O.splitmix_uniform(2, 0, len(s))
    r = O.lanczos(hv, v0, 120)
    e = O.tridiag_lowest(r["alpha"], r["beta"])[0]
    psi = O.lanczos_ground_vector(hv, v0, r["alpha"], r["beta"])
    assert np.linalg.norm(hv(psi) - e * psi) < 1e-7


def test_tridiag_against_dense():
    rng = np.random.default_rng(0)
    a, b = rng.normal(size=50), np.concatenate([[0.0], rng.normal(size=49)])
    T = np.diag(a) + np.diag(b[1:], 1) + np.diag(b[1:], -1)
    assert np.allclose(O.tridiag_lowest(a, b, 5), np.linalg.eigvalsh(T)[:5], atol=1e-13)


# ------------------------------------------------------------------- cTPQ --

def test_ctpq_step_truncation_bound():
    m = W.heisenberg_chain(10)
    s, hv = spin_setup(m)
    Hd = O.spin_sparse(m, s).toarray()
    rng = np.random.default_rng(5)
    phi = rng.normal(size=len(s)) + 1j * rng.normal(size=len(s))
    phi /= np.linalg.norm(phi)
    nrm = np.abs(np.linalg.eigvalsh(Hd)).max()
    for n_max, dtau in [(6, 0.02), (2, 0.1), (10, 0.01)]:
        out = O.ctpq(hv, phi, n_max, dtau, 1)
        exact = scipy.linalg.expm(-dtau / 2 * Hd) @ phi
        got = out["phi"] * math.sqrt(out["D"][1, 0])   # undo the renormalization
        x = dtau * nrm / 2
        bound = x ** (n_max + 1) / math.factorial(n_max + 1) * math.exp(x)
        assert np.linalg.norm(got - exact) <= bound * 1.0001 + 1e-15
        if n_max == 2:
            assert np.linalg.norm(got - exact) > 1e-8        # the bound is not vacuous


def test_ctpq_beta0_mean_and_low_temperature():
    m = W.heisenberg_chain(12)
    s, hv = spin_setup(m)
    Hd = O.spin_sparse(m, s).toarray()
    ev = np.linalg.eigvalsh(Hd)
    B = 8
    phi0 = np.stack([O.splitmix_complex_gaussian(100 + k, len(s)) for k in range(B)], axis=1)
    out = O.ctpq(hv, phi0, 6, 0.02, 400)
    # beta = 0: <H> averages to Tr H / d within O(|H| / sqrt(d B))
    trd = np.trace(Hd) / len(s)
    assert abs(out["E"][0].mean() - trd) < 4 * np.std(ev) / math.sqrt(len(s) * B)
    # canonical energy E(beta) from the spectrum; TPQ matches within sampling
    for k in (50, 200, 400):
        beta = out["beta"][k]
        wts = np.exp(-beta * (ev - ev[0]))
        e_can = np.sum(ev * wts) / np.sum(wts)
        # TPQ estimate weighted by the per-vector squared norms
        logN = np.cumsum(np.log(out["D"][1:k + 1]), axis=0)[-1]
        wv = np.exp(logN - logN.max())
        e_tpq = np.sum(wv * out["E"][k]) / np.sum(wv)
        assert abs(e_tpq - e_can) < 0.05 * abs(e_can) + 0.05
    # beta = 8 is deep in the low-temperature regime of L = 12
    assert out["E"][400].mean() - ev[0] < 0.2


def test_ctpq_norm_bookkeeping():
    m = W.heisenberg_chain(8)
    s, hv = spin_setup(m)
    Hd = O.spin_sparse(m, s).toarray()
    phi = O.splitmix_complex_gaussian(3, len(s))
    out = O.ctpq(hv, phi, 12, 0.05, 10)
    # prod_l D_l = N_k = |U_c^k phi|^2 (D_0 = N_0)
    acc = np.zeros_like(Hd); term = np.eye(len(s))
    for n in range(13):
        acc = acc + term
        term = term @ (-0.05 / 2 * Hd) / (n + 1)
    x = phi.copy()
    for _ in range(10):
        x = acc @ x
    assert abs(np.prod(out["D"][:11]) / np.vdot(x, x).real - 1) < 1e-10


# ---------------------------------------------------------------- D(z) ----

def sqw_setup(n=10, q=math.pi, lattice="chain", seed=3):
    m = W.random_heisenberg(n, lattice, seed)
    s, hv = spin_setup(m, n % 2)
    Hs = O.spin_sparse(m, s)
    ev, U = np.linalg.eigh(Hs.toarray())
    psi = U[:, 0]
    b = O.szq_excitation(m, s, q, psi)
    return m, s, hv, Hs, ev, b


def test_dyn_corr_direct_equals_spectral():
    m, s, hv, Hs, ev, b = sqw_setup()
    zs = ev[0] + np.linspace(0, 4, 9) + 0.05j
    d1 = O.dyn_corr_direct(Hs, b, zs)
    d2 = O.dyn_corr_spectral(Hs.toarray(), b, zs)
    assert np.allclose(d1, d2, rtol=1e-10, atol=1e-12)


def test_dyn_corr_properties():
    m, s, hv, Hs, ev, b = sqw_setup(10, math.pi / 5 * 2)
    zs = ev[0] + np.linspace(0, 4, 7) + 0.05j
    d = O.dyn_corr_direct(Hs, b, zs)
    assert np.all(-d.imag > 0)
    dc = O.dyn_corr_direct(Hs, b, np.conj(zs))
    assert np.allclose(dc, np.conj(d), rtol=1e-12)
    zbig = np.array([1e6 + 1j])
    assert abs(O.dyn_corr_direct(Hs, b, zbig)[0] * zbig[0] / np.vdot(b, b) - 1) < 1e-4


def test_szq_q0_vanishes_in_sz0():
    m, s, hv, Hs, ev, b = sqw_setup(10, 0.0)
    assert np.linalg.norm(b) < 1e-12


def test_szq_parseval():
    n = 12
    m = W.random_heisenberg(n, "chain", 4)
    s, hv = spin_setup(m)
    r = O.lanczos(hv, O.splitmix_uniform(1, 0, len(s)), 150)
    psi = O.lanczos_ground_vector(hv, O.splitmix_uniform(1, 0, len(s)), r["alpha"], r["beta"])
    tot = sum(np.vdot(bq, bq).real for bq in
              (O.szq_excitation(m, s, 2 * math.pi * k / n, psi) for k in range(n)))
    assert abs(tot - n * n / 4) < 1e-9


def test_hubbard_szq_q0_is_total_sz():
    # sum_l S^z_l = (N_up - N_dn) / 2 on every configuration
    m = W.hubbard_chain(7)
    ups, dns = O.hubbard_basis(7, 4, 2)
    psi = W.random_vector(len(ups) * len(dns), 3)
    b = O.hubbard_szq_excitation(m, ups, dns, 0.0, psi)
    assert np.max(np.abs(b - 1.0 * psi)) < 1e-14


def test_hubbard_szq_singly_occupied_equals_spin():
    # with every site singly occupied (down = complement of up) the Hubbard
    # S^z_l acts as the spin-1/2 one on the up bitstring
    n, nu = 8, 3
    hm = W.hubbard_chain(n)
    sm = W.random_heisenberg(n, "chain", 2)
    ups, dns = O.hubbard_basis(n, nu, n - nu)
    mask = (1 << n) - 1
    pos = {int(y): i for i, y in enumerate(dns)}
    psi_s = W.random_vector(len(ups), 8)
    psi = np.zeros(len(ups) * len(dns))
    rows = np.array([r * len(dns) + pos[~int(x) & mask] for r, x in enumerate(ups)])
    psi[rows] = psi_s
    q = 2 * math.pi * 3 / n
    bh = O.hubbard_szq_excitation(hm, ups, dns, q, psi)
    bs = O.szq_excitation(sm, ups, q, psi_s)
    assert np.max(np.abs(bh[rows] - bs)) < 1e-14
    other = np.setdiff1d(np.arange(len(psi)), rows)
    assert np.all(bh[other] == 0)


def test_hubbard_szq_parseval_counts_single_occupancy():
    # sum over the n momenta 2 pi k / n of |b_q|^2 = n sum_r |psi_r|^2 s_r / 4
    # with s_r the number of singly occupied sites of configuration r
    n = 6
    m = W.hubbard_chain(n)
    ups, dns = O.hubbard_basis(n, 3, 2)
    psi = W.random_vector(len(ups) * len(dns), 5)
    tot = sum(np.vdot(bq, bq).real for bq in
              (O.hubbard_szq_excitation(m, ups, dns, 2 * math.pi * k / n, psi) for k in range(n)))
    single = np.array([bin(int(x) ^ int(y)).count("1") for x in ups for y in dns], dtype=np.float64)
    assert abs(tot - n * np.sum(psi ** 2 * single) / 4) < 1e-10


def test_dyn_corr_splits_into_real_and_imaginary_parts():
    # H real symmetric: D_b(z) = D_Re b(z) + D_Im b(z) for complex b, the form
    # the device solver uses when b^T b vanishes (momentum q != 0, pi)
    m = W.heisenberg_chain(10)
    s = O.basis_list(10, 5)
    Hs = O.spin_sparse(m, s)
    ev, U = np.linalg.eigh(Hs.toarray())
    b = O.szq_excitation(m, s, 2 * math.pi / 5, U[:, 0])
    assert abs(np.sum(b * b)) < 1e-10 * np.vdot(b, b).real
    zs = ev[0] + np.linspace(0, 4, 7) + 0.1j
    d = O.dyn_corr_direct(Hs, b, zs)
    d_split = O.dyn_corr_direct(Hs, b.real.astype(np.complex128), zs) + \
        O.dyn_corr_direct(Hs, b.imag.astype(np.complex128), zs)
    assert np.allclose(d, d_split, rtol=1e-12, atol=0)


def test_continued_fraction_matches_direct():
    m, s, hv, Hs, ev, b = sqw_setup()
    zs = ev[0] + np.linspace(0, 4, 5) + 0.1j
    a, bb = O.lanczos_complex(hv, b, 250)
    d_cf = O.continued_fraction(a, bb, np.vdot(b, b).real, zs)
    d_dir = O.dyn_corr_direct(Hs, b, zs)
    assert np.allclose(d_cf, d_dir, rtol=1e-8)


# ----------------------------------------------------------------- random --

def test_splitmix_published_outputs():
    vals = [int(x) for x in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if x.strip() and not x.startswith("#")]
    assert [int(x) for x in O.splitmix_u64(1234567, 0, 5)] == vals
    # counter-based: element i alone equals element i of the stream
    assert int(O.splitmix_u64(1234567, 3, 1)[0]) == vals[3]


def test_uniform_and_gaussian_statistics():
    u = O.splitmix_uniform(9, 0, 200000)
    assert u.min() >= -0.5 and u.max() < 0.5
    assert abs(u.mean()) < 0.003 and abs(u.var() - 1 / 12) < 0.002
    g = O.splitmix_complex_gaussian(9, 100000)
    assert abs(np.mean(np.abs(g) ** 2) - 2.0) < 0.03
    assert abs(np.mean(g.real)) < 0.01 and abs(np.mean(g.imag)) < 0.01


# --------------------------------------------------------- time evolution --

def _small_hubbard():
    m = W.hubbard_chain(6, 1.0, 8.0)
    ups, dns = O.hubbard_basis(6, 3, 3)
    Hs = O.hubbard_sparse(m, ups, dns).toarray()
    return m, ups, dns, Hs


def test_taylor_evolve_matches_dense_exponential():
    # exact propagator exp(-i H t) from the full spectrum; the truncated
    # series differs per step by at most (|H| dt)^(n_max+1) / (n_max+1)!
    m, ups, dns, Hd = _small_hubbard()
    ev, U = np.linalg.eigh(Hd)
    rng = np.random.default_rng(4)
    psi0 = rng.normal(size=len(Hd)) + 1j * rng.normal(size=len(Hd))
    psi0 /= np.linalg.norm(psi0)
    dt, n_steps = 0.02, 25
    for n_max, tol in [(10, 1e-9), (4, None)]:
        o = O.taylor_evolve(lambda x: Hd @ x, psi0, n_max, dt, n_steps)
        exact = U @ (np.exp(-1j * ev * dt * n_steps) * (U.conj().T @ psi0))
        err = np.linalg.norm(o["psi"][:, 0] - exact)
        hn = float(np.max(np.abs(ev)))
        bound = n_steps * (hn * dt) ** (n_max + 1) / math.factorial(n_max + 1) * np.exp(hn * dt)
        assert err <= bound + 1e-13
        if tol is not None:
            assert err < tol


def test_taylor_evolve_conserves_norm_and_energy():
    m, ups, dns, Hd = _small_hubbard()
    rng = np.random.default_rng(5)
    psi0 = rng.normal(size=len(Hd)) + 1j * rng.normal(size=len(Hd))
    o = O.taylor_evolve(lambda x: Hd @ x, psi0, 10, 0.01, 40)
    assert np.max(np.abs(o["norm"] / o["norm"][0] - 1)) < 1e-12
    assert np.max(np.abs(o["energy"] - o["energy"][0])) < 1e-12
    # a too short series visibly breaks unitarity
    o2 = O.taylor_evolve(lambda x: Hd @ x, psi0, 2, 0.05, 40)
    assert np.max(np.abs(o2["norm"] / o2["norm"][0] - 1)) > 1e-6


def test_taylor_evolve_diagonal_hamiltonian_phases():
    # t = 0 (no hopping): every configuration only picks up exp(-i E_x t)
    m = W.hubbard_chain(4, 0.0, 3.0)
    ups, dns = O.hubbard_basis(4, 2, 2)
    rng = np.random.default_rng(6)
    psi0 = rng.normal(size=len(ups) * len(dns)) + 0j
    diag = O.hubbard_hv(m, ups, dns, np.ones(len(psi0)))
    o = O.taylor_evolve(lambda x: O.hubbard_hv(m, ups, dns, x), psi0, 12, 0.01, 30)
    assert np.max(np.abs(o["psi"][:, 0] - np.exp(-1j * diag * 0.3) * psi0)) < 1e-12


def test_double_occupancy_weight_atomic_limits():
    ups, dns = O.hubbard_basis(4, 2, 2)
    w = O.hubbard_double_occupancy_weight(ups, dns, 4)
    # the all-doubly-occupied pattern exists only when up == down
    assert w.max() == 0.5 and w.min() == 0.0
    # uniform superposition: mean over states of (#doubles) / N_s
    m = W.hubbard_chain(4, 0.0, 1.0)
    tr = np.sum(O.hubbard_hv(m, ups, dns, np.ones(len(w))))
    assert abs(np.mean(w) - tr / len(w) / 4) < 1e-15


def test_lanczos_stop_rule_and_residual_estimate():
    """The stopping rule of a checked Lanczos run, and the residual estimate
    it uses: beta_m |s_{m-1}| equals |H y - theta y| for the Ritz vector
    y = Q_m s (before orthogonality is lost), checked by forming y."""
    m = W.random_heisenberg(12, "chain", 4)
    s = O.basis_list(12, 6)
    Hs = O.spin_sparse(m, s)
    hv = lambda x: Hs @ x
    v0 = O.splitmix_uniform(3, 0, len(s))
    lz = O.lanczos(hv, v0, 200)
    assert len(lz["beta_full"]) == len(lz["alpha"]) + 1
    for mm in (8, 15, 25):
        a, bf = lz["alpha"][:mm], lz["beta_full"]
        th, sv = scipy.linalg.eigh_tridiagonal(a, bf[1:mm], select="i", select_range=(0, 0))
        y = O.lanczos_ground_vector(hv, v0, a, lz["beta"][:mm])
        ry = np.linalg.norm(hv(y) - th[0] * y)
        est = bf[mm] * abs(sv[mm - 1, 0])
        assert abs(ry - est) <= 1e-9 * max(1.0, est) + 1e-12
    # brute force over the checks
    def brute(tol, rtol):
        last = None
        for k in range(10, len(lz["alpha"]) + 1, 10):
            a, bf = lz["alpha"][:k], lz["beta_full"]
            th, sv = scipy.linalg.eigh_tridiagonal(a, bf[1:k], select="i", select_range=(0, 0))
            ok = last is not None and abs(th[0] - last) < tol * max(1, abs(th[0]))
            if ok and rtol > 0:
                ok = bf[k] * abs(sv[k - 1, 0]) < rtol * max(1, abs(th[0]))
            if ok:
                return k
            last = th[0]
        return len(lz["alpha"])
    for tol, rtol in ((1e-12, 0.0), (1e-12, 1e-9), (1e-6, 0.0), (1e-6, 1e-4)):
        assert O.lanczos_stop(lz["alpha"], lz["beta_full"], 10, tol, rtol) == brute(tol, rtol)
    # the residual rule can only stop later
    assert O.lanczos_stop(lz["alpha"], lz["beta_full"], 10, 1e-12, 1e-10) >= \
        O.lanczos_stop(lz["alpha"], lz["beta_full"], 10, 1e-12, 0.0)
