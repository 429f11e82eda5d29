"""GPU: the Hubbard Hamiltonian with the two-body terms of Eq. ham_general
(Sec. 5: inter-site Coulomb, Hund, exchange, pair hopping) against the
oracle.

  * H*v element by element (FP64, complex, FP32) on random pair lists that
    include long-range pairs (fermion signs over the sites between), on the
    Wannier-form nearest-neighbour model (one V and one J per bond), on
    several sectors, under the built-in schedule and the other T_up / T_dn
    kernel variants;
  * the 4x4 half-filled Wannier-form model (the size of the bench workload)
    on sampled up rows, in the padded launch that Lanczos runs;
  * Lanczos alpha/beta against the oracle's recurrence, E0 against the
    oracle's sparse eigensolver, the FP32-storage refined energy within
    1e-8, LOBPCG (diagonal preconditioner with the two-body diagonal) and the
    trace against the oracle's matrix, and one cTPQ run.

Tolerances: FP64 H*v 1e-12 of max|Hv| (different summation order of at
most ~100 terms); FP32 H*v 3e-6 of max|Hv| against the oracle on the FP32
input; Lanczos alpha/beta 1e-11 for 20 steps; energies 1e-10.
"""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import core as O
from paper_2307_13222_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    from paper_2307_13222_amd import api as A
    return A


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def random_pairs_model(n, lattice_model, seed, frac=0.4):
    """Random couplings on a random subset of all site pairs (both orders
    allowed), on top of a lattice hopping model."""
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n) for j in range(n) if i != j and rng.random() < frac / 2]
    k = len(pairs)
    return W.with_pair_terms(lattice_model, pairs, rng.normal(size=k), rng.normal(size=k),
                             rng.normal(size=k), rng.normal(size=k))


CASES = [
    ("ext 3x4 half", lambda: W.extended_hubbard_square(3, 4, 1.0, 4.0, 1.0, 0.3), 12, 6, 6),
    ("random pairs 10 chain", lambda: random_pairs_model(10, W.hubbard_chain(10, 1.0, 3.0), 5), 10, 5, 4),
    ("random pairs 2x4", lambda: random_pairs_model(8, W.hubbard_square(2, 4, 1.0, 2.0), 6, 0.8), 8, 3, 5),
    ("ext 3x3 empty down", lambda: W.extended_hubbard_square(3, 3, 1.0, 4.0, 0.5, 0.2), 9, 4, 0),
]


@pytest.mark.parametrize("name,make,n,nu,nd", CASES, ids=[c[0] for c in CASES])
def test_extended_mult_vs_oracle(api, ctx, name, make, n, nu, nd):
    import torch
    say("extended mult", name)
    m = make()
    b = api.Basis.hubbard(ctx, n, nu, nd)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(n, nu, nd)
    v = W.random_vector(b.dim, 41)
    ref = O.hubbard_hv(m, ups, dns, v)
    w = host(h.mult(dev(v)))
    assert relmax(w, ref) < 1e-12
    vc = W.random_vector(b.dim, 42, np.complex128)
    assert relmax(host(h.mult(dev(vc))), O.hubbard_hv(m, ups, dns, vc)) < 1e-12
    vf = dev(v).to(torch.float32)
    wf = host(h.mult(vf)).astype(np.float64)
    assert relmax(wf, O.hubbard_hv(m, ups, dns, host(vf).astype(np.float64))) < 3e-6
    # the pair terms alone are what the two-body model adds
    m0 = W.HubbardModel(m.n_sites, m.hi, m.hj, m.t, m.u_site)
    w0 = host(api.Hamiltonian.hubbard(b, m0).mult(dev(v)))
    assert relmax(w - w0, O.hubbard_pairs_hv(m, ups, dns, v)) < 1e-11


SCHEDULES = [dict(hub_sweep=5), dict(hub_sweep=1, hub_row_cols=2), dict(hub_sweep=3, hub_row_cols=1),
             dict(hub_sweep=5, hub_row_cols=4), dict(hub_sweep=5, hub_slab_cols=32, hub_row_cols=3)]


@pytest.mark.parametrize("sched", SCHEDULES, ids=[str(s) for s in SCHEDULES])
def test_extended_mult_schedules(api, ctx, sched):
    say("extended schedules", sched)
    m = W.extended_hubbard_square(3, 4, 1.0, 4.0, 1.0, 0.3)
    b = api.Basis.hubbard(ctx, 12, 6, 5)
    h = api.Hamiltonian.hubbard(b, m)
    h.set_schedule(**sched)
    ups, dns = O.hubbard_basis(12, 6, 5)
    v = W.random_vector(b.dim, 43)
    assert relmax(host(h.mult(dev(v))), O.hubbard_hv(m, ups, dns, v)) < 1e-12
    vc = W.random_vector(b.dim, 44, np.complex128)
    assert relmax(host(h.mult(dev(vc))), O.hubbard_hv(m, ups, dns, vc)) < 1e-12


def test_extended_4x4_sampled_rows(api, ctx):
    say("extended 4x4 sampled rows")
    m = W.extended_hubbard_square(4, 4, 1.0, 4.0, 1.0, 0.3)
    b = api.Basis.hubbard(ctx, 16, 8, 8)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(16, 8, 8)
    v = O.splitmix_uniform(3, 0, b.dim)
    w = host(h.mult(dev(v))).reshape(len(ups), len(dns))
    for r0 in (0, 4321, len(ups) - 3):
        ref = O.hubbard_hv_rows(m, ups, dns, v, r0, 3).reshape(3, len(dns))
        assert relmax(w[r0:r0 + 3], ref) < 1e-12, r0
    # Lanczos runs the padded fused launch (rows kernel with the update,
    # pair kernel, tile kernel). The oracle's whole product at this size
    # takes minutes, so its link is the sampled rows above; here the first
    # coefficient alpha_0 = <v0, H v0> / <v0, v0> of the padded launch is
    # checked against the plain launch's product
    r = api.lanczos(h, 3, seed=3)
    a0 = float(np.dot(v, w.ravel()) / np.dot(v, v))
    assert abs(r["alpha"][0] - a0) < 1e-11 * max(1.0, abs(a0))


def test_extended_3x4_padded_lanczos_vs_oracle(api, ctx):
    say("extended 3x4 padded lanczos")
    m = W.extended_hubbard_square(3, 4, 1.0, 4.0, 1.0, 0.3)
    b = api.Basis.hubbard(ctx, 12, 6, 6)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(12, 6, 6)
    ro = O.lanczos(lambda x: O.hubbard_hv(m, ups, dns, x), O.splitmix_uniform(2, 0, b.dim), 10)
    r = api.lanczos(h, 10, seed=2)
    assert np.allclose(r["alpha"], ro["alpha"], rtol=0, atol=1e-11)
    assert np.allclose(r["beta"][1:], ro["beta"][1:], rtol=0, atol=1e-11)


def test_extended_lanczos_vs_oracle(api, ctx):
    say("extended lanczos")
    m = random_pairs_model(10, W.hubbard_chain(10, 1.0, 4.0), 8)
    b = api.Basis.hubbard(ctx, 10, 5, 5)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(10, 5, 5)
    hv = lambda x: O.hubbard_hv(m, ups, dns, x)
    v0 = O.splitmix_uniform(1, 0, b.dim)
    ro = O.lanczos(hv, v0, 20)
    r = api.lanczos(h, 300, seed=1)
    assert np.allclose(r["alpha"][:20], ro["alpha"], rtol=0, atol=1e-11)
    assert np.allclose(r["beta"][1:20], ro["beta"][1:], rtol=0, atol=1e-11)
    e0 = sla.eigsh(O.hubbard_sparse(m, ups, dns), k=1, which="SA", v0=v0, tol=1e-14)[0][0]
    assert abs(r["energies"][0] - e0) < 1e-10
    r32 = api.lanczos(h, 300, seed=1, storage="f32", refine=True)
    say(f"  E0 {e0:.14f} fp32 refined {r32['energies'][0]:.14f}")
    assert abs(r32["energies"][0] - e0) <= 1e-8


def test_extended_lobpcg_trace_ctpq(api, ctx):
    say("extended lobpcg / trace / ctpq")
    m = W.extended_hubbard_square(2, 4, 1.0, 4.0, 0.8, 0.4)
    b = api.Basis.hubbard(ctx, 8, 3, 3)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(8, 3, 3)
    Hs = O.hubbard_sparse(m, ups, dns)
    ev = np.linalg.eigvalsh(Hs.toarray())
    assert abs(h.trace() - Hs.diagonal().sum()) < 1e-9 * max(1.0, abs(Hs.diagonal().sum()))
    r = api.lobpcg(h, 3, max_iter=500, tol=1e-9)
    assert r["converged"]
    assert np.allclose(r["energies"], ev[:3], atol=1e-8)
    phi0 = O.splitmix_complex_gaussian(5, b.dim)[:, None]
    g = api.ctpq(h, 1, 6, 0.02, 10, phi0=dev(phi0))
    o = O.ctpq(lambda x: O.hubbard_hv(m, ups, dns, x), phi0, 6, 0.02, 10)
    assert relmax(g["D"], o["D"]) < 1e-11
    assert relmax(g["E"], o["E"]) < 1e-11


def test_extended_invalid(api, ctx):
    m = W.hubbard_chain(6, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 6, 3, 3)
    for bad in ([(0, 0)], [(0, 6)], [(-1, 2)]):
        with pytest.raises(api.HphiError):
            api.Hamiltonian.hubbard(b, W.with_pair_terms(m, bad, 1.0, 0.0, 0.0, 0.0))
