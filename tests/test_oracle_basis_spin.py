"""Pins of the oracle's basis, ranking and spin H*v against things other than
itself: binomial counts, two independent rank routes, an independent
Pauli-matrix construction of H on the full 2^N space, closed-form energies
(two sites, 4-site ring, Ising limit, XX ring via Jordan-Wigner free
fermions), the closed-form trace, Bethe-ansatz energy of the 16-site ring,
hermiticity, SU(2) commutation and S^+ intertwining."""
import math

import numpy as np
import pytest
import scipy.optimize
import scipy.sparse as sp

from oracle import core as O
from paper_2307_13222_amd import workloads as W


# ------------------------------------------------------------------ basis --

@pytest.mark.parametrize("n", range(1, 17))
def test_basis_counts_and_ranks_exhaustive(n):
    for k in range(0, n + 1):
        s = O.basis_list(n, k)
        assert s.shape[0] == math.comb(n, k)
        assert np.all(np.diff(s.astype(np.int64)) > 0) if len(s) > 1 else True
        assert all(bin(int(x)).count("1") == k for x in s[:50])
        idx = np.arange(len(s))
        assert np.array_equal(O.rank_combinadic(s), idx)
        assert np.array_equal(O.rank_search(s, s), idx)


def test_rank_absent_state():
    s = O.basis_list(10, 5)
    assert O.rank_search(s, np.array([0b11], dtype=np.uint64))[0] == -1


def test_unrank_roundtrip_large():
    # N = 36, n = 18 (dim 9,075,135,300): sampled ranks, incl. both ends
    n, k = 36, 18
    dim = math.comb(n, k)
    rng = np.random.default_rng(3)
    rows = np.concatenate([[0, 1, dim - 2, dim - 1], rng.integers(0, dim, 200)])
    for r in rows:
        x = O.unrank_combinadic(int(r), k)
        assert bin(x).count("1") == k and x < (1 << n)
        assert O.rank_combinadic(np.array([x], dtype=np.uint64))[0] == r
    assert O.unrank_combinadic(0, k) == (1 << k) - 1
    assert O.unrank_combinadic(dim - 1, k) == ((1 << k) - 1) << (n - k)


# ---------------------------------------------- independent dense spin H --

def pauli_dense_spin(m) -> np.ndarray:
    """H on the full 2^N space from Kronecker products of single-site spin
    matrices (site i = bit i, bit 1 = up); an independent construction."""
    n = m.n_sites
    sz = sp.csr_matrix(np.diag([-0.5, 0.5]))
    splus = sp.csr_matrix(np.array([[0.0, 0.0], [1.0, 0.0]]))   # |0> -> |1>
    sminus = splus.T.tocsr()

    def site(op, i):
        mats = [sp.identity(2, format="csr")] * n
        mats[n - 1 - i] = op
        out = mats[0]
        for mm in mats[1:]:
            out = sp.kron(out, mm, format="csr")
        return out

    dim = 1 << n
    H = sp.csr_matrix((dim, dim))
    for b in range(m.n_bonds):
        i, j = int(m.bi[b]), int(m.bj[b])
        H = H + m.jz[b] * site(sz, i) @ site(sz, j)
        H = H + 0.5 * m.jxy[b] * (site(splus, i) @ site(sminus, j) + site(sminus, i) @ site(splus, j))
    if m.hz is not None:
        for i in range(n):
            H = H - m.hz[i] * site(sz, i)
    return H.toarray()


def oracle_dense_spin(m, states):
    return O.spin_sparse(m, states).toarray()


@pytest.mark.parametrize("n,seed", [(4, 0), (6, 1), (7, 2), (8, 3)])
def test_spin_h_matches_pauli_construction(n, seed):
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.6]
    m = W._spin(n, pairs, rng.normal(size=(len(pairs), 2)), "rand", hz=rng.normal(size=n))
    Hfull = pauli_dense_spin(m)
    for k in range(n + 1):
        s = O.basis_list(n, k)
        Hs = oracle_dense_spin(m, s)
        ref = Hfull[np.ix_(s.astype(np.int64), s.astype(np.int64))]
        assert np.allclose(Hs, ref, atol=1e-13, rtol=0)
        # H*v through the row-wise product equals the matrix product
        v = W.random_vector(len(s), seed + k)
        assert np.allclose(O.spin_hv(m, s, v), ref @ v, atol=1e-12)
    # the sectors exhaust the full space: the blocks carry all of H
    off = 0.0
    for k in range(n + 1):
        s = O.basis_list(n, k).astype(np.int64)
        rest = np.setdiff1d(np.arange(1 << n), s)
        off += np.abs(Hfull[np.ix_(s, rest)]).sum()
    assert off == 0.0


def e0(m, two_sz=0):
    s = O.basis_list(m.n_sites, O.sector_popcount_spin(m.n_sites, two_sz))
    return np.linalg.eigvalsh(oracle_dense_spin(m, s))[0]


def test_two_site_singlet():
    m = W._spin(2, [(0, 1)], [(1.0, 1.0)], "pair")
    assert abs(e0(m) + 0.75) < 1e-14


def test_four_site_ring():
    assert abs(e0(W.heisenberg_chain(4)) + 2.0) < 1e-13


@pytest.mark.parametrize("n", [4, 6, 8, 10])
def test_ising_limit(n):
    m = W._spin(n, W.chain_pairs(n), [(1.3, 0.0)] * n, "ising")
    assert abs(e0(m) + n * 1.3 / 4) < 1e-12


@pytest.mark.parametrize("n", [6, 8, 10, 12])
def test_xx_ring_free_fermions(n):
    m = W._spin(n, W.chain_pairs(n), [(0.0, 1.0)] * n, "xx")
    assert abs(e0(m) + 1.0 / math.sin(math.pi / n)) < 1e-12


def test_xx_ring_16_lanczos():
    m = W._spin(16, W.chain_pairs(16), [(0.0, 1.0)] * 16, "xx")
    s = O.basis_list(16, 8)
    r = O.lanczos(lambda v: O.spin_hv(m, s, v), W.random_vector(len(s), 1), 200)
    assert abs(O.tridiag_lowest(r["alpha"], r["beta"])[0] + 1 / math.sin(math.pi / 16)) < 1e-10
    assert abs(-1 / math.sin(math.pi / 16) - (-5.1258308955)) < 1e-9


@pytest.mark.parametrize("n,k", [(8, 4), (10, 3), (12, 6), (16, 8)])
def test_trace_closed_form(n, k):
    rng = np.random.default_rng(n)
    m = W._spin(n, W.chain_pairs(n) + W.chain_pairs(n, 2), rng.normal(size=(2 * n, 2)), "t")
    s = O.basis_list(n, k)
    tr = O.spin_sparse(m, s).diagonal().sum()
    c = math.comb
    ref = m.jz.sum() * 0.25 * (c(n - 2, k - 2) + c(n - 2, k) - 2 * c(n - 2, k - 1))
    assert abs(tr - ref) < 1e-9 * max(1, abs(ref))
    if (n, k) == (16, 8):
        m1 = W.heisenberg_chain(16)
        assert abs(O.spin_sparse(m1, s).diagonal().sum() + 3432.0) < 1e-9


def bethe_xxx_ring(n: int) -> float:
    """Ground energy of the periodic spin-1/2 Heisenberg ring (J = 1, n even)
    from the logarithmic Bethe equations
        n arctan(2 l_j) = pi I_j + sum_{k != j} arctan(l_j - l_k),
        I_j = -(M-1)/2 ... (M-1)/2, M = n/2,
    E = n/4 - sum_j (1/2) / (l_j^2 + 1/4)."""
    M = n // 2
    I = np.arange(M) - (M - 1) / 2.0

    def f(l):
        d = l[:, None] - l[None, :]
        return n * np.arctan(2 * l) - np.pi * I - np.arctan(d).sum(axis=1)

    l0 = 0.5 * np.tan(np.pi * I / n)
    l = scipy.optimize.fsolve(f, l0, xtol=1e-13)
    assert np.max(np.abs(f(l))) < 1e-11
    return n / 4.0 - np.sum(0.5 / (l ** 2 + 0.25))


def test_bethe_solver_small_rings():
    for n in (4, 6, 8, 10):
        assert abs(bethe_xxx_ring(n) - e0(W.heisenberg_chain(n))) < 1e-10


def test_heisenberg16_ground_energy_bethe():
    ref = bethe_xxx_ring(16)
    assert abs(ref - (-7.142296360616785)) < 1e-10
    m = W.heisenberg_chain(16)
    s = O.basis_list(16, 8)
    r = O.lanczos(lambda v: O.spin_hv(m, s, v), O.splitmix_uniform(1, 0, len(s)), 200)
    assert abs(O.tridiag_lowest(r["alpha"], r["beta"])[0] - ref) < 1e-10


# ------------------------------------------------------------- invariants --

def test_hermiticity_random():
    m = W.xxz_chain_j2(14)
    s = O.basis_list(14, 7)
    u, v = W.random_vector(len(s), 1), W.random_vector(len(s), 2)
    lhs, rhs = u @ O.spin_hv(m, s, v), O.spin_hv(m, s, u) @ v
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-12


def s2_model(n):
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    return W._spin(n, pairs, [(2.0, 2.0)] * len(pairs), "s2")


@pytest.mark.parametrize("n", [8, 10])
def test_su2_commutation(n):
    # S^2 = 2 sum_{i<j} S_i.S_j + 3n/4; H (Heisenberg) must commute with it
    m = W.random_heisenberg(n, "chain", 5)
    s = O.basis_list(n, n // 2)
    S2 = s2_model(n)
    v = W.random_vector(len(s), 9)
    a = O.spin_hv(m, s, O.spin_hv(S2, s, v))
    b = O.spin_hv(S2, s, O.spin_hv(m, s, v))
    assert np.max(np.abs(a - b)) < 1e-11
    # the XXZ model (Jz != Jxy) does not commute: the check can fail
    mx = W.xxz_chain_j2(n)
    a = O.spin_hv(mx, s, O.spin_hv(S2, s, v))
    b = O.spin_hv(S2, s, O.spin_hv(mx, s, v))
    assert np.max(np.abs(a - b)) > 1e-3


def test_ground_state_singlet_4x4():
    # bipartite Heisenberg ground state is a singlet (S(S+1) = 0)
    m = W._spin(16, W.square_pairs(4, 4), [(1.0, 1.0)] * 32, "sq")
    s = O.basis_list(16, 8)
    hv = lambda v: O.spin_hv(m, s, v)
    r = O.lanczos(hv, W.random_vector(len(s), 4), 150)
    psi = O.lanczos_ground_vector(hv, W.random_vector(len(s), 4), r["alpha"], r["beta"])
    S2 = s2_model(16)
    # S^2 = 3n/4 + 2 sum_{i<j} S_i.S_j; the all-pairs bonds carry the 2
    s2 = psi @ O.spin_hv(S2, s, psi) + 3 * 16 / 4
    assert abs(s2) < 1e-6


def test_splus_intertwines_sectors():
    n = 10
    m = W.random_heisenberg(n, "ladder", 11)
    s4, s5 = O.basis_list(n, 4), O.basis_list(n, 5)
    # S^+_tot maps the 4-up sector to the 5-up sector
    rows, cols = [], []
    for c, x in enumerate(s4):
        for i in range(n):
            if not (int(x) >> i) & 1:
                rows.append(O.rank_search(s5, np.array([int(x) | (1 << i)], dtype=np.uint64))[0])
                cols.append(c)
    Sp = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(len(s5), len(s4)))
    v = W.random_vector(len(s4), 3)
    assert np.max(np.abs(O.spin_hv(m, s5, Sp @ v) - Sp @ O.spin_hv(m, s4, v))) < 1e-12


def test_spin_flip_symmetric_spectrum():
    m = W.xxz_chain_j2(10)
    a = np.linalg.eigvalsh(oracle_dense_spin(m, O.basis_list(10, 3)))
    b = np.linalg.eigvalsh(oracle_dense_spin(m, O.basis_list(10, 7)))
    assert np.allclose(a, b, atol=1e-11)


def test_row_by_index_matches_list_rows():
    m = W.j1j2_square(4, 4)
    s = O.basis_list(16, 8)
    Hs = O.spin_sparse(m, s)
    for r in [0, 1, 77, 5000, len(s) - 1]:
        cols, vals = O.spin_row(m, 8, r)
        dense = np.zeros(len(s))
        np.add.at(dense, cols, vals)
        assert np.allclose(dense, Hs.getrow(r).toarray()[0], atol=1e-15)
