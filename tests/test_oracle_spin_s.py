"""Pins of the oracle's spin-S H*v (keyword 2S, Sec. 4.1, "Remarks on the
keyword model"): spin matrices checked against the angular-momentum
algebra, then a Kronecker-product construction restricted to each S^z
sector; the two-spin multiplet energies; S = 1/2 against the spin-1/2
sector oracle; spin-rotation invariance of the isotropic model (levels of
S^z = 1 reappear at S^z = 0)."""
import numpy as np
import pytest

from oracle import core as O
from paper_2307_13222_amd import workloads as W


def spin_matrices(two_s):
    """S^z, S^+, S^- in the basis m = 0 .. 2S (S^z = m - S)."""
    S = two_s / 2
    d = two_s + 1
    sz = np.diag(np.arange(d) - S)
    sp = np.zeros((d, d))
    for m in range(d - 1):
        s = m - S
        sp[m + 1, m] = np.sqrt(S * (S + 1) - s * (s + 1))
    return sz, sp, sp.T.copy()


@pytest.mark.parametrize("two_s", [1, 2, 3, 4])
def test_spin_matrices_obey_the_algebra(two_s):
    sz, sp, sm = spin_matrices(two_s)
    sx, sy = (sp + sm) / 2, (sp - sm) / 2j
    S = two_s / 2
    assert np.allclose(sx @ sy - sy @ sx, 1j * sz)
    assert np.allclose(sx @ sx + sy @ sy + sz @ sz, S * (S + 1) * np.eye(two_s + 1))


def kron_dense(m):
    """Full (2S+1)^N matrix, site 0 the fastest digit."""
    sz, sp, sm = spin_matrices(m.two_s)
    d = m.two_s + 1
    n = m.n_sites

    def site(op, i):
        out = np.array([[1.0]])
        for k in range(n - 1, -1, -1):
            out = np.kron(out, op if k == i else np.eye(d))
        return out
    H = np.zeros((d ** n, d ** n))
    for b in range(m.n_bonds):
        i, j = int(m.bi[b]), int(m.bj[b])
        H += m.jz[b] * site(sz, i) @ site(sz, j)
        H += 0.5 * m.jxy[b] * (site(sp, i) @ site(sm, j) + site(sm, i) @ site(sp, j))
    for i in range(n):
        if m.hz is not None:
            H -= m.hz[i] * site(sz, i)
        if m.d_ion is not None:
            H += m.d_ion[i] * site(sz @ sz, i)
    return H


def digits_index(states, n, two_s):
    """Row of each encoded configuration in the Kronecker basis."""
    b = 1
    while (1 << b) <= two_s:
        b += 1
    out = []
    for x in states:
        x = int(x)
        idx = 0
        for i in range(n - 1, -1, -1):
            idx = idx * (two_s + 1) + ((x >> (i * b)) & ((1 << b) - 1))
        out.append(idx)
    return np.array(out)


@pytest.mark.parametrize("n,two_s,lat,seed", [(4, 2, "chain", 1), (5, 2, "chain", 2), (4, 3, "ladder", 3),
                                             (3, 4, "chain", 4)])
def test_spin_s_matches_kronecker_products(n, two_s, lat, seed):
    m = W.random_spin_s(n, two_s, lat, seed)
    H = kron_dense(m)
    for two_sz in range(-n * two_s, n * two_s + 1, 2):
        s = O.spin_s_basis(n, two_s, two_sz)
        idx = digits_index(s, n, two_s)
        ref = H[np.ix_(idx, idx)]
        # the sector is closed under H
        outside = np.setdiff1d(np.arange(H.shape[0]), idx)
        assert np.max(np.abs(H[np.ix_(outside, idx)]), initial=0.0) < 1e-14
        Hs = O.spin_s_sparse(m, s).toarray()
        assert np.allclose(Hs, ref, atol=1e-13), two_sz
        v = W.random_vector(len(s), seed + two_sz + 100)
        assert np.allclose(O.spin_s_hv(m, s, v), ref @ v, atol=1e-13)


@pytest.mark.parametrize("two_s", [1, 2, 3, 4])
def test_two_spin_multiplets(two_s):
    # J S_1.S_2 = J/2 [T(T+1) - 2 S(S+1)], T = 0 .. 2S, each once at S^z = 0
    S = two_s / 2
    m = W.spin_s_model(2, two_s, [(0, 1)], 1.0, 1.0)
    ev = np.sort(np.linalg.eigvalsh(O.spin_s_sparse(m, O.spin_s_basis(2, two_s, 0)).toarray()))
    ref = np.sort([0.5 * (T * (T + 1) - 2 * S * (S + 1)) for T in range(0, two_s + 1)])
    assert np.allclose(ev, ref, atol=1e-13)


def test_spin_half_is_the_spin_half_oracle():
    sm = W.random_heisenberg(10, "ladder", 8)
    sm.hz = np.random.default_rng(8).normal(size=10)
    m = W.spin_s_model(10, 1, np.stack([sm.bi, sm.bj], 1), sm.jz, sm.jxy, sm.hz)
    for two_sz in (0, 2, -4):
        s = O.spin_s_basis(10, 1, two_sz)
        s2 = O.basis_list(10, (10 + two_sz) // 2)
        assert np.array_equal(s, s2)
        assert abs(O.spin_s_sparse(m, s) - O.spin_sparse(sm, s2)).max() < 1e-14


@pytest.mark.parametrize("n,two_s", [(6, 2), (5, 3)])
def test_isotropic_levels_nest(n, two_s):
    rng = np.random.default_rng(n)
    pairs = W.chain_pairs(n)
    j = rng.uniform(0.5, 1.5, len(pairs))
    m = W.spin_s_model(n, two_s, pairs, j, j)
    base = (n * two_s) % 2
    lo = np.linalg.eigvalsh(O.spin_s_sparse(m, O.spin_s_basis(n, two_s, base)).toarray())
    hi = np.linalg.eigvalsh(O.spin_s_sparse(m, O.spin_s_basis(n, two_s, base + 2)).toarray())
    assert max(np.min(np.abs(lo - e)) for e in hi) < 1e-10
    # anisotropy breaks it
    m2 = W.spin_s_model(n, two_s, pairs, j, 0.7 * j)
    lo = np.linalg.eigvalsh(O.spin_s_sparse(m2, O.spin_s_basis(n, two_s, base)).toarray())
    hi = np.linalg.eigvalsh(O.spin_s_sparse(m2, O.spin_s_basis(n, two_s, base + 2)).toarray())
    assert max(np.min(np.abs(lo - e)) for e in hi) > 1e-3


def test_row_matches_sparse():
    m = W.random_spin_s(6, 2, "chain", 12)
    s = O.spin_s_basis(6, 2, 0)
    Hs = O.spin_s_sparse(m, s)
    for r in (0, 17, len(s) - 1):
        cols, vals = O.spin_s_row(m, s, r)
        dense = np.zeros(len(s))
        np.add.at(dense, cols, vals)
        assert np.allclose(dense, Hs.getrow(r).toarray()[0], atol=1e-15)
