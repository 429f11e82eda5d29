"""GPU: the spin-S Heisenberg model with total S^z conserved (keyword 2S,
Sec. 4.1) against the oracle: H*v element by element (FP64, complex, FP32)
for S = 1, 3/2, 2 with fields and single-ion terms, Lanczos coefficients and
E0, the S = 1 ring's levels against the oracle's spectrum, LOBPCG, trace,
cTPQ, S^z(q) and the host/device state and rank maps. Tolerances as for the
spin-1/2 kernels: FP64 1e-12 of max|Hv|, FP32 3e-6, alpha/beta 1e-11,
energies 1e-10."""
import math
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


@pytest.mark.parametrize("n,two_s,two_sz,lat,seed", [(10, 2, 0, "chain", 1), (8, 3, 2, "ladder", 2),
                                                     (7, 4, -2, "chain", 3), (14, 2, 2, "ladder", 4)])
def test_spin_s_mult_vs_oracle(api, ctx, n, two_s, two_sz, lat, seed):
    import torch
    say("spin-S mult", n, two_s, two_sz)
    m = W.random_spin_s(n, two_s, lat, seed)
    b = api.Basis.spin_s(ctx, n, two_s, two_sz)
    s = O.spin_s_basis(n, two_s, two_sz)
    assert b.dim == len(s)
    assert np.array_equal(b.states(0, len(s)), s)
    h = api.Hamiltonian.spin_s(b, m)
    v = W.random_vector(len(s), seed)
    assert relmax(host(h.mult(dev(v))), O.spin_s_hv(m, s, v)) < 1e-12
    vc = W.random_vector(len(s), seed + 5, np.complex128)
    assert relmax(host(h.mult(dev(vc))), O.spin_s_hv(m, s, vc)) < 1e-12
    vf = dev(v).to(torch.float32)
    assert relmax(host(h.mult(vf)).astype(np.float64), O.spin_s_hv(m, s, host(vf).astype(np.float64))) < 3e-6


def test_spin_s_lanczos_vs_oracle(api, ctx):
    say("spin-S lanczos")
    m = W.random_spin_s(12, 2, "chain", 6)
    b = api.Basis.spin_s(ctx, 12, 2, 0)
    h = api.Hamiltonian.spin_s(b, m)
    s = O.spin_s_basis(12, 2, 0)
    v0 = O.splitmix_uniform(1, 0, len(s))
    ro = O.lanczos(lambda x: O.spin_s_hv(m, s, x), v0, 20)
    r = api.lanczos(h, 400, seed=1)
    assert np.allclose(r["alpha"][:20], ro["alpha"], rtol=0, atol=1e-11)
    assert np.allclose(r["beta"][1:20], ro["beta"][1:], rtol=0, atol=1e-11)
    e0 = sla.eigsh(O.spin_s_sparse(m, s), k=1, which="SA", v0=v0, tol=1e-14)[0][0]
    assert abs(r["energies"][0] - e0) < 1e-10


def test_spin1_ring_levels(api, ctx):
    # isotropic S = 1 ring of 8: the lowest levels of S^z = 0 and 1 from
    # LOBPCG against the oracle's dense spectra (the S^z = 1 levels reappear
    # at S^z = 0)
    say("spin-1 ring")
    m = W.spin_s_model(8, 2, W.chain_pairs(8), 1.0, 1.0)
    for two_sz in (0, 2):
        b = api.Basis.spin_s(ctx, 8, 2, two_sz)
        h = api.Hamiltonian.spin_s(b, m)
        ev = np.linalg.eigvalsh(O.spin_s_sparse(m, O.spin_s_basis(8, 2, two_sz)).toarray())
        r = api.lobpcg(h, 6, max_iter=1500, tol=1e-8)
        assert r["converged"], r
        assert np.allclose(r["energies"][:4], ev[:4], atol=1e-9)
        assert abs(h.trace() - np.sum(ev)) < 1e-9 * max(1.0, float(np.sum(np.abs(ev))))


def test_spin_s_ctpq_szq_rank(api, ctx):
    say("spin-S ctpq / szq / rank")
    m = W.random_spin_s(8, 2, "chain", 9)
    b = api.Basis.spin_s(ctx, 8, 2, 0)
    h = api.Hamiltonian.spin_s(b, m)
    s = O.spin_s_basis(8, 2, 0)
    phi0 = O.splitmix_complex_gaussian(4, len(s))[:, None]
    g = api.ctpq(h, 1, 6, 0.02, 10, phi0=dev(phi0))
    o = O.ctpq(lambda x: O.spin_s_hv(m, s, x), phi0, 6, 0.02, 10)
    assert relmax(g["D"], o["D"]) < 1e-11 and relmax(g["E"], o["E"]) < 1e-11
    psi = W.random_vector(len(s), 3)
    bq = host(api.szq(h, math.pi, dev(psi)))
    # S^z(q) on spin-S: S^z_l = m_l - S read from each site's 2-bit field
    sz = np.array([[((int(x) >> (2 * l)) & 3) - 1.0 for l in range(8)] for x in s])
    ref = (sz @ np.exp(1j * math.pi * np.arange(8))) * psi
    assert relmax(bq, ref) < 1e-14
    # ranks: every state, and configurations outside the sector
    assert np.array_equal(b.rank(s), np.arange(len(s)))
    bad = np.array([0, 0b11, int(s[0]) + 1, 1 << 16], dtype=np.uint64)
    assert np.all(b.rank(bad) == -1)
    import torch
    sd = torch.from_numpy(np.concatenate([s[::97], bad]).astype(np.int64)).cuda()
    idx = host(b.rank_device(sd))
    assert np.array_equal(idx[:len(s[::97])], np.arange(len(s))[::97]) and np.all(idx[-4:] == -1)
    assert np.array_equal(host(b.states_device(3, 50)).astype(np.uint64), s[3:53])


def test_spin_s_invalid(api, ctx):
    with pytest.raises(api.HphiError):
        api.Basis.spin_s(ctx, 8, 2, 1)      # parity
    with pytest.raises(api.HphiError):
        api.Basis.spin_s(ctx, 8, 8, 0)      # 2S > 7
    with pytest.raises(api.HphiError):
        api.Basis.spin_s(ctx, 21, 2, 0)     # 42 bits
    b = api.Basis.spin_s(ctx, 6, 2, 0)
    with pytest.raises(api.HphiError):
        api.Hamiltonian.spin_s(b, W.spin_s_model(6, 2, [(0, 6)], 1.0, 1.0))
