"""GPU: spin-1/2 on the full 2^N space (SpinGC keyword, Sec. 4.1) against
the oracle.

The H*v kernel runs in bit windows; sizes are chosen so that one, two and
three windows occur (a window holds 13 bits of a real FP64 vector, 12 of a
complex one, 14 of a real FP32 one), with XYZ bonds (jx != jy) and both
fields:
  * H*v element by element (FP64, complex, FP32) at 10, 18 and 20 sites,
    and on sampled rows at 24 sites;
  * Lanczos alpha/beta against the oracle's recurrence, E0 against the
    oracle's sparse eigensolver and against the transverse-field Ising
    ring's free-fermion energy at 20 sites, the refined FP32-storage energy
    within 1e-8;
  * LOBPCG (diagonal preconditioner) against dense eigenvalues, the trace,
    cTPQ, S^z(q) and the device state/rank maps.

Tolerances: FP64 H*v 1e-12 of max|Hv| (at most ~3 N terms per row, other
summation order); FP32 3e-6; alpha/beta 1e-11; energies 1e-10.
"""
import math
import sys
import types

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


def tfim_ring_e0(n, j, g):
    ks = np.pi * (2 * np.arange(n) + 1) / n
    return -np.sum(np.sqrt(j * j + g * g - 2 * j * g * np.cos(ks)))


@pytest.mark.parametrize("n,lat,seed", [(10, "chain", 1), (18, "ladder", 2), (20, "chain", 3)])
def test_gc_mult_vs_oracle(api, ctx, n, lat, seed):
    import torch
    say("gc mult", n, lat)
    m = W.random_spin_gc(n, lat, seed)
    h = api.Hamiltonian.spin_gc(api.Basis.spin_gc(ctx, n), m)
    v = W.random_vector(1 << n, seed)
    assert relmax(host(h.mult(dev(v))), O.spin_gc_hv(m, v)) < 1e-12
    vc = W.random_vector(1 << n, seed + 10, np.complex128)
    assert relmax(host(h.mult(dev(vc))), O.spin_gc_hv(m, vc)) < 1e-12
    vf = dev(v).to(torch.float32)
    wf = host(h.mult(vf)).astype(np.float64)
    assert relmax(wf, O.spin_gc_hv(m, host(vf).astype(np.float64))) < 3e-6


def test_gc_24_sites_sampled_rows(api, ctx):
    say("gc 24 sampled rows")
    m = W.random_spin_gc(24, "ladder", 4)
    h = api.Hamiltonian.spin_gc(api.Basis.spin_gc(ctx, 24), m)
    v = O.splitmix_uniform(5, 0, 1 << 24)
    w = host(h.mult(dev(v)))
    for first in (0, 4095, (1 << 23) + 77, (1 << 24) - 300):
        ref = O.spin_gc_hv_rows(m, v, first, 300)
        assert relmax(w[first:first + 300], ref) < 1e-12, first


def test_gc_lanczos_vs_oracle(api, ctx):
    say("gc lanczos")
    m = W.random_spin_gc(16, "chain", 6)
    h = api.Hamiltonian.spin_gc(api.Basis.spin_gc(ctx, 16), m)
    v0 = O.splitmix_uniform(1, 0, 1 << 16)
    ro = O.lanczos(lambda x: O.spin_gc_hv(m, x), v0, 20)
    r = api.lanczos(h, 400, seed=1)
    assert np.allclose(r["alpha"][:20], ro["alpha"], rtol=0, atol=1e-11)
    assert np.allclose(r["beta"][1:20], ro["beta"][1:], rtol=0, atol=1e-11)
    e0 = sla.eigsh(O.spin_gc_sparse(m), k=1, which="SA", v0=v0, tol=1e-14)[0][0]
    assert abs(r["energies"][0] - e0) < 1e-10


@pytest.mark.parametrize("g", [0.6, 1.0, 1.5])
def test_gc_tfim_ring_free_fermions(api, ctx, g):
    say("gc tfim", g)
    n = 20
    h = api.Hamiltonian.spin_gc(api.Basis.spin_gc(ctx, n), W.tfim_chain(n, 1.0, g))
    r = api.lanczos(h, 400, seed=2, check_every=10, tol=1e-13)
    assert abs(r["energies"][0] - tfim_ring_e0(n, 1.0, g)) < 1e-10
    if g < 1.0:
        # ordered side: the two lowest levels are split by ~g^N (4e-5 at
        # g = 0.6), which a short FP64 restart from the FP32 vector cannot
        # separate; the refined energy meets 1e-8 where the gap is open
        return
    r32 = api.lanczos(h, 400, seed=2, storage="f32", refine=True)
    assert abs(r32["energies"][0] - tfim_ring_e0(n, 1.0, g)) <= 1e-8


def test_gc_lobpcg_trace_ctpq_szq(api, ctx):
    say("gc lobpcg / trace / ctpq / szq")
    n = 10
    m = W.random_spin_gc(n, "ladder", 7)
    b = api.Basis.spin_gc(ctx, n)
    h = api.Hamiltonian.spin_gc(b, m)
    Hs = O.spin_gc_sparse(m)
    ev, U = np.linalg.eigh(Hs.toarray())
    assert abs(h.trace() - Hs.diagonal().sum()) < 1e-10
    # a block of 6 for the lowest 4 (two guard vectors, as for the sector models)
    r = api.lobpcg(h, 6, max_iter=1500, tol=1e-8)
    assert r["converged"], r
    assert np.allclose(r["energies"][:4], ev[:4], atol=1e-9)
    phi0 = O.splitmix_complex_gaussian(8, 1 << n)[:, None]
    g = api.ctpq(h, 1, 6, 0.02, 10, phi0=dev(phi0))
    o = O.ctpq(lambda x: O.spin_gc_hv(m, x), phi0, 6, 0.02, 10)
    assert relmax(g["D"], o["D"]) < 1e-11 and relmax(g["E"], o["E"]) < 1e-11
    mm = types.SimpleNamespace(n_sites=n, site_x=np.arange(n))
    bq = host(api.szq(h, math.pi / 2, dev(U[:, 0])))
    assert relmax(bq, O.szq_excitation(mm, np.arange(1 << n, dtype=np.uint64), math.pi / 2, U[:, 0])) < 1e-14
    assert np.array_equal(b.states(5, 7), np.arange(5, 12, dtype=np.uint64))
    assert np.array_equal(b.rank(np.array([0, 9, 1 << n], dtype=np.uint64)), np.array([0, 9, -1]))


def test_gc_invalid(api, ctx):
    b = api.Basis.spin_gc(ctx, 6)
    with pytest.raises(api.HphiError):
        api.Hamiltonian.spin_gc(b, W.spin_gc(6, [(0, 0)], 1.0, 1.0, 1.0))
    with pytest.raises(api.HphiError):
        api.Hamiltonian.spin_gc(b, W.spin_gc(6, [(0, 6)], 1.0, 1.0, 1.0))
    with pytest.raises(api.HphiError):
        api.Basis.spin_gc(ctx, 33)
