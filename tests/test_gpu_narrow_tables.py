"""GPU: the stored-list spin kernel with each placement of its rank tables,
against the oracle.

Sectors of 23 to 28 sites run the kernel with hi_off in 32 bits and lo_rank
narrowed to 16 bits in LDS, on 1024-thread workgroups; with fused dots it is
the product of every large served Lanczos and S(q, w) request. The schedule
knob spin_tables forces each placement on sectors the oracle checks
element by element:
  * H*v (FP64, complex and block lanes, FP32) under all three placements,
    and the three products equal bit for bit (the same sums, same order);
  * 20 Lanczos steps' alpha/beta and the converged E0 (fused dots);
  * shifted-COCG D(z) against sparse direct solves (the COCG mu folded
    into the complex product's dots).
A 24-site chain takes the narrowed tables by itself: 20 Lanczos steps of
its alpha/beta against the oracle's recurrence with the oracle's H*v.

Tolerances: FP64 H*v 1e-12 of max|Hv| (74 terms at most per row, different
summation order); Lanczos alpha/beta 1e-12 absolute for the first 20 steps
at 12,870 states and 1e-11 relative at 2.7e6 states (two FP64 dot
products over n terms in different order differ by about sqrt(n) u |alpha|,
1.6e-13 |alpha| at n = 2.7e6, grown by the recurrence); E0 1e-10; D(z) 1e-8
of max|D| with the COCG tolerance 1e-10.
"""
import math
import sys

import numpy as np
import pytest

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


@pytest.mark.parametrize("n,lat,two_sz", [(16, "ladder", 0), (13, "chain", 1), (18, "chain", 2)])
def test_table_placements_mult(api, ctx, n, lat, two_sz):
    import torch
    say("spin tables mult", n, lat, two_sz)
    m = W.random_heisenberg(n, lat, 21)
    b = api.Basis.spin(ctx, n, two_sz)
    h = api.Hamiltonian.spin(b, m)
    s = O.basis_list(n, O.sector_popcount_spin(n, two_sz))
    v = W.random_vector(len(s), 31)
    vc = W.random_vector(len(s), 32, np.complex128, nvec=2)
    ref = O.spin_hv(m, s, v)
    refc = O.spin_hv(m, s, vc)
    outs, outs_c, outs_f = [], [], []
    for tables in (2, 1, 3):
        h.set_schedule(spin_tables=tables)
        assert h.get_schedule()["spin_tables"] == tables
        w = host(h.mult(dev(v)))
        assert relmax(w, ref) < 1e-12, tables
        wc = host(h.mult(dev(vc))).reshape(len(s), 2)
        assert relmax(wc, refc) < 1e-12, tables
        vf = dev(v).to(torch.float32)
        wf = host(h.mult(vf))
        assert relmax(wf, O.spin_hv(m, s, host(vf).astype(np.float64))) < 3e-6
        outs.append(w)
        outs_c.append(wc)
        outs_f.append(wf)
    for k in (1, 2):
        assert np.array_equal(outs[0], outs[k])
        assert np.array_equal(outs_c[0], outs_c[k])
        assert np.array_equal(outs_f[0], outs_f[k])
    h.set_schedule(spin_tables=-1)
    assert h.get_schedule()["spin_tables"] == 0


def test_narrow_tables_lanczos_vs_oracle(api, ctx):
    say("narrow tables lanczos")
    m = W.random_heisenberg(16, "ladder", 5)
    b = api.Basis.spin(ctx, 16, 0)
    h = api.Hamiltonian.spin(b, m)
    h.set_schedule(spin_tables=2)
    r = api.lanczos(h, 200, seed=1)
    s = O.basis_list(16, 8)
    v0 = O.splitmix_uniform(1, 0, len(s))
    ro = O.lanczos(lambda x: O.spin_hv(m, s, x), v0, 200)
    assert np.allclose(r["alpha"][:20], ro["alpha"][:20], rtol=0, atol=1e-12)
    assert np.allclose(r["beta"][1:20], ro["beta"][1:20], rtol=0, atol=1e-12)
    e_or = O.tridiag_lowest(ro["alpha"], ro["beta"])[0]
    assert abs(r["energies"][0] - e_or) < 1e-10
    # converged: the dense-free check against the oracle's sparse eigensolver
    import scipy.sparse.linalg as sla
    ev = sla.eigsh(O.spin_sparse(m, s), k=1, which="SA", v0=v0, tol=1e-14)[0][0]
    assert abs(r["energies"][0] - ev) < 1e-10
    # the checked Ritz vector through the same kernel
    r2 = api.lanczos(h, 200, seed=1, want_vector=True, check_every=10, tol=1e-12)
    assert r2["converged"] and abs(r2["energies"][0] - ev) < 1e-10


@pytest.mark.parametrize("lattice,n,q", [("chain", 12, math.pi), ("ladder", 12, math.pi), ("chain", 13, math.pi),
                                         ("ladder", 12, 2 * math.pi / 3)])
def test_narrow_tables_sqw_vs_direct_solve(api, ctx, lattice, n, q):
    say("narrow tables sqw", lattice, n, q)
    m = W.random_heisenberg(n, lattice, 17)
    two_sz = n % 2
    b = api.Basis.spin(ctx, n, two_sz)
    h = api.Hamiltonian.spin(b, m)
    h.set_schedule(spin_tables=2)
    s = O.basis_list(n, O.sector_popcount_spin(n, two_sz))
    Hs = O.spin_sparse(m, s)
    ev, U = np.linalg.eigh(Hs.toarray())
    bo = O.szq_excitation(m, s, q, U[:, 0])
    bg = api.szq(h, q, dev(U[:, 0]))
    assert relmax(host(bg), bo) < 1e-14
    z = ev[0] + np.linspace(0, 4 * 1.5, 64) + 0.05j
    g = api.sqw(h, bg, z, max_iter=3000, tol=1e-10)
    assert g["converged"], g["max_residual"]
    assert relmax(g["D"], O.dyn_corr_direct(Hs, bo, z)) < 1e-8
    assert np.all(-g["D"].imag > 0)


def test_lanczos_24_sites_vs_oracle(api, ctx):
    say("lanczos 24 sites")
    m = W.random_heisenberg(24, "chain", 9)
    b = api.Basis.spin(ctx, 24, 0)
    h = api.Hamiltonian.spin(b, m)
    r = api.lanczos(h, 20, seed=1)
    # the automatic choice at 24 sites is the narrowed-table kernel
    h.set_schedule(spin_tables=2)
    r2 = api.lanczos(h, 20, seed=1)
    assert np.array_equal(r["alpha"], r2["alpha"]) and np.array_equal(r["beta"], r2["beta"])
    s = O.basis_list(24, 12)
    v0 = O.splitmix_uniform(1, 0, len(s))
    ro = O.lanczos(lambda x: O.spin_hv(m, s, x), v0, 20)
    assert np.allclose(r["alpha"], ro["alpha"], rtol=1e-11, atol=0)
    assert np.allclose(r["beta"][1:], ro["beta"][1:], rtol=1e-11, atol=0)
    assert abs(r["energies"][0] - O.tridiag_lowest(ro["alpha"], ro["beta"])[0]) < 1e-10
