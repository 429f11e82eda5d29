"""GPU: the Hubbard paths of the spectral and finite-temperature rows through
the C ABI -- S^z(q) excitation against the oracle, S^zz(q, w) by shifted
COCG against the full-spectrum sum, canonical TPQ against the oracle's
propagator and, with the bootstrap, against exact canonical values of the
sector; FP32 / complex64 H*v and FP32-storage Lanczos."""
import math
import sys

import numpy as np
import pytest
import scipy.sparse.linalg

from oracle import core as O
from paper_2307_13222_amd import thermo as T
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


def ground(Hs):
    e, u = scipy.sparse.linalg.eigsh(Hs, k=1, which="SA")
    return float(e[0]), u[:, 0]


@pytest.mark.parametrize("lx,ly,nu,nd,q", [(4, 2, 4, 4, math.pi / 2), (4, 2, 5, 3, math.pi),
                                           (3, 3, 4, 5, 2 * math.pi / 3), (2, 3, 3, 0, 0.7)])
def test_hubbard_szq_matches_oracle(api, ctx, lx, ly, nu, nd, q):
    say("hub szq", lx, ly, nu, nd)
    m = W.hubbard_square(lx, ly, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, m.n_sites, nu, nd)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(m.n_sites, nu, nd)
    psi = W.random_vector(b.dim, 31)
    bg = host(api.szq(h, q, dev(psi)))
    bo = O.hubbard_szq_excitation(m, ups, dns, q, psi)
    assert relmax(bg, bo) < 1e-14


def test_hubbard_sqw_matches_spectral_sum(api, ctx):
    say("hub sqw")
    m = W.hubbard_square(4, 2, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 8, 3, 3)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(8, 3, 3)
    Hd = O.hubbard_sparse(m, ups, dns).toarray()
    ev, U = np.linalg.eigh(Hd)
    e0, psi = ev[0], U[:, 0]
    q = math.pi / 2                      # complex phases 1, i, -1, -i along x
    bo = O.hubbard_szq_excitation(m, ups, dns, q, psi)
    # momentum excitation: b^T b vanishes, the device solver splits Re / Im
    assert np.max(np.abs(bo.imag)) > 1e-3 and abs(np.sum(bo * bo)) < 1e-12
    bg = api.szq(h, q, dev(psi))
    assert relmax(host(bg), bo) < 1e-14
    z = e0 + np.linspace(0.0, 12.0, 48) + 0.1j
    g = api.sqw(h, bg, z, max_iter=3000, tol=1e-10)
    assert g["converged"], g["max_residual"]
    # spectral sum over the full spectrum (pinned to direct solves on the CPU)
    d_ref = O.dyn_corr_spectral(Hd, bo, z)
    assert relmax(g["D"], d_ref) < 1e-8
    assert np.all(-g["D"].imag > 0)


@pytest.mark.parametrize("dt,tol", [("c128", 1e-11), ("c64", 2e-5)])
def test_hubbard_ctpq_matches_oracle(api, ctx, dt, tol):
    import torch
    say("hub ctpq", dt)
    m = W.hubbard_square(3, 3, 1.0, 6.0)
    b = api.Basis.hubbard(ctx, 9, 4, 5)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(9, 4, 5)
    phi0 = O.splitmix_complex_gaussian(77, b.dim)[:, None]
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    g = api.ctpq(h, 1, 6, 0.02, 20, storage=dt, phi0=dev(phi0).to(tdt))
    phi_in = host(dev(phi0).to(tdt)).astype(np.complex128)
    o = O.ctpq(lambda x: O.hubbard_hv(m, ups, dns, x), phi_in, 6, 0.02, 20)
    assert relmax(g["D"], o["D"]) < tol
    assert relmax(g["E"], o["E"]) < tol
    assert relmax(g["E2"], o["E2"]) < tol


def test_hubbard_ctpq_thermodynamics_against_canonical(api, ctx):
    say("hub ctpq thermo")
    m = W.hubbard_square(2, 3, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 6, 3, 3)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(6, 3, 3)
    ev = np.linalg.eigvalsh(O.hubbard_sparse(m, ups, dns).toarray())
    runs = [api.ctpq(h, 1, 6, 0.02, 150, storage="c128", seed=11 + j) for j in range(12)]
    D = np.concatenate([r["D"] for r in runs], axis=1)
    E = np.concatenate([r["E"] for r in runs], axis=1)
    E2 = np.concatenate([r["E2"] for r in runs], axis=1)
    th = T.tpq_thermo(runs[0]["beta"], D, E, E2, b.dim, 6, n_boot=200)
    ex = O.canonical_thermo(ev, runs[0]["beta"], 6)
    for key in ("E", "C", "S"):
        dev_ = np.abs(th[key] - ex[key])
        assert np.all(dev_ < 5 * th[key + "_err"] + 5e-3), (key, float(dev_.max()))
    assert abs(th["S"][0] - math.log(b.dim) / 6) < 1e-12


@pytest.mark.parametrize("lx,ly,nu,nd", [(4, 2, 4, 4), (3, 4, 6, 5)])
def test_hubbard_mult_f32_c64(api, ctx, lx, ly, nu, nd):
    import torch
    say("hub mult f32", lx, ly, nu, nd)
    m = W.hubbard_square(lx, ly, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, m.n_sites, nu, nd)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(m.n_sites, nu, nd)
    # the oracle gets the FP32-rounded input; FP32 accumulation over at most
    # 2 * hops + 1 terms of size <= U / 2 bounds the error well below 1e-5
    v = dev(W.random_vector(b.dim, 41)).to(torch.float32)
    w = host(h.mult(v)).astype(np.float64)
    assert relmax(w, O.hubbard_hv(m, ups, dns, host(v).astype(np.float64))) < 1e-5
    vc = dev(W.random_vector(b.dim, 42, np.complex128)).to(torch.complex64)
    wc = host(h.mult(vc)).astype(np.complex128)
    assert relmax(wc, O.hubbard_hv(m, ups, dns, host(vc).astype(np.complex128))) < 1e-5


def test_hubbard_lanczos_f32_storage(api, ctx):
    say("hub lanczos f32")
    m = W.hubbard_square(4, 2, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 8, 4, 4)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(8, 4, 4)
    e0, _ = ground(O.hubbard_sparse(m, ups, dns))
    r = api.lanczos(h, 200, seed=3, storage="f32")
    # FP32 vectors, FP64 scalars: the Ritz value sits within FP32 rounding of E0
    assert abs(r["energies"][0] - e0) < 1e-4 * abs(e0)


@pytest.mark.parametrize("lx,ly,nu,nd", [(3, 4, 6, 5), (4, 4, 3, 5)])
def test_hubbard_batched_list_walk_bit_identical(api, ctx, lx, ly, nu, nd):
    # T_up with the batched list walk (hub_sweep 5) and T_dn with the batched
    # row staging (hub_row_cols 5, and 6 with pre-scaled slot words) keep
    # every sum's order, also with several rows per wave on 32-column slabs:
    # real, complex and FP32 products, the fused Lanczos epilogue and dots,
    # and the complex Taylor epilogue equal the two-list walk bit for bit
    import torch
    say("hub batched walk", lx, ly, nu, nd)
    m = W.hubbard_square(lx, ly, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, m.n_sites, nu, nd)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(m.n_sites, nu, nd)
    base = dict(hub_slab_cols=128, hub_groups=128, hub_item_rows=32)
    ins = [dev(W.random_vector(b.dim, 51)), dev(W.random_vector(b.dim, 52, np.complex128)),
           dev(W.random_vector(b.dim, 53)).to(torch.float32)]
    out = {}
    for key, sch in (("two_list", dict(hub_row_cols=4, hub_sweep=3, hub_row_order=1)),
                     ("batched", dict(hub_row_cols=5, hub_sweep=5, hub_row_order=1)),
                     ("rcm", dict(hub_row_cols=5, hub_sweep=5, hub_row_order=2)),
                     ("prescaled", dict(hub_row_cols=6, hub_sweep=5, hub_row_order=2)),
                     ("narrow", dict(hub_slab_cols=32, hub_row_cols=6, hub_sweep=5, hub_row_order=2))):
        h.set_schedule(**{**base, **sch})
        prods = [host(h.mult(x)) for x in ins]
        lz = api.lanczos(h, 60, seed=4) if sch["hub_row_cols"] == 4 else None
        psi = dev(W.random_vector(b.dim, 54, np.complex128))
        te = api.time_evolve(h, psi, 3, dt=0.05, n_max=6)
        out[key] = (prods, lz, host(psi), te)
    a = out["two_list"]
    for c in (out["batched"], out["rcm"], out["prescaled"], out["narrow"]):
        for x, y in zip(a[0], c[0]):
            assert np.array_equal(x, y)
        assert np.array_equal(a[2], c[2])
    assert relmax(a[0][0], O.hubbard_hv(m, ups, dns, host(ins[0]))) < 1e-12


def test_hubbard_lanczos_fused_update(api, ctx):
    # with hub_row_cols 5 (and 6) the Lanczos update (w -= alpha q,
    # beta = |w|) runs inside the next product's rows kernel: same recurrence
    # as the separate update kernel up to the order of the |w|^2 sum
    say("hub lanczos fused")
    m = W.hubbard_square(4, 4, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 16, 3, 5)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(16, 3, 5)
    h.set_schedule(hub_row_cols=4)
    ref = api.lanczos(h, 80, seed=6)
    h.set_schedule(hub_row_cols=5)
    fz = api.lanczos(h, 80, seed=6)
    # pre-scaled slot words: the same sums in the same order
    h.set_schedule(hub_row_cols=6)
    f6 = api.lanczos(h, 80, seed=6)
    assert np.array_equal(f6["alpha"], fz["alpha"]) and np.array_equal(f6["beta"], fz["beta"])
    assert f6["fused_update"]
    # rounding differences grow along a Lanczos sequence without
    # reorthogonalization: early coefficients agree to rounding, the ground
    # energy to the Lanczos bar
    assert relmax(fz["alpha"][:20], ref["alpha"][:20]) < 1e-12
    assert relmax(fz["beta"][:20], ref["beta"][:20]) < 1e-12
    assert abs(fz["energies"][0] - ref["energies"][0]) < 1e-10
    assert fz["fused_update"] and not ref["fused_update"]
    # oracle Lanczos on the same start vector (SplitMix64 stream)
    ro = O.lanczos(lambda x: O.hubbard_hv(m, ups, dns, x), O.splitmix_uniform(6, 0, b.dim), 20)
    assert relmax(fz["alpha"][:20], ro["alpha"][:20]) < 1e-11
    assert relmax(fz["beta"][1:20], ro["beta"][1:20]) < 1e-11
    # fixed-order reductions: run to run and graph replay bit-identical
    fz2 = api.lanczos(h, 80, seed=6)
    fg = api.lanczos(h, 80, seed=6, use_graph=True)
    for r in (fz2, fg):
        assert np.array_equal(r["alpha"], fz["alpha"]) and np.array_equal(r["beta"], fz["beta"])
    # Ritz vector from the second pass through the same fused steps
    rv = api.lanczos(h, 200, seed=6, want_vector=True)
    psi = host(rv["psi"])
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12
    res = O.hubbard_hv(m, ups, dns, psi) - rv["energies"][0] * psi
    assert np.linalg.norm(res) < 1e-6
    # convergence checks read the lagging iteration count correctly
    rc = api.lanczos(h, 400, seed=6, check_every=10, tol=1e-12)
    assert rc["converged"] and abs(rc["energies"][0] - rv["energies"][0]) < 1e-10
    # FP32 vectors take the fused kernel too
    r4 = api.lanczos(h, 200, seed=6, storage="f32")
    assert abs(r4["energies"][0] - rv["energies"][0]) < 1e-4 * abs(rv["energies"][0])
    h.set_schedule(hub_row_cols=5)
    r45 = api.lanczos(h, 200, seed=6, storage="f32")
    assert np.array_equal(r4["alpha"], r45["alpha"]) and np.array_equal(r4["beta"], r45["beta"])


@pytest.mark.parametrize("rc", [5, 6])
def test_hubbard_lanczos_fused_update_edges(api, ctx, rc):
    # the fused path's scalar step (and breakdown test) runs in the rows
    # kernel's last block; the last step's update after the loop
    say("hub lanczos fused edges", rc)
    m = W.hubbard_square(2, 3, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 6, 2, 3)
    h = api.Hamiltonian.hubbard(b, m)
    h.set_schedule(hub_row_cols=rc)
    ups, dns = O.hubbard_basis(6, 2, 3)
    hv = lambda x: O.hubbard_hv(m, ups, dns, x)
    v0 = O.splitmix_uniform(9, 0, b.dim)
    ro = O.lanczos(hv, v0, 3)
    for n in (1, 2, 3):
        r = api.lanczos(h, n, seed=9)
        assert r["fused_update"] and r["iterations"] == n
        assert relmax(r["alpha"], ro["alpha"][:n]) < 1e-12
        if n > 1:
            assert relmax(r["beta"][1:], np.asarray(ro["beta"])[1:n]) < 1e-12
    # more steps than states: the recurrence breaks down (beta -> 0) inside
    # the fused kernel; the lowest level is still found
    m2 = W.hubbard_square(2, 2, 1.0, 4.0)
    b2 = api.Basis.hubbard(ctx, 4, 1, 1)
    h2 = api.Hamiltonian.hubbard(b2, m2)
    h2.set_schedule(hub_row_cols=rc)
    u2, d2 = O.hubbard_basis(4, 1, 1)
    e = np.linalg.eigvalsh(O.hubbard_sparse(m2, u2, d2).toarray())
    r2 = api.lanczos(h2, 40, seed=2)
    assert r2["fused_update"] and r2["breakdown"] and r2["iterations"] <= b2.dim
    assert abs(r2["energies"][0] - e[0]) < 1e-10
    r3 = api.lanczos(h2, 40, seed=2, want_vector=True)
    psi = host(r3["psi"])
    assert np.linalg.norm(O.hubbard_hv(m2, u2, d2, psi) - e[0] * psi) < 1e-8


@pytest.mark.parametrize("nu,nd", [(1, 7), (2, 7)])
def test_hubbard_complex_wide_rows(api, ctx, nu, nd):
    # complex128 rows of 11440 down states (183 KB) exceed LDS: the rows
    # kernel stages one lane (re, im) at a time; the slab kernel takes the
    # uniform-|t| path
    say("hub complex wide rows", nu, nd)
    m = W.hubbard_square(4, 4, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 16, nu, nd)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(16, nu, nd)
    vc = W.random_vector(b.dim, 61, np.complex128)
    wc = host(h.mult(dev(vc)))
    assert relmax(wc, O.hubbard_hv(m, ups, dns, vc)) < 1e-12
    # the same product through the general rows kernel (hop lists in order)
    h.set_schedule(hub_row_cols=1)
    wg = host(h.mult(dev(vc)))
    assert relmax(wg, O.hubbard_hv(m, ups, dns, vc)) < 1e-12
    h.set_schedule(hub_row_cols=5)


def test_hubbard_4x4_complex_full_size_sampled_rows(api, ctx):
    # the complex FP64 product of the full half-filled 4x4 sector (the real-time
    # evolution workload): lane-by-lane rows kernel + complex slab kernel
    import torch
    say("hub 4x4 complex full size")
    m = W.hubbard_square(4, 4, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 16, 8, 8)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(16, 8, 8)
    g = torch.Generator(device="cuda").manual_seed(5)
    v = torch.complex(torch.rand(b.dim, dtype=torch.float64, device="cuda", generator=g) - 0.5,
                      torch.rand(b.dim, dtype=torch.float64, device="cuda", generator=g) - 0.5)
    w = h.mult(v)
    assert torch.equal(w, h.mult(v))
    rng = np.random.default_rng(9)
    rows = np.concatenate([[0, b.dim - 1], rng.integers(0, b.dim, 2000)])
    wmax = float(w.abs().max())
    errs = []
    for r in rows:
        cols, vals = O.hubbard_row(m, ups, dns, int(r) // 12870, int(r) % 12870)
        vv = host(v[torch.from_numpy(cols).cuda()])
        errs.append(abs(complex(w[int(r)]) - complex(np.dot(vals, vv))))
    assert max(errs) / wmax < 1e-12
    del v, w
