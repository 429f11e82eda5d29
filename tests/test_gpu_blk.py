"""GPU: the block-staged spin product on the implicit basis (schedule
spin_split = 2, and the default 3 there: a workgroup stages the block of one high pattern in LDS;
low bonds read partners there, high bonds read the same positions of the
partner block, bonds across the split read one position of it) against the
oracle and the one-pass product. Split points below, at and above the
basis's own, down to one low site and up to all sites in one block; odd
sites and nonzero S^z; fields; FP64 and FP32; the Lanczos epilogue against
the oracle's recurrence; the 36-site J1-J2 sector at full size on sampled
rows. Tolerances as for the one-pass kernel: FP64 1e-12 of max|Hv|, FP32
3e-6."""
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


def model(name, n):
    if name.startswith("j1j2"):
        return W.j1j2_square(n // 4, 4, 1.0, 0.5)
    if name.startswith("xxz_j2"):
        return W.xxz_chain_j2(n)
    if name.startswith("ladder"):
        m = W.random_heisenberg(n, "ladder", n)
        if "field" in name:
            m.hz = np.random.default_rng(n).normal(size=n)
        return m
    m = W.random_heisenberg(n, "chain", n)
    if "field" in name:
        m.hz = np.random.default_rng(n + 1).normal(size=n)
    return m


# (model, sites, 2S^z, dtype, split point; -1 = the automatic choice)
CASES = [("j1j2_16", 16, 0, "f64", -1), ("j1j2_16", 16, 0, "f32", 5), ("chain_17_field", 17, 1, "f64", 6),
         ("ladder_18_field", 18, 0, "f64", 12), ("xxz_j2_20", 20, 0, "f32", -1), ("xxz_j2_16", 16, 0, "f64", 16),
         ("chain_16", 16, 14, "f64", 3), ("ladder_14", 14, 0, "f64", 1), ("chain_19", 19, 3, "f32", 11),
         ("ladder_16", 16, 0, "f32", 8)]


@pytest.mark.parametrize("name,n,two_sz,dt,lo", CASES, ids=[f"{c[0]}-{c[2]}-{c[3]}-lo{c[4]}" for c in CASES])
def test_blk_mult_vs_oracle(api, ctx, name, n, two_sz, dt, lo):
    import torch
    say("block-staged mult", name, n, two_sz, dt, lo)
    m = model(name, n)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, n, two_sz), m)
    h.set_schedule(spin_implicit=1, spin_split=2, spin_blk_lo=lo)
    sch = h.get_schedule()
    assert sch["spin_split"] == 2 and sch["spin_blk_lo"] == (0 if lo == -1 else lo)
    s = O.basis_list(n, O.sector_popcount_spin(n, two_sz))
    tdt = torch.float64 if dt == "f64" else torch.float32
    vt = dev(W.random_vector(len(s), 11)).to(tdt)
    w = host(h.mult(vt)).astype(np.float64)
    ref = O.spin_hv(m, s, host(vt).astype(np.float64))
    assert relmax(w, ref) < (1e-12 if dt == "f64" else 3e-6)
    # the epilogue: w = c1 H v + c2 u through Lanczos below; here the
    # one-pass product, equal up to summation order
    h.set_schedule(spin_split=-1)
    w1 = host(h.mult(vt)).astype(np.float64)
    assert relmax(w, w1) < (1e-13 if dt == "f64" else 2e-6)


@pytest.mark.parametrize("n,lo", [(18, -1), (17, 4)])
def test_blk_lanczos(api, ctx, n, lo):
    say("block-staged lanczos", n, lo)
    m = W.xxz_chain_j2(n) if n == 18 else W.random_heisenberg(n, "chain", 3)
    two_sz = n % 2
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, n, two_sz), m)
    h.set_schedule(spin_implicit=1, spin_split=2, spin_blk_lo=lo)
    s = O.basis_list(n, O.sector_popcount_spin(n, two_sz))
    r = api.lanczos(h, 60, seed=2)
    o = O.lanczos(lambda x: O.spin_hv(m, s, x), O.splitmix_uniform(2, 0, len(s)), 20)
    assert np.max(np.abs(r["alpha"][:20] - o["alpha"][:20])) < 1e-11
    assert np.max(np.abs(r["beta"][1:20] - o["beta"][1:20])) < 1e-11
    h.set_schedule(spin_split=-1)
    r1 = api.lanczos(h, 60, seed=2)
    assert abs(r["energies"][0] - r1["energies"][0]) < 1e-10
    # FP32 vectors through the same path
    h.set_schedule(spin_split=2)
    r32 = api.lanczos(h, 60, seed=2, storage="f32")
    assert abs(r32["energies"][0] - r1["energies"][0]) < 1e-4 * abs(r1["energies"][0])


def test_blk_is_the_implicit_default(api, ctx):
    # schedule spin_split 3 (the default): block-staged on the implicit
    # basis, one pass on the stored list
    import torch
    say("block-staged default")
    m = W.xxz_chain_j2(18)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 18, 0), m)
    assert h.get_schedule()["spin_split"] == 3
    v = dev(W.random_vector(math.comb(18, 9), 5))
    w_list = host(h.mult(v))
    h.set_schedule(spin_split=-1)
    assert np.array_equal(host(h.mult(v)), w_list)
    h.set_schedule(spin_implicit=1, spin_split=3)
    w_auto = host(h.mult(v))
    h.set_schedule(spin_split=2)
    assert np.array_equal(host(h.mult(v)), w_auto)
    h.set_schedule(spin_split=-1)
    assert relmax(host(h.mult(v)), w_auto) < 1e-13
    torch.cuda.synchronize()


def test_blk_split_point_errors(api, ctx):
    import torch
    say("block-staged split point errors")
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 20, 0), W.xxz_chain_j2(20))
    with pytest.raises(Exception):
        h.set_schedule(spin_blk_lo=25)
    with pytest.raises(Exception):
        h.set_schedule(spin_split=4)
    # all 20 sites in one block of C(20, 10) FP64 values: beyond LDS
    h.set_schedule(spin_implicit=1, spin_split=2, spin_blk_lo=20)
    v = torch.ones(math.comb(20, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(Exception, match="LDS"):
        h.mult(v)
    # the automatic choice runs
    h.set_schedule(spin_blk_lo=-1)
    w = h.mult(v)
    torch.cuda.synchronize()
    assert torch.isfinite(w).all()


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_blk_36_sites_sampled_rows(api, ctx, dt):
    # the 36-site J1-J2 sector (dim 9,075,135,300) at full size in the
    # launch configuration the Lanczos workload times: sampled output rows
    # against the oracle's row formula
    import torch
    say("block-staged 36 sites", dt)
    m = W.j1j2_square(6, 6, 1.0, 0.5)
    b = api.Basis.spin(ctx, 36, 0)
    h = api.Hamiltonian.spin(b, m)
    h.set_schedule(spin_split=2)
    dim = b.dim
    tdt = torch.float32 if dt == "f32" else torch.float64
    g = torch.Generator(device="cuda").manual_seed(6)
    v = torch.rand(dim, dtype=tdt, device="cuda", generator=g) - 0.5
    w = torch.empty_like(v)
    torch.cuda.synchronize()
    h.mult(v, w)
    torch.cuda.synchronize()
    say("  mult done")
    rng = np.random.default_rng(37)
    rows = np.concatenate([[0, 1, dim // 2, dim - 2, dim - 1], rng.integers(0, dim, 400)])
    worst = 0.0
    for r in rows:
        cols, vals = O.spin_row(m, 18, int(r))
        vv = host(v[torch.from_numpy(cols).cuda()]).astype(np.float64)
        ref = float(np.dot(vals, vv))
        scale = float(np.dot(np.abs(vals), np.abs(vv)))
        worst = max(worst, abs(float(w[int(r)]) - ref) / scale)
    assert worst < (2e-6 if dt == "f32" else 1e-13), worst
    del v, w
    torch.cuda.empty_cache()


# blocks of vectors and complex vectors, stored list and implicit basis
VCASES = [("xxz_j2_16", 16, 0, 4, "c128", False), ("ladder_14_field", 14, 0, 16, "c64", False),
          ("chain_15", 15, 1, 1, "c128", True), ("j1j2_16", 16, 0, 8, "f32", True),
          ("xxz_j2_18", 18, 0, 16, "c64", False), ("chain_13", 13, 3, 2, "f64", False)]


@pytest.mark.parametrize("name,n,two_sz,nvec,dt,implicit", VCASES,
                         ids=[f"{c[0]}-{c[3]}x{c[4]}-{'imp' if c[5] else 'list'}" for c in VCASES])
def test_blk_vector_blocks_vs_oracle(api, ctx, name, n, two_sz, nvec, dt, implicit):
    import torch
    say("block-staged vector blocks", name, nvec, dt, implicit)
    m = model(name, n)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, n, two_sz), m)
    h.set_schedule(spin_split=2, spin_implicit=1 if implicit else -1)
    s = O.basis_list(n, O.sector_popcount_spin(n, two_sz))
    cplx = dt.startswith("c")
    v = W.random_vector(len(s), 13, np.complex128 if cplx else np.float64, nvec=nvec)
    if v.ndim == 1:
        v = v[:, None]
    tdt = {"c128": torch.complex128, "c64": torch.complex64, "f64": torch.float64, "f32": torch.float32}[dt]
    vt = dev(v).to(tdt)
    if nvec == 1:
        vt = vt[:, 0].contiguous()
    w = host(h.mult(vt)).reshape(len(s), nvec)
    ref = O.spin_hv(m, s, host(vt).reshape(len(s), nvec).astype(np.complex128 if cplx else np.float64))
    assert relmax(w, ref) < (1e-12 if dt in ("c128", "f64") else 3e-6)
    h.set_schedule(spin_split=-1)
    if implicit and (cplx or nvec > 1):
        # the one-pass implicit kernel takes one real vector only
        with pytest.raises(api.HphiError, match="block-staged"):
            h.mult(vt)
        return
    w1 = host(h.mult(vt)).reshape(len(s), nvec)
    assert relmax(w, w1) < (1e-13 if dt in ("c128", "f64") else 2e-6)


def test_blk_ctpq_and_time_evolution(api, ctx):
    # the caller's epilogues through the block-staged product on a stored
    # list: cTPQ (real coefficients, the first order's raw product) and
    # real-time steps (complex coefficients) against the oracle
    say("block-staged ctpq / time evolution")
    m = W.xxz_chain_j2(16)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 16, 0), m)
    h.set_schedule(spin_split=2)
    s = O.basis_list(16, 8)
    phi = np.stack([O.splitmix_complex_gaussian(30 + j, len(s)) for j in range(4)], axis=1)
    g = api.ctpq(h, 4, 6, 0.02, 10, phi0=dev(phi))
    o = O.ctpq(lambda x: O.spin_hv(m, s, x), phi, 6, 0.02, 10)
    assert relmax(g["D"], o["D"]) < 1e-11 and relmax(g["E"], o["E"]) < 1e-11 and relmax(g["E2"], o["E2"]) < 1e-11
    m2 = W.random_heisenberg(12, "ladder", 8)
    h2 = api.Hamiltonian.spin(api.Basis.spin(ctx, 12, 0), m2)
    h2.set_schedule(spin_split=2)
    s2 = O.basis_list(12, 6)
    phi0 = np.stack([O.splitmix_complex_gaussian(300 + j, len(s2)) for j in range(2)], axis=1)
    psi = dev(phi0)
    t = api.time_evolve(h2, psi, 20, dt=0.02, n_max=8)
    ot = O.taylor_evolve(lambda x: O.spin_hv(m2, s2, x), phi0, 8, 0.02, 20)
    assert np.max(np.abs(t["norm"] - ot["norm"]) / ot["norm"]) < 1e-12
    assert np.max(np.abs(t["energy"] - ot["energy"])) < 1e-10
    assert relmax(host(psi), ot["psi"]) < 1e-11


def test_blk_implicit_basis_complex_methods(api, ctx):
    # complex vectors on the implicit basis (default layout there: the
    # block-staged product; the one-pass kernel takes one real vector):
    # cTPQ and real-time steps against the oracle, their <psi|H psi> from
    # the raw product by a streaming pass
    say("block-staged implicit cTPQ / time evolution")
    m = W.random_heisenberg(14, "ladder", 5)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 14, 0), m)
    h.set_schedule(spin_implicit=1)
    assert h.get_schedule()["spin_split"] == 3
    s = O.basis_list(14, 7)
    phi = np.stack([O.splitmix_complex_gaussian(40 + j, len(s)) for j in range(2)], axis=1)
    g = api.ctpq(h, 2, 5, 0.03, 8, phi0=dev(phi))
    o = O.ctpq(lambda x: O.spin_hv(m, s, x), phi, 5, 0.03, 8)
    assert relmax(g["D"], o["D"]) < 1e-11 and relmax(g["E"], o["E"]) < 1e-11 and relmax(g["E2"], o["E2"]) < 1e-11
    psi = dev(phi)
    t = api.time_evolve(h, psi, 12, dt=0.02, n_max=8)
    ot = O.taylor_evolve(lambda x: O.spin_hv(m, s, x), phi, 8, 0.02, 12)
    assert np.max(np.abs(t["norm"] - ot["norm"]) / ot["norm"]) < 1e-12
    assert np.max(np.abs(t["energy"] - ot["energy"])) < 1e-10
    assert relmax(host(psi), ot["psi"]) < 1e-11


def test_blk_graph_replay(api, ctx):
    # the block-staged product inside captured steps (its tables are built
    # by the eager first step; its queue counters re-arm themselves):
    # replays equal the eager runs bit for bit
    import torch
    say("block-staged graph replay")
    m = W.xxz_chain_j2(16)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 16, 0), m)
    h.set_schedule(spin_implicit=1)
    r0 = api.lanczos(h, 40, seed=3)
    r1 = api.lanczos(h, 40, seed=3, use_graph=True)
    assert np.array_equal(r0["alpha"], r1["alpha"]) and np.array_equal(r0["beta"], r1["beta"])
    phi = np.stack([O.splitmix_complex_gaussian(50 + j, math.comb(16, 8)) for j in range(2)], axis=1)
    a, b = dev(phi), dev(phi)
    t0 = api.time_evolve(h, a, 6, dt=0.02, n_max=6)
    t1 = api.time_evolve(h, b, 6, dt=0.02, n_max=6, use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and np.array_equal(t0["energy"], t1["energy"])
    c0 = api.ctpq(h, 2, 4, 0.02, 6, phi0=dev(phi))
    c1 = api.ctpq(h, 2, 4, 0.02, 6, phi0=dev(phi), use_graph=True)
    assert np.array_equal(c0["E"], c1["E"]) and np.array_equal(c0["D"], c1["D"])


@pytest.mark.parametrize("case", ["all_up_16", "one_down_17", "ising_ladder_14", "long_range_15"])
def test_blk_edge_sectors_and_bonds(api, ctx, case):
    # degenerate sectors (one state, one flipped spin), Ising bonds (no
    # flips) and bonds across the whole chain (every split point cuts
    # them) through the block-staged default on the implicit basis
    import dataclasses
    say("block-staged edge", case)
    if case == "all_up_16":
        m, two_sz = W.xxz_chain_j2(16), 16
        m.hz = np.linspace(-1.0, 1.0, 16)
    elif case == "one_down_17":
        m, two_sz = W.random_heisenberg(17, "chain", 2), 15
    elif case == "ising_ladder_14":
        m0 = W.random_heisenberg(14, "ladder", 3)
        m, two_sz = dataclasses.replace(m0, jxy=np.zeros_like(m0.jxy)), 0
    else:
        rng = np.random.default_rng(15)
        bi = np.arange(15)
        bj = (bi + 7) % 15
        m = W.SpinModel(15, np.concatenate([bi, bi]), np.concatenate([bj, (bi + 1) % 15]),
                        rng.uniform(0.5, 1.5, 30), rng.uniform(0.5, 1.5, 30))
        two_sz = 1
    n = m.n_sites
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, n, two_sz), m)
    h.set_schedule(spin_implicit=1)
    s = O.basis_list(n, O.sector_popcount_spin(n, two_sz))
    v = W.random_vector(len(s), 17)
    w = host(h.mult(dev(v)))
    assert relmax(w, O.spin_hv(m, s, v)) < 1e-12
    h.set_schedule(spin_split=-1)
    assert relmax(host(h.mult(dev(v))), w) < 1e-13
