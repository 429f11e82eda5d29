"""GPU: hipGraph replay of the cTPQ and real-time-evolution steps, and the
schedule autotuner.

Graph replay: one step's launches are captured once and replayed; the
launches, buffers and reductions are those of the eager steps, so D_k,
<H>, <H^2> (cTPQ) and norms, energies, double occupancy and the final
state (Taylor evolution) agree bit for bit -- for a wide spin block (the
raw-dots path), complex64 storage, and the Hubbard product.

Autotuner: a sweep over the schedule knobs (T_up kernel, tile split, block
width of the spin kernel's rank tables, workgroups) picks a schedule whose
products match the oracle (FP64 1e-12 of max|Hv|), records it, and a second
call applies the record without sweeping."""
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


@pytest.mark.parametrize("kind,dt,nv", [("spin", "c128", 4), ("spin", "c64", 2), ("hubbard", "c128", 1)])
def test_ctpq_graph_equals_eager(api, ctx, kind, dt, nv):
    say("ctpq graph", kind, dt, nv)
    if kind == "spin":
        h = api.Hamiltonian.spin(api.Basis.spin(ctx, 14, 0), W.random_heisenberg(14, "ladder", 4))
    else:
        h = api.Hamiltonian.hubbard(api.Basis.hubbard(ctx, 9, 4, 5), W.hubbard_square(3, 3, 1.0, 6.0))
    e = api.ctpq(h, nv, 6, 0.02, 12, storage=dt, seed=31)
    g = api.ctpq(h, nv, 6, 0.02, 12, storage=dt, seed=31, use_graph=True)
    for key in ("D", "E", "E2"):
        assert np.array_equal(e[key], g[key]), key
    assert np.array_equal(host(e["phi"]), host(g["phi"]))
    # and the graph run against the oracle from the same start block
    if kind == "spin" and dt == "c128":
        m = h.model
        s = O.basis_list(14, 7)
        phi0 = np.stack([O.splitmix_complex_gaussian(31 + j, len(s)) for j in range(nv)], axis=1)
        o = O.ctpq(lambda x: O.spin_hv(m, s, x), phi0, 6, 0.02, 12)
        assert relmax(g["E"], o["E"]) < 1e-11 and relmax(g["D"], o["D"]) < 1e-11


@pytest.mark.parametrize("kind", ["spin", "hubbard"])
def test_tevol_graph_equals_eager(api, ctx, kind):
    import torch
    say("tevol graph", kind)
    if kind == "spin":
        h = api.Hamiltonian.spin(api.Basis.spin(ctx, 12, 0), W.random_heisenberg(12, "chain", 6))
        nv, docc = 2, False
    else:
        h = api.Hamiltonian.hubbard(api.Basis.hubbard(ctx, 10, 5, 5), W.hubbard_chain(10, 1.0, 8.0))
        nv, docc = 1, True
    g = torch.Generator(device="cuda").manual_seed(9)
    shape = (h.basis.dim, nv) if nv > 1 else (h.basis.dim,)
    psi0 = torch.complex(torch.rand(shape, dtype=torch.float64, device="cuda", generator=g) - 0.5,
                         torch.rand(shape, dtype=torch.float64, device="cuda", generator=g) - 0.5)
    psi0 /= torch.linalg.norm(psi0)
    pa, pb = psi0.clone(), psi0.clone()
    ea = api.time_evolve(h, pa, 15, dt=0.01, n_max=8, double_occupancy=docc)
    eb = api.time_evolve(h, pb, 15, dt=0.01, n_max=8, double_occupancy=docc, use_graph=True)
    for key in ea:
        assert np.array_equal(ea[key], eb[key]), key
    assert torch.equal(pa, pb)


def test_autotune_sweep_and_record(api, ctx, tmp_path):
    import torch
    from paper_2307_13222_amd import autotune
    say("autotune")
    table = str(tmp_path / "schedules.json")
    m = W.hubbard_square(3, 4, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 12, 6, 6)
    h = api.Hamiltonian.hubbard(b, m)
    cands = autotune.candidates(h, quick=True)
    assert any(c.get("hub_sweep") == 7 for c in cands) and any(c.get("hub_sweep") == 5 for c in cands)
    r = autotune.tune(h, "f64", 1, reps=3, table=table, cands=cands)
    assert r["swept"] and r["n_valid"] >= 2
    ups, dns = O.hubbard_basis(12, 6, 6)
    v = W.random_vector(b.dim, 91)
    assert relmax(host(h.mult(dev(v))), O.hubbard_hv(m, ups, dns, v)) < 1e-12
    r2 = autotune.tune(h, "f64", 1, table=table)
    assert not r2["swept"] and r2["schedule"] == r["schedule"]
    # spin: the one-pass kernel (rank-table placement x workgroups per CU)
    # against the block-staged product, for a batched product; every
    # candidate names its layout
    ms = W.xxz_chain_j2(18)
    hs = api.Hamiltonian.spin(api.Basis.spin(ctx, 18, 0), ms)
    cs = autotune.candidates(hs, quick=True)
    assert all("spin_split" in c for c in cs) and any(c["spin_split"] == 2 for c in cs)
    rs = autotune.tune(hs, "c64", 8, reps=3, table=table, cands=cs)
    assert rs["swept"] and hs.get_schedule()["spin_split"] == rs["schedule"]["spin_split"]
    s = O.basis_list(18, 9)
    vb = W.random_vector(len(s), 92, np.complex128, nvec=8)
    vt = dev(vb).to(torch.complex64)
    w = host(hs.mult(vt)).reshape(len(s), 8)
    assert relmax(w, O.spin_hv(ms, s, host(vt).astype(np.complex128))) < 3e-6
