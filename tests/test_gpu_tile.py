"""GPU: the block-tile T_up kernel of the Hubbard product (hub_sweep 7)
against the oracle, alone and inside the Lanczos recurrence, where the run
stores its vectors with rows padded to whole 128-byte lines.

The up rows split by their top hub_tile_bits sites into blocks of
consecutive rows; hops inside a block read the block's rows staged in LDS,
the others gather from memory. Checks: H*v element by element (1e-12 of
max|Hv|) for several splits, a split whose lists exceed the kernel refused
cleanly; the full 4x4 half-filled sector on sampled rows
(its 12870 down states leave a last slab of 6 columns); Lanczos alpha/beta
(first 20 steps, 1e-12) and E0 (1e-10) against the oracle's recurrence with
the oracle's H*v, through the padded layout (first product: plain rows
kernel; later ones: the update fused into the rows kernel), with the Ritz
vector and the FP64 refinement; FP32 storage; padded and unpadded runs of
the same schedule agree to rounding."""
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


@pytest.mark.parametrize("lx,ly,nu,nd,bits", [(3, 4, 6, 6, 0), (3, 4, 6, 5, 4), (4, 3, 5, 5, 3), (4, 4, 3, 5, 0),
                                              (4, 4, 5, 7, 4)])
def test_tile_mult_matches_oracle(api, ctx, lx, ly, nu, nd, bits):
    import torch
    say("tile mult", lx, ly, nu, nd, bits)
    m = W.hubbard_square(lx, ly, 1.0, 4.0)
    n = lx * ly
    b = api.Basis.hubbard(ctx, n, nu, nd)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(n, nu, nd)
    v = W.random_vector(b.dim, 71)
    ref = O.hubbard_hv(m, ups, dns, v)
    h.set_schedule(hub_sweep=5)
    w5 = host(h.mult(dev(v)))
    h.set_schedule(hub_sweep=7, hub_tile_bits=bits if bits else -1)
    w7 = host(h.mult(dev(v)))
    assert relmax(w7, ref) < 1e-12
    assert relmax(w7, w5) < 1e-13
    # run to run identical; FP32 storage through the same kernel
    assert np.array_equal(w7, host(h.mult(dev(v))))
    vf = dev(v).to(torch.float32)
    wf = host(h.mult(vf))
    assert relmax(wf, O.hubbard_hv(m, ups, dns, host(vf).astype(np.float64))) < 3e-6


def test_tile_split_beyond_the_kernel_is_refused(api, ctx):
    # one-row blocks make every hop far (more than a row's register lists
    # hold): the schedule is refused and the product keeps its kernel
    m = W.hubbard_square(4, 3, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 12, 5, 5)
    h = api.Hamiltonian.hubbard(b, m)
    v = W.random_vector(b.dim, 72)
    ref = host(h.mult(dev(v)))
    with pytest.raises(api.HphiError) as e:
        h.set_schedule(hub_sweep=7, hub_tile_bits=12)
    assert e.value.code == -6
    h.set_schedule(hub_tile_bits=-1)
    h.set_schedule(hub_sweep=7)
    ups, dns = O.hubbard_basis(12, 5, 5)
    assert relmax(host(h.mult(dev(v))), O.hubbard_hv(m, ups, dns, v)) < 1e-12
    assert relmax(host(h.mult(dev(v))), ref) < 1e-13


def test_tile_4x4_full_size_sampled_rows(api, ctx):
    import torch
    say("tile 4x4 full size")
    m = W.hubbard_square(4, 4, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 16, 8, 8)
    h = api.Hamiltonian.hubbard(b, m)
    h.set_schedule(hub_sweep=7)
    ups, dns = O.hubbard_basis(16, 8, 8)
    g = torch.Generator(device="cuda").manual_seed(13)
    v = torch.rand(b.dim, dtype=torch.float64, device="cuda", generator=g) - 0.5
    w = h.mult(v)
    assert torch.equal(w, h.mult(v))
    rng = np.random.default_rng(17)
    last = np.arange(b.dim - 12870, b.dim)[-8:]     # the ragged last slab of the last row
    rows = np.concatenate([[0], last, rng.integers(0, b.dim, 3000)])
    wmax = float(w.abs().max())
    errs = []
    for r in rows:
        cols, vals = O.hubbard_row(m, ups, dns, int(r) // 12870, int(r) % 12870)
        vv = host(v[torch.from_numpy(cols).cuda()])
        errs.append(abs(float(w[int(r)]) - float(np.dot(vals, vv))))
    assert max(errs) / wmax < 1e-12
    del v, w


def test_tile_lanczos_padded_vs_oracle(api, ctx):
    import torch
    say("tile lanczos 3x4 (padded rows)")
    m = W.hubbard_square(3, 4, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 12, 6, 6)     # 924 x 924 states: rows padded to 928
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(12, 6, 6)
    hv = lambda x: O.hubbard_hv(m, ups, dns, x)
    v0 = O.splitmix_uniform(3, 0, b.dim)
    ro = O.lanczos(hv, v0, 250)
    e_or = O.tridiag_lowest(ro["alpha"], ro["beta"])[0]
    assert h.get_schedule()["hub_sweep"] == 7     # the default where the tables exist
    h.set_schedule(hub_sweep=5)
    r5 = api.lanczos(h, 250, seed=3)
    h.set_schedule(hub_sweep=7)
    r7 = api.lanczos(h, 250, seed=3, want_vector=True)
    assert r7["fused_update"]
    assert np.allclose(r7["alpha"][:20], ro["alpha"][:20], rtol=0, atol=1e-12)
    assert np.allclose(r7["beta"][1:20], ro["beta"][1:20], rtol=0, atol=1e-12)
    assert abs(r7["energies"][0] - e_or) < 1e-10
    assert abs(r7["energies"][0] - r5["energies"][0]) < 1e-10
    # the Ritz vector leaves the padded layout through the accumulation
    psi = host(r7["psi"])
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12
    assert np.linalg.norm(hv(psi) - r7["energies"][0] * psi) < 1e-6
    # caller start vector, graph capture, refinement through the same path
    rg = api.lanczos(h, 250, v0=dev(v0), use_graph=True)
    assert np.array_equal(rg["alpha"], r7["alpha"])
    rr = api.lanczos(h, 250, seed=3, refine=True)
    assert abs(rr["rq_e0"] - e_or) < 1e-10 and rr["residual"] < 1e-6
    # FP32 vectors: padded to 32 floats per line
    rf = api.lanczos(h, 250, seed=3, storage="f32", refine=True)
    assert abs(rf["energies"][0] - e_or) < 1e-9
    # the static-scratch entry point keeps unpadded rows; every sum runs in
    # the same order (the start norm is taken in the unpadded order), so the
    # numbers are the same bit for bit
    rn = api.lanczos(h, 250, seed=3, no_alloc=True)
    assert np.array_equal(rn["alpha"], r7["alpha"]) and np.array_equal(rn["beta"], r7["beta"])
    del torch
