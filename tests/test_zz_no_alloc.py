"""GPU: the Lanczos entry point that allocates nothing
(hphi_lanczos_noalloc, buffers from the library's static device scratch)
against hphi_lanczos, which allocates them: the same kernels on the same
reductions, so alpha/beta, energies and the Ritz vector agree bit for bit.
Two calls in a row, the second on a smaller sector (the scratch keeps the
first call's contents, so what must start at zero is cleared by the call);
FP32 storage with the FP64 refinement; a Hubbard sector (fused update);
a sector whose workspace exceeds the scratch fails with INVALID_ARG."""
import sys

import numpy as np
import pytest

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


def _same(r1, r2):
    assert r1["iterations"] == r2["iterations"]
    assert np.array_equal(r1["alpha"], r2["alpha"])
    assert np.array_equal(r1["beta"], r2["beta"])
    assert np.array_equal(r1["energies"], r2["energies"])


def test_noalloc_matches_allocating_entry_point(api, ctx):
    import torch
    say("no-alloc lanczos: 18-site ladder, then 12-site chain")
    big = api.Hamiltonian.spin(api.Basis.spin(ctx, 18, 0), W.random_heisenberg(18, "ladder", 3))
    small = api.Hamiltonian.spin(api.Basis.spin(ctx, 12, 0), W.random_heisenberg(12, "chain", 4))
    for h, it, seed in ((big, 120, 5), (small, 80, 6)):
        ref = api.lanczos(h, it, seed=seed, n_energies=2, want_vector=True)
        got = api.lanczos(h, it, seed=seed, n_energies=2, want_vector=True, no_alloc=True)
        _same(ref, got)
        assert torch.equal(ref["psi"], got["psi"])
    # checked run with a residual stop and a caller start vector
    v0 = torch.rand(small.basis.dim, dtype=torch.float64, device="cuda") - 0.5
    ref = api.lanczos(small, 300, v0=v0, check_every=10, tol=1e-12, resid_tol=1e-9)
    got = api.lanczos(small, 300, v0=v0, check_every=10, tol=1e-12, resid_tol=1e-9, no_alloc=True)
    _same(ref, got)
    assert got["converged"]


def test_noalloc_fp32_refined_and_hubbard(api, ctx):
    say("no-alloc lanczos: FP32 refined, Hubbard")
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 16, 0), W.heisenberg_chain(16))
    ref = api.lanczos(h, 200, seed=1, storage="f32", refine=True)
    got = api.lanczos(h, 200, seed=1, storage="f32", refine=True, no_alloc=True)
    _same(ref, got)
    assert got["rq_e0"] == ref["rq_e0"] and got["residual"] == ref["residual"]
    assert got["polish_e0"] == ref["polish_e0"] and got["polish_resid"] == ref["polish_resid"]
    hh = api.Hamiltonian.hubbard(api.Basis.hubbard(ctx, 10, 5, 5), W.hubbard_square(2, 5, 1.0, 4.0))
    ref = api.lanczos(hh, 150, seed=2)
    got = api.lanczos(hh, 150, seed=2, no_alloc=True)
    _same(ref, got)
    # and the smaller spin sector again after the larger Hubbard one
    _same(api.lanczos(h, 50, seed=3), api.lanczos(h, 50, seed=3, no_alloc=True))


def test_noalloc_implicit_basis_takes_one_pass(api, ctx):
    # on the implicit basis the default spin layout builds device tables on
    # first use; the entry point that allocates nothing takes the one-pass
    # product instead, so it matches hphi_lanczos with spin_split = -1
    say("no-alloc lanczos: implicit basis")
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 16, 0), W.xxz_chain_j2(16))
    h.set_schedule(spin_implicit=1)
    got = api.lanczos(h, 60, seed=4, no_alloc=True)
    h.set_schedule(spin_split=-1)
    _same(api.lanczos(h, 60, seed=4), got)
    h.set_schedule(spin_split=3)
    auto = api.lanczos(h, 60, seed=4)
    assert abs(auto["energies"][0] - got["energies"][0]) < 1e-10


def test_noalloc_rejects_oversized_and_unsupported(api, ctx):
    from paper_2307_13222_amd import _lib as L
    say("no-alloc lanczos: limits")
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 26, 0), W.heisenberg_chain(26))   # 10.4e6 states
    with pytest.raises(api.HphiError) as e:
        api.lanczos(h, 10, seed=1, no_alloc=True)
    assert e.value.code == -1 and "static scratch" in str(e.value)
    h2 = api.Hamiltonian.spin(api.Basis.spin(ctx, 12, 0), W.heisenberg_chain(12))
    with pytest.raises(api.HphiError):
        api.lanczos(h2, 10, seed=1, use_graph=True, no_alloc=True)
    # still usable after the refusals
    _same(api.lanczos(h2, 40, seed=2), api.lanczos(h2, 40, seed=2, no_alloc=True))
    assert L.NOALLOC_SCRATCH_BYTES == 64 << 20
