"""GPU: resuming a run from its saved state. cTPQ restarted from the states
a first run returns continues the sequence of a single longer run (D_k,
<H>, <H^2> to rounding); real-time evolution split in two calls equals one
call bit for bit."""
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


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("storage,tol", [("c128", 1e-12), ("c64", 1e-5)])
def test_ctpq_resume_from_saved_states(api, ctx, storage, tol):
    say("ctpq resume", storage)
    m = W.xxz_chain_j2(16)
    b = api.Basis.spin(ctx, 16, 0)
    h = api.Hamiltonian.spin(b, m)
    full = api.ctpq(h, 4, 6, 0.05, 12, storage=storage, seed=5)
    first = api.ctpq(h, 4, 6, 0.05, 6, storage=storage, seed=5)
    second = api.ctpq(h, 4, 6, 0.05, 6, storage=storage, phi0=first["phi"].clone())
    # the first half is the same run (its last record takes the final-step path)
    assert np.max(np.abs(first["D"] - full["D"][:7])) < 1e-13 * np.max(np.abs(full["D"][:7]))
    assert np.max(np.abs(first["E"] - full["E"][:7])) < tol * max(1.0, np.max(np.abs(full["E"])))
    # the resumed half: D_0 of the restart is the saved states' squared norm (1)
    assert np.max(np.abs(second["D"][0] - 1.0)) < tol
    assert np.max(np.abs(second["D"][1:] - full["D"][7:])) < tol * np.max(np.abs(full["D"][7:]))
    assert np.max(np.abs(second["E"] - full["E"][6:])) < tol * max(1.0, np.max(np.abs(full["E"])))
    assert np.max(np.abs(second["E2"] - full["E2"][6:])) < tol * max(1.0, np.max(np.abs(full["E2"])))
    ph_full = host(full["phi"]).astype(np.complex128)
    ph_res = host(second["phi"]).astype(np.complex128)
    assert np.max(np.abs(ph_full - ph_res)) < 10 * tol * np.max(np.abs(ph_full))


def test_time_evolution_split_equals_single_run(api, ctx):
    import torch
    say("tevol split")
    m = W.heisenberg_chain(14)
    b = api.Basis.spin(ctx, 14, 0)
    h = api.Hamiltonian.spin(b, m)
    psi0 = torch.from_numpy(W.random_vector(b.dim, 4, np.complex128, nvec=2)).cuda()
    a = psi0.clone()
    ga = api.time_evolve(h, a, 10, dt=0.03, n_max=8)
    c = psi0.clone()
    api.time_evolve(h, c, 4, dt=0.03, n_max=8)
    gc = api.time_evolve(h, c, 6, dt=0.03, n_max=8)
    assert torch.equal(a, c)
    assert np.max(np.abs(ga["energy"][4:] - gc["energy"])) < 1e-13
