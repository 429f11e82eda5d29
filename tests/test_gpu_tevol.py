"""GPU: real-time evolution (truncated Taylor series) against the oracle --
the interaction quench of a half-filled Hubbard ring (ground state of U = 0
evolved with U = 8: norm, energy and double occupancy at every step, final
state), a block of two spin vectors, and complex64 storage."""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg

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


@pytest.fixture(scope="module")
def quench():
    n = 10
    ups, dns = O.hubbard_basis(n, 5, 5)
    m0 = W.hubbard_chain(n, 1.0, 0.0)
    ev, vec = scipy.sparse.linalg.eigsh(O.hubbard_sparse(m0, ups, dns), k=1, which="SA")
    psi0 = vec[:, 0].astype(np.complex128)
    return n, ups, dns, psi0


def test_hubbard_quench_matches_oracle(api, ctx, quench):
    say("tevol quench")
    n, ups, dns, psi0 = quench
    m = W.hubbard_chain(n, 1.0, 8.0)
    h = api.Hamiltonian.hubbard(api.Basis.hubbard(ctx, n, 5, 5), m)
    psi = dev(psi0)
    g = api.time_evolve(h, psi, 50, dt=0.01, n_max=10, double_occupancy=True)
    wgt = O.hubbard_double_occupancy_weight(ups, dns, n)
    o = O.taylor_evolve(lambda x: O.hubbard_hv(m, ups, dns, x), psi0, 10, 0.01, 50, weight=wgt)
    assert np.max(np.abs(g["norm"][:, 0] - o["norm"][:, 0])) < 1e-12
    assert np.max(np.abs(g["energy"][:, 0] - o["energy"][:, 0])) < 1e-10
    assert np.max(np.abs(g["double_occupancy"] - o["obs"][:, 0])) < 1e-12
    assert relmax(host(psi), o["psi"][:, 0]) < 1e-11
    # the checks of the paper's example: unit norm and a conserved energy
    assert np.max(np.abs(g["norm"] - 1.0)) < 1e-12
    assert np.max(np.abs(g["energy"] - g["energy"][0])) < 1e-10
    # U = 0 ground state at half filling: double occupancy starts at 1/4
    assert abs(g["double_occupancy"][0] - 0.25) < 1e-12


def test_spin_block_matches_oracle(api, ctx):
    say("tevol spin block")
    m = W.random_heisenberg(12, "ladder", 8)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 12, 0), m)
    s = O.basis_list(12, 6)
    phi0 = np.stack([O.splitmix_complex_gaussian(300 + j, len(s)) for j in range(2)], axis=1)
    psi = dev(phi0)
    g = api.time_evolve(h, psi, 20, dt=0.02, n_max=8)
    o = O.taylor_evolve(lambda x: O.spin_hv(m, s, x), phi0, 8, 0.02, 20)
    assert np.max(np.abs(g["norm"] - o["norm"]) / o["norm"]) < 1e-12
    assert np.max(np.abs(g["energy"] - o["energy"])) < 1e-10
    assert relmax(host(psi), o["psi"]) < 1e-11


def test_complex64_storage(api, ctx, quench):
    import torch
    say("tevol c64")
    n, ups, dns, psi0 = quench
    m = W.hubbard_chain(n, 1.0, 8.0)
    h = api.Hamiltonian.hubbard(api.Basis.hubbard(ctx, n, 5, 5), m)
    psi = dev(psi0).to(torch.complex64)
    g = api.time_evolve(h, psi, 20, dt=0.01, n_max=10, double_occupancy=True)
    wgt = O.hubbard_double_occupancy_weight(ups, dns, n)
    o = O.taylor_evolve(lambda x: O.hubbard_hv(m, ups, dns, x), psi0, 10, 0.01, 20, weight=wgt)
    assert np.max(np.abs(g["energy"][:, 0] - o["energy"][:, 0])) < 1e-5
    assert np.max(np.abs(g["double_occupancy"] - o["obs"][:, 0])) < 1e-6
    assert relmax(host(psi).astype(np.complex128), o["psi"][:, 0]) < 1e-5


def test_invalid_options(api, ctx):
    import torch
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 8, 0), W.heisenberg_chain(8))
    psi = torch.zeros(70, dtype=torch.complex128, device="cuda")
    with pytest.raises(api.HphiError):
        api.time_evolve(h, psi, 5, dt=0.0)
    with pytest.raises(api.HphiError):
        api.time_evolve(h, psi, 5, n_max=0)
    with pytest.raises(api.HphiError):
        api.time_evolve(h, psi, 5, double_occupancy=True)
