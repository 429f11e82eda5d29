"""GPU: degenerate inputs through the C ABI against the oracle -- sectors with
one state, a full and an empty Hubbard species, the two-site singlet, the
S(q, w) excitation that vanishes (q = 0 in the S^z = 0 sector), a block of
one TPQ vector, a batched request on a one-state sector."""
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


def test_spin_fully_polarized_sector(api, ctx):
    # 2S^z = N: one state, every bond parallel: E = sum_b Jz_b / 4
    say("edge: polarized")
    m = W.random_heisenberg(6, "chain", 5)
    b = api.Basis.spin(ctx, 6, 6)
    assert b.dim == 1
    h = api.Hamiltonian.spin(b, m)
    v = np.array([0.7])
    w = host(h.mult(dev(v)))
    e = float(np.sum(m.jz)) / 4.0
    assert abs(w[0] - e * 0.7) < 1e-14
    s = O.basis_list(6, 6)
    assert abs(w[0] - O.spin_hv(m, s, v)[0]) < 1e-14
    r = api.lanczos(h, 10, seed=2)
    assert r["iterations"] == 1 and abs(r["energies"][0] - e) < 1e-14


def test_spin_two_site_singlet(api, ctx):
    say("edge: two sites")
    m = W._spin(2, [(0, 1)], [(1.0, 1.0)], "dimer")
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 2, 0), m)
    r = api.lanczos(h, 5, seed=1)
    assert abs(r["energies"][0] + 0.75) < 1e-14


def test_hubbard_full_and_empty_species(api, ctx):
    # all up orbitals filled, no down electrons: no hop is possible, no
    # double occupancy: H = 0 on the one state
    say("edge: hubbard full/empty")
    m = W.hubbard_chain(4, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 4, 4, 0)
    assert b.dim == 1
    h = api.Hamiltonian.hubbard(b, m)
    w = host(h.mult(dev(np.array([1.3]))))
    ups, dns = O.hubbard_basis(4, 4, 0)
    assert w[0] == 0.0 == O.hubbard_hv(m, ups, dns, np.array([1.3]))[0]
    # both species full: U on every site
    b2 = api.Basis.hubbard(ctx, 4, 4, 4)
    h2 = api.Hamiltonian.hubbard(b2, m)
    w2 = host(h2.mult(dev(np.array([0.5]))))
    assert abs(w2[0] - 4 * 4.0 * 0.5) < 1e-14


def test_hubbard_one_site(api, ctx):
    say("edge: hubbard one site")
    m = W.HubbardModel(1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0), np.array([3.0]), "site")
    b = api.Basis.hubbard(ctx, 1, 1, 1)
    h = api.Hamiltonian.hubbard(b, m)
    w = host(h.mult(dev(np.array([2.0]))))
    assert abs(w[0] - 6.0) < 1e-14


def test_sqw_vanishing_excitation(api, ctx):
    # q = 0 in the S^z = 0 sector: b = S^z_tot psi = 0, so D(z) = 0
    say("edge: sqw b = 0")
    m = W.heisenberg_chain(10)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 10, 0), m)
    r = api.lanczos(h, 80, seed=1, want_vector=True)
    bq = api.szq(h, 0.0, r["psi"])
    assert float(np.max(np.abs(host(bq)))) < 1e-12
    import torch
    zero = torch.zeros_like(bq)
    z = r["energies"][0] + np.linspace(0.0, 4.0, 8) + 0.05j
    d = api.sqw(h, zero, z, max_iter=50, tol=1e-8)
    assert d["converged"] and d["iterations"] == 0
    assert np.all(d["D"] == 0) and np.all(np.isfinite(d["residual"]))


def test_ctpq_single_vector(api, ctx):
    say("edge: ctpq one vector")
    m = W.heisenberg_chain(10)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 10, 0), m)
    s = O.basis_list(10, 5)
    phi0 = O.splitmix_complex_gaussian(77, len(s))[:, None]
    g = api.ctpq(h, 1, 6, 0.02, 10, storage="c128", phi0=dev(phi0))
    o = O.ctpq(lambda x: O.spin_hv(m, s, x), phi0, 6, 0.02, 10)
    assert np.max(np.abs(g["D"] - o["D"]) / np.abs(o["D"])) < 1e-12
    assert np.max(np.abs(g["E"] - o["E"])) < 1e-12


def test_batched_one_state_request(api, ctx):
    say("edge: batch one state")
    m = W.random_heisenberg(6, "chain", 3)
    h1 = api.Hamiltonian.spin(api.Basis.spin(ctx, 6, 6), m)
    h2 = api.Hamiltonian.spin(api.Basis.spin(ctx, 12, 0), W.heisenberg_chain(12))
    out = api.lanczos_batch([h1, h2], 100, [1, 2])
    assert out[0]["iterations"] == 1 and abs(out[0]["energy"] - float(np.sum(m.jz)) / 4.0) < 1e-14
    s = O.basis_list(12, 6)
    e_ref = np.linalg.eigvalsh(O.spin_sparse(W.heisenberg_chain(12), s).toarray())[0]
    assert abs(out[1]["energy"] - e_ref) < 1e-10


def test_ham_busy_on_another_stream(api, ctx):
    """A Hamiltonian serves one stream at a time: while products queued on
    one stream still run, a call on another stream returns HPHI_ERR_BUSY and
    launches nothing; on the same stream calls queue; after a
    synchronization the other stream may take it."""
    import torch
    from paper_2307_13222_amd import _lib as L
    say("edge: busy guard")
    m = W.hubbard_square(4, 4, 1.0, 4.0)
    b = api.Basis.hubbard(ctx, 16, 6, 6)
    h = api.Hamiltonian.hubbard(b, m)
    v = torch.rand(b.dim, dtype=torch.float64, device="cuda")
    w = torch.empty_like(v)
    w2 = torch.zeros_like(v)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(8):   # about 10 ms of products in flight on s1
        h.mult(v, w, stream=s1)
    with pytest.raises(api.HphiError) as e:
        h.mult(v, w2, stream=s2)
    assert e.value.code == L.ERR_BUSY
    h.mult(v, w, stream=s1)            # same stream: fine
    s1.synchronize()
    h.mult(v, w2, stream=s2)           # drained: the other stream may use it
    s2.synchronize()
    assert torch.equal(w, w2)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_spin_gc_tiny_spaces(api, ctx, n):
    # fewer sites than the four low bits of a window tile: one tile holds
    # the whole space; one site is a spin in a field, E0 = -|h|/2
    say("spin gc tiny", n)
    m = W.random_spin_gc(max(n, 2), "chain", 40 + n) if n > 1 else W.spin_gc(1, np.zeros((0, 2)), 0, 0, 0, 0.6, 0.8)
    if n == 1:
        h = api.Hamiltonian.spin_gc(api.Basis.spin_gc(ctx, 1), m)
        w = host(h.mult(dev(np.array([1.0, 0.0]))))
        assert np.allclose(w, O.spin_gc_hv(m, np.array([1.0, 0.0])), atol=1e-15)
        r = api.lanczos(h, 2, seed=1)
        assert abs(r["energies"][0] + 0.5) < 1e-14
        return
    m = W.random_spin_gc(n, "chain", 40 + n)
    h = api.Hamiltonian.spin_gc(api.Basis.spin_gc(ctx, n), m)
    v = W.random_vector(1 << n, n)
    assert np.allclose(host(h.mult(dev(v))), O.spin_gc_hv(m, v), atol=1e-13)


@pytest.mark.parametrize("n,two_s,two_sz", [(1, 2, 0), (1, 3, 3), (2, 2, -4), (2, 3, 2), (3, 2, 6)])
def test_spin_s_tiny_sectors(api, ctx, n, two_s, two_sz):
    # one-site and fully polarized sectors (one state), two sites
    say("spin-S tiny", n, two_s, two_sz)
    pairs = W.chain_pairs(n) if n > 2 else ([(0, 1)] if n == 2 else np.zeros((0, 2)))
    m = W.spin_s_model(n, two_s, pairs, 0.9, 1.1, hz=0.3, d_ion=0.2)
    b = api.Basis.spin_s(ctx, n, two_s, two_sz)
    s = O.spin_s_basis(n, two_s, two_sz)
    assert b.dim == len(s)
    h = api.Hamiltonian.spin_s(b, m)
    v = W.random_vector(len(s), n + two_s)
    assert np.allclose(host(h.mult(dev(v))), O.spin_s_hv(m, s, v), atol=1e-13)
