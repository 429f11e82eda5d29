"""GPU: complex transfer amplitudes (t c+_i c_j + t* c+_j c_i: fluxes and
Peierls phases) against the oracle. Products in complex128 and complex64
on random complex hops with two-body terms (row in LDS) and on the 16-site
ring with a flux (row beyond LDS, sampled rows); frames of a light pulse,
switched one by one and stepped through by the Taylor evolution; the
real-vector methods refused."""
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


def random_complex_model(n, seed):
    rng = np.random.default_rng(seed)
    m = W.hubbard_chain(n, 1.0, 3.0)
    m = W.with_pair_terms(m, np.stack([m.hi, m.hj], axis=1), 0.6, 0.2, 0.15, 0.1)
    extra = np.array([[0, 3], [2, 7], [1, 5]], dtype=np.int32)
    hi = np.concatenate([m.hi, extra[:, 0]])
    hj = np.concatenate([m.hj, extra[:, 1]])
    t = rng.uniform(0.3, 1.2, size=len(hi))
    t_im = rng.normal(size=len(hi)) * 0.7
    return W.HubbardModel(n, hi, hj, t, rng.normal(size=n) + 2.0, "cplx", m.site_x,
                          m.pi, m.pj, m.pv, m.pjh, m.pjx, m.pjp, t_im)


@pytest.mark.parametrize("nu,nd", [(5, 4), (3, 6)])
def test_complex_products_match_oracle(api, ctx, nu, nd):
    import torch
    say("complex hops mult", nu, nd)
    n = 10
    m = random_complex_model(n, 4)
    b = api.Basis.hubbard(ctx, n, nu, nd)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(n, nu, nd)
    v = W.random_vector(b.dim, 7, np.complex128)
    ref = O.hubbard_hv(m, ups, dns, v)
    w = host(h.mult(dev(v)))
    assert relmax(w, ref) < 1e-12
    w32 = host(h.mult(dev(v.astype(np.complex64))))
    assert relmax(w32.astype(np.complex128), ref) < 2e-6
    # real vectors are refused, and so are the real-vector methods
    with pytest.raises(api.HphiError):
        h.mult(dev(W.random_vector(b.dim, 1)))
    with pytest.raises(api.HphiError):
        api.lanczos(h, 10, seed=1)


def test_flux_ring_16_sites_sampled_rows(api, ctx):
    # the 16-site half-filled ring threaded by a flux: complex FP64 rows of
    # 12870 elements (beyond LDS), sampled rows against the oracle
    import torch
    say("complex hops 16-site ring")
    m = W.with_flux(W.hubbard_chain(16, 1.0, 8.0), 0.9)
    b = api.Basis.hubbard(ctx, 16, 8, 8)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(16, 8, 8)
    g = torch.Generator(device="cuda").manual_seed(8)
    v = torch.complex(torch.rand(b.dim, dtype=torch.float64, device="cuda", generator=g) - 0.5,
                      torch.rand(b.dim, dtype=torch.float64, device="cuda", generator=g) - 0.5)
    w = h.mult(v)
    rng = np.random.default_rng(12)
    rows = np.concatenate([[0, b.dim - 1], rng.integers(0, b.dim, 600)])
    wmax = float(w.abs().max())
    errs = []
    for r in rows:
        cols, vals = O.hubbard_row(m, ups, dns, int(r) // 12870, int(r) % 12870)
        vv = host(v[torch.from_numpy(cols).cuda()])
        errs.append(abs(complex(w[int(r)]) - complex(np.dot(vals, vv))))
    assert max(errs) / wmax < 1e-12
    del v, w


def pulse_case(n):
    m = W.hubbard_chain(n, 1.0, 4.0)
    return m, W.peierls_pulse(m, 1.2, 4.0, 0.2, 0.08, 0.02, 21)


def test_pulse_frames_products(api, ctx):
    say("pulse frames mult")
    n = 10
    m, fr = pulse_case(n)
    b = api.Basis.hubbard(ctx, n, 5, 5)
    h = api.Hamiltonian.hubbard(b, m, frames=fr)
    ups, dns = O.hubbard_basis(n, 5, 5)
    v = W.random_vector(b.dim, 9, np.complex128)
    vd = dev(v)
    for k in [0, 10, 13, 20, 0]:
        h.set_frame(k)
        w = host(h.mult(vd))
        assert relmax(w, O.hubbard_hv(W.model_at_frame(m, fr, k), ups, dns, v)) < 1e-12, k


@pytest.mark.parametrize("storage", ["c128", "c64"])
def test_pulse_evolution_matches_oracle(api, ctx, storage):
    say("pulse evolution", storage)
    n = 8
    m, fr = pulse_case(n)
    ups, dns = O.hubbard_basis(n, 4, 4)
    ev, vec = scipy.sparse.linalg.eigsh(O.hubbard_sparse(m, ups, dns), k=1, which="SA")
    psi0 = vec[:, 0].astype(np.complex128)
    h = api.Hamiltonian.hubbard(api.Basis.hubbard(ctx, n, 4, 4), m, frames=fr)
    psi = dev(psi0 if storage == "c128" else psi0.astype(np.complex64))
    g = api.time_evolve(h, psi, 20, dt=0.02, n_max=10, double_occupancy=True)
    mats = {}

    def hv_at(k):
        if k not in mats:
            mats[k] = O.hubbard_sparse(W.model_at_frame(m, fr, k), ups, dns)
        return lambda x: mats[k] @ x
    wt = O.hubbard_double_occupancy_weight(ups, dns, n)
    o = O.taylor_evolve_td(hv_at, psi0, 10, 0.02, 20, weight=wt)
    tol = 1e-10 if storage == "c128" else 2e-5
    assert relmax(host(psi).astype(np.complex128), o["psi"][:, 0]) < tol
    assert np.max(np.abs(g["energy"][:, 0] - o["energy"][:, 0])) < (1e-10 if storage == "c128" else 1e-4)
    assert np.max(np.abs(g["double_occupancy"] - o["obs"][:, 0])) < (1e-11 if storage == "c128" else 1e-5)
    # the pulse does work: the energy moves off its starting value
    assert np.ptp(o["energy"][:, 0]) > 1e-2


def test_complex_refusals(api, ctx):
    say("complex refusals")
    m = W.with_flux(W.hubbard_chain(6, 1.0, 2.0), 0.5)
    b = api.Basis.hubbard(ctx, 6, 3, 3)
    h = api.Hamiltonian.hubbard(b, m)
    psi = dev(W.random_vector(b.dim, 2, np.complex128))
    with pytest.raises(api.HphiError):
        api.sqw(h, psi, np.array([0.5 + 0.05j]))
    # a complex-free model built through the same path stays real
    h2 = api.Hamiltonian.hubbard(b, W.hubbard_chain(6, 1.0, 2.0),
                                 frames=W.HubbardFrames(1, hop_t_im=np.zeros((1, 6))))
    r = api.lanczos(h2, 30, seed=1)
    assert np.isfinite(r["energies"][0])


def embed_real(H):
    """The complex Hermitian H as the real symmetric matrix acting on
    interleaved (re, im) coordinates: [[Re H, -Im H], [Im H, Re H]]."""
    import scipy.sparse as sp
    Hc = sp.coo_matrix(H)
    r, c, v = Hc.row, Hc.col, Hc.data
    rows = np.concatenate([2 * r, 2 * r, 2 * r + 1, 2 * r + 1])
    cols = np.concatenate([2 * c, 2 * c + 1, 2 * c, 2 * c + 1])
    vals = np.concatenate([v.real, -v.imag, v.imag, v.real])
    n = 2 * H.shape[0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


@pytest.mark.parametrize("storage", ["c128", "c64"])
def test_complex_lanczos_flux_ring(api, ctx, storage):
    # complex-vector Lanczos on a Hermitian H with complex transfers: the
    # same recurrence as a real Lanczos of the real embedding on the
    # interleaved start vector (SplitMix64 uniform over 2 dim reals)
    say("complex lanczos", storage)
    n, nu, nd = 10, 5, 4
    m = W.with_flux(W.hubbard_chain(n, 1.0, 4.0), 1.3)
    b = api.Basis.hubbard(ctx, n, nu, nd)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(n, nu, nd)
    H = O.hubbard_sparse(m, ups, dns)
    e_ref = scipy.sparse.linalg.eigsh(H, k=1, which="SA")[0][0]
    r = api.lanczos(h, 250, seed=3, storage=storage, want_vector=True)
    tol = 1e-10 if storage == "c128" else 1e-5
    assert abs(r["energies"][0] - e_ref) < tol * max(1.0, abs(e_ref))
    psi = host(r["psi"]).astype(np.complex128)
    assert abs(np.linalg.norm(psi) - 1.0) < (1e-12 if storage == "c128" else 1e-5)
    res = np.linalg.norm(H @ psi - r["energies"][0] * psi)
    assert res < (1e-5 if storage == "c128" else 1e-2)
    if storage == "c128":
        Hr = embed_real(H)
        o = O.lanczos(lambda x: Hr @ x, O.splitmix_uniform(3, 0, 2 * b.dim), 20)
        assert np.max(np.abs(r["alpha"][:20] - o["alpha"][:20])) < 1e-10
        assert np.max(np.abs(r["beta"][1:20] - o["beta"][1:20])) < 1e-10
    with pytest.raises(api.HphiError):
        api.lanczos(h, 10, seed=3, storage="c128", refine=True)


@pytest.mark.parametrize("dt,tol", [("c128", 1e-11), ("c64", 2e-5)])
def test_complex_transfers_ctpq_matches_oracle(api, ctx, dt, tol):
    import torch
    say("complex hops ctpq", dt)
    m = W.with_flux(W.hubbard_square(3, 3, 1.0, 6.0), 0.8)
    b = api.Basis.hubbard(ctx, 9, 4, 5)
    h = api.Hamiltonian.hubbard(b, m)
    ups, dns = O.hubbard_basis(9, 4, 5)
    phi0 = O.splitmix_complex_gaussian(78, b.dim)[:, None]
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    g = api.ctpq(h, 1, 6, 0.02, 20, storage=dt, phi0=dev(phi0).to(tdt))
    phi_in = host(dev(phi0).to(tdt)).astype(np.complex128)
    H = O.hubbard_sparse(m, ups, dns)
    o = O.ctpq(lambda x: H @ x, phi_in, 6, 0.02, 20)
    assert relmax(g["D"], o["D"]) < tol
    assert relmax(g["E"], o["E"]) < tol
    assert relmax(g["E2"], o["E2"]) < tol
