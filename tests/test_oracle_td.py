"""Pins of the oracle's time-dependent evolution (Sec. 3.4, H(t) with
t_ij(t) and two-body I(t), held over each step): a Hamiltonian that only
scales in time, H(t) = f(t) H_0, against the closed form exp(-i Theta H_0),
Theta = dt sum f(t_k); non-commuting frames against the ordered product of
dense exponentials exp(-i H_k dt); the energy change of an interaction ramp
against the work (U_k+1 - U_k) N_s <D>; frame selection and clamping."""
import numpy as np
import scipy.linalg

from oracle import core as O
from paper_2307_13222_amd import workloads as W


def small_model(n=5, u=3.0):
    m = W.hubbard_chain(n, 1.0, u)
    return W.with_pair_terms(m, np.stack([m.hi, m.hj], axis=1), 0.7, 0.3, 0.2, 0.1)


def frame_matrices(m, fr, ups, dns):
    return [O.hubbard_sparse(W.model_at_frame(m, fr, f), ups, dns).toarray() for f in range(fr.n_frames)]


def start_state(dim, seed):
    rng = np.random.default_rng(seed)
    psi = rng.normal(size=dim) + 1j * rng.normal(size=dim)
    return psi / np.linalg.norm(psi)


def test_scaled_hamiltonian_closed_form():
    # every amplitude (t, U, V, J_H, J_X, J_P) times f_k: H_k = f_k H_0, all
    # frames commute, psi(t_K) = exp(-i Theta H_0) psi(0)
    m = small_model()
    ups, dns = O.hubbard_basis(5, 2, 2)
    H0 = O.hubbard_sparse(m, ups, dns).toarray()
    n_steps, dt = 30, 0.02
    f = 1.0 + 0.8 * np.sin(0.7 * np.arange(n_steps + 1))
    base_p = np.stack([m.pv, m.pjh, m.pjx, m.pjp], axis=1)
    fr = W.HubbardFrames(n_steps + 1, hop_t=f[:, None] * m.t[None, :], u_site=f[:, None] * m.u_site[None, :],
                         pair_v=f[:, None, None] * base_p[None])
    mats = frame_matrices(m, fr, ups, dns)
    psi0 = start_state(len(H0), 1)
    o = O.taylor_evolve_td(lambda k: (lambda x: mats[k] @ x), psi0, 12, dt, n_steps)
    ev, U = np.linalg.eigh(H0)
    theta = dt * np.sum(f[:n_steps])
    exact = U @ (np.exp(-1j * ev * theta) * (U.conj().T @ psi0))
    assert np.max(np.abs(o["psi"][:, 0] - exact)) < 1e-11
    e0 = float(np.real(np.vdot(psi0, H0 @ psi0)))
    assert np.max(np.abs(o["energy"][:, 0] - f * e0)) < 1e-11
    assert np.max(np.abs(o["norm"][:, 0] - 1.0)) < 1e-12


def test_non_commuting_frames_match_ordered_exponentials():
    m = small_model()
    ups, dns = O.hubbard_basis(5, 3, 2)
    fr = W.random_frames(m, 13, 4, repeat=2)
    mats = frame_matrices(m, fr, ups, dns)
    # the frames do not commute: the order of the factors matters
    assert np.max(np.abs(mats[0] @ mats[2] - mats[2] @ mats[0])) > 1e-2
    n_steps, dt = 12, 0.05
    psi0 = start_state(len(mats[0]), 2)
    o = O.taylor_evolve_td(lambda k: (lambda x: mats[k] @ x), psi0, 16, dt, n_steps)
    psi = psi0.copy()
    for k in range(n_steps + 1):
        e = float(np.real(np.vdot(psi, mats[k] @ psi)) / np.real(np.vdot(psi, psi)))
        assert abs(o["energy"][k, 0] - e) < 1e-10
        if k < n_steps:
            psi = scipy.linalg.expm(-1j * dt * mats[k]) @ psi
    assert np.max(np.abs(o["psi"][:, 0] - psi)) < 1e-10


def test_interaction_ramp_energy_change_is_work():
    # exact evolution under H_k conserves <H_k>, so the recorded energies
    # step by <H_k+1 - H_k> = (U_k+1 - U_k) N_s <D>(t_k+1), D the double
    # occupancy per site
    n = 6
    m = W.hubbard_chain(n, 1.0, 0.0)
    ups, dns = O.hubbard_basis(n, 3, 3)
    fr = W.interaction_ramp(m, 0.0, 8.0, 10, 16)
    mats = frame_matrices(m, fr, ups, dns)
    ev, vec = np.linalg.eigh(mats[0])
    psi0 = vec[:, 0].astype(np.complex128)
    wt = O.hubbard_double_occupancy_weight(ups, dns, n)
    o = O.taylor_evolve_td(lambda k: (lambda x: mats[k] @ x), psi0, 14, 0.02, 15, weight=wt)
    u = fr.u_site[:, 0]
    de = np.diff(o["energy"][:, 0])
    work = np.diff(u) * n * o["obs"][1:, 0]
    assert np.max(np.abs(de - work)) < 1e-11
    # the ramp does work: the energy rises while U does, then stays
    assert np.all(de[:10] > 0) and np.max(np.abs(de[10:])) < 1e-11


def test_frames_clamp_and_keep_unset_kinds():
    m = small_model(4)
    fr = W.HubbardFrames(3, u_site=np.arange(12, dtype=np.float64).reshape(3, 4))
    for k, f in [(0, 0), (2, 2), (7, 2)]:
        mk = W.model_at_frame(m, fr, k)
        assert np.array_equal(mk.u_site, fr.u_site[f])
        assert np.array_equal(mk.t, m.t) and np.array_equal(mk.pv, m.pv) and np.array_equal(mk.pjp, m.pjp)
    # held past the last frame: the evolution after it is the fixed-H one
    ups, dns = O.hubbard_basis(4, 2, 2)
    fr2 = W.random_frames(m, 3, 5, repeat=1)
    mats = frame_matrices(m, fr2, ups, dns)
    psi0 = start_state(len(mats[0]), 3)
    o = O.taylor_evolve_td(lambda k: (lambda x: mats[min(k, 2)] @ x), psi0, 14, 0.03, 8)
    mid = O.taylor_evolve_td(lambda k: (lambda x: mats[k] @ x), psi0, 14, 0.03, 2)
    rest = O.taylor_evolve(lambda x: mats[2] @ x, mid["psi"][:, 0], 14, 0.03, 6)
    assert np.max(np.abs(o["psi"][:, 0] - rest["psi"][:, 0])) < 1e-13
