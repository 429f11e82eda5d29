"""Seeded synthetic inputs shared by the library's callers and by the tests.

This module holds lattice geometry, coupling draws and seeded random test
vectors only; it contains none of the Hamiltonian, basis or solver
arithmetic. Both the HIP path (through its Python binding) and the oracle are
fed from here, so the two sides see identical inputs.

Lattices follow the Standard-mode lattice keywords of the HPhi update paper
(Sec. 4.1, Table "Keywords": Chain, Ladder, Square), with periodic boundaries.
Site numbering: chain s = x; 2-leg ladder s = x + L*leg (rung coordinate
x = s mod L); square s = x + Lx*y.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class SpinModel:
    """Spin-1/2 XXZ couplings: H = sum_b Jz_b Sz_i Sz_j + Jxy_b (Sx Sx + Sy Sy)
    - sum_i hz_i Sz_i. Bond lists are literal (a repeated pair adds)."""
    n_sites: int
    bi: np.ndarray
    bj: np.ndarray
    jz: np.ndarray
    jxy: np.ndarray
    hz: Optional[np.ndarray] = None
    site_x: Optional[np.ndarray] = None   # coordinate used for S^z(q) phases
    name: str = ""

    @property
    def n_bonds(self) -> int:
        return int(self.bi.shape[0])


@dataclass
class HubbardModel:
    """H = -sum_h sum_sigma (t_h c+_i c_j + t_h* c+_j c_i) + sum_i U_i n_up n_dn
    (t_h = t + i t_im; real unless t_im is given), plus
    the optional two-body terms of Eq. ham_general (Sec. 5) per site pair
    p = (pi, pj): inter-site Coulomb pv n_i n_j, Hund -pjh (n_i,up n_j,up +
    n_i,dn n_j,dn), exchange pjx (c+_i,up c_j,up c+_j,dn c_i,dn + h.c.) and
    pair hopping pjp (c+_i,up c_j,up c+_i,dn c_j,dn + h.c.)."""
    n_sites: int
    hi: np.ndarray
    hj: np.ndarray
    t: np.ndarray
    u_site: np.ndarray
    name: str = ""
    site_x: Optional[np.ndarray] = None   # coordinate used for S^z(q) phases
    pi: Optional[np.ndarray] = None
    pj: Optional[np.ndarray] = None
    pv: Optional[np.ndarray] = None
    pjh: Optional[np.ndarray] = None
    pjx: Optional[np.ndarray] = None
    pjp: Optional[np.ndarray] = None
    t_im: Optional[np.ndarray] = None       # imaginary parts of the transfers (None: real)

    @property
    def n_hops(self) -> int:
        return int(self.hi.shape[0])

    @property
    def n_pairs(self) -> int:
        return 0 if self.pi is None else int(self.pi.shape[0])


@dataclass
class SpinSModel:
    """Spin-S Heisenberg model (keyword 2S, Sec. 4.1): H = sum_b [jz S^z_i S^z_j
    + jxy (S^x_i S^x_j + S^y_i S^y_j)] - sum_i hz_i S^z_i + sum_i d_i (S^z_i)^2."""
    n_sites: int
    two_s: int
    bi: np.ndarray
    bj: np.ndarray
    jz: np.ndarray
    jxy: np.ndarray
    hz: Optional[np.ndarray] = None
    d_ion: Optional[np.ndarray] = None
    site_x: Optional[np.ndarray] = None
    name: str = ""

    @property
    def n_bonds(self) -> int:
        return int(self.bi.shape[0])


def spin_s_model(n: int, two_s: int, pairs, jz, jxy, hz=None, d_ion=None, name: str = "") -> SpinSModel:
    p = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    k = len(p)
    bonds = lambda x: np.broadcast_to(np.asarray(x, dtype=np.float64), (k,)).copy()
    sites = lambda x: None if x is None else np.broadcast_to(np.asarray(x, dtype=np.float64), (n,)).copy()
    return SpinSModel(n, two_s, p[:, 0].copy(), p[:, 1].copy(), bonds(jz), bonds(jxy), sites(hz), sites(d_ion),
                      np.arange(n, dtype=np.int64), name)


def random_spin_s(n: int, two_s: int, lattice: str, seed: int) -> SpinSModel:
    """XXZ couplings in [0.5, 1.5), fields and single-ion terms from N(0, 1)."""
    rng = np.random.default_rng(seed)
    pairs = chain_pairs(n) if lattice == "chain" else ladder_pairs(n)
    k = len(pairs)
    return spin_s_model(n, two_s, pairs, rng.uniform(0.5, 1.5, k), rng.uniform(0.5, 1.5, k),
                        rng.normal(size=n), rng.normal(size=n), f"random_spin{two_s}_{lattice}_{n}")


@dataclass
class SpinGCModel:
    """Spin-1/2 model without S^z conservation (SpinGC keyword, Sec. 4.1):
    H = sum_b (jx S^x_i S^x_j + jy S^y_i S^y_j + jz S^z_i S^z_j)
        - sum_i (hx_i S^x_i + hz_i S^z_i)."""
    n_sites: int
    bi: np.ndarray
    bj: np.ndarray
    jx: np.ndarray
    jy: np.ndarray
    jz: np.ndarray
    hx: np.ndarray
    hz: np.ndarray
    name: str = ""

    @property
    def n_bonds(self) -> int:
        return int(self.bi.shape[0])


def spin_gc(n: int, pairs, jx, jy, jz, hx=0.0, hz=0.0, name: str = "") -> SpinGCModel:
    p = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    k = len(p)
    bonds = lambda x: np.broadcast_to(np.asarray(x, dtype=np.float64), (k,)).copy()
    sites = lambda x: np.broadcast_to(np.asarray(x, dtype=np.float64), (n,)).copy()
    return SpinGCModel(n, p[:, 0].copy(), p[:, 1].copy(), bonds(jx), bonds(jy), bonds(jz), sites(hx), sites(hz),
                       name)


def tfim_chain(n: int, j: float = 1.0, g: float = 1.0) -> SpinGCModel:
    """Transverse-field Ising ring -J sum sigma^z sigma^z - g sum sigma^x,
    written in spin operators (sigma = 2 S): jz = -4 J, hx = 2 g."""
    return spin_gc(n, chain_pairs(n), 0.0, 0.0, -4.0 * j, 2.0 * g, 0.0, f"tfim_chain_{n}")


def random_spin_gc(n: int, lattice: str, seed: int) -> SpinGCModel:
    """XYZ couplings and both fields drawn from N(0, 1) on a chain or ladder."""
    rng = np.random.default_rng(seed)
    pairs = chain_pairs(n) if lattice == "chain" else ladder_pairs(n)
    k = len(pairs)
    return spin_gc(n, pairs, rng.normal(size=k), rng.normal(size=k), rng.normal(size=k),
                   rng.normal(size=n), rng.normal(size=n), f"random_gc_{lattice}_{n}")


def _spin(n, pairs, couplings, name, site_x=None, hz=None) -> SpinModel:
    pairs = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    c = np.asarray(couplings, dtype=np.float64).reshape(-1, 2)
    if site_x is None:
        site_x = np.arange(n, dtype=np.int64)
    return SpinModel(n, pairs[:, 0].copy(), pairs[:, 1].copy(), c[:, 0].copy(),
                     c[:, 1].copy(), None if hz is None else np.asarray(hz, np.float64),
                     np.asarray(site_x, dtype=np.int64), name)


def chain_pairs(n: int, dist: int = 1) -> List[Tuple[int, int]]:
    return [(s, (s + dist) % n) for s in range(n)]


def ladder_pairs(n: int) -> List[Tuple[int, int]]:
    """2-leg ladder with n sites (n even): legs periodic along x, rungs."""
    if n % 2:
        raise ValueError("a 2-leg ladder needs an even site count")
    L = n // 2
    pairs = []
    for leg in range(2):
        for x in range(L):
            pairs.append((x + L * leg, (x + 1) % L + L * leg))
    for x in range(L):
        pairs.append((x, x + L))
    return pairs


def square_pairs(lx: int, ly: int, diagonal: bool = False) -> List[Tuple[int, int]]:
    """Nearest-neighbour bonds (s, s+x), (s, s+y); with diagonal=True the
    next-nearest (s, s+x+y), (s, s+x-y). Periodic in both directions."""
    pairs = []
    for y in range(ly):
        for x in range(lx):
            s = x + lx * y
            if not diagonal:
                pairs.append((s, (x + 1) % lx + lx * y))
                pairs.append((s, x + lx * ((y + 1) % ly)))
            else:
                pairs.append((s, (x + 1) % lx + lx * ((y + 1) % ly)))
                pairs.append((s, (x + 1) % lx + lx * ((y - 1) % ly)))
    return pairs


def heisenberg_chain(n: int, j: float = 1.0) -> SpinModel:
    p = chain_pairs(n)
    return _spin(n, p, [(j, j)] * len(p), f"heisenberg_chain_{n}")


def xxz_chain_j2(n: int, j1=(1.0, 0.8), j2=(0.5, 0.4)) -> SpinModel:
    """XXZ chain with nearest (Jz, Jxy) = j1 and next-nearest j2 bonds."""
    p1, p2 = chain_pairs(n, 1), chain_pairs(n, 2)
    return _spin(n, p1 + p2, [j1] * len(p1) + [j2] * len(p2), f"xxz_j2_chain_{n}")


def j1j2_square(lx: int, ly: int, j1: float = 1.0, j2: float = 0.5) -> SpinModel:
    p1 = square_pairs(lx, ly, False)
    p2 = square_pairs(lx, ly, True)
    n = lx * ly
    return _spin(n, p1 + p2, [(j1, j1)] * len(p1) + [(j2, j2)] * len(p2),
                 f"j1j2_square_{lx}x{ly}", site_x=np.arange(n) % lx)


def random_heisenberg(n: int, lattice: str, seed: int, lo: float = 0.5,
                      hi: float = 1.5) -> SpinModel:
    """Heisenberg chain or 2-leg ladder, J_b ~ U[lo, hi] per bond (seeded)."""
    if lattice == "chain":
        p, site_x = chain_pairs(n), np.arange(n)
    elif lattice == "ladder":
        p, site_x = ladder_pairs(n), np.arange(n) % (n // 2)
    else:
        raise ValueError(lattice)
    rng = np.random.default_rng(seed)
    j = rng.uniform(lo, hi, size=len(p))
    return _spin(n, p, np.stack([j, j], axis=1), f"rand_{lattice}_{n}_s{seed}",
                 site_x=site_x)


def hubbard_square(lx: int, ly: int, t: float = 1.0, u: float = 4.0) -> HubbardModel:
    p = np.asarray(square_pairs(lx, ly, False), dtype=np.int32)
    n = lx * ly
    return HubbardModel(n, p[:, 0].copy(), p[:, 1].copy(), np.full(len(p), t),
                        np.full(n, u, dtype=np.float64), f"hubbard_square_{lx}x{ly}",
                        np.arange(n, dtype=np.int64) % lx)


def hubbard_chain(n: int, t: float = 1.0, u: float = 4.0) -> HubbardModel:
    p = np.asarray(chain_pairs(n), dtype=np.int32)
    return HubbardModel(n, p[:, 0].copy(), p[:, 1].copy(), np.full(len(p), t),
                        np.full(n, u, dtype=np.float64), f"hubbard_chain_{n}",
                        np.arange(n, dtype=np.int64))


def with_pair_terms(m: HubbardModel, pairs, v=0.0, jh=0.0, jx=0.0, jp=0.0, name: str = "") -> HubbardModel:
    """A copy of m with two-body terms on the given site pairs (scalars or
    one value per pair)."""
    p = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    k = len(p)
    full = lambda x: np.broadcast_to(np.asarray(x, dtype=np.float64), (k,)).copy()
    return HubbardModel(m.n_sites, m.hi, m.hj, m.t, m.u_site, name or m.name + "_ext", m.site_x,
                        p[:, 0].copy(), p[:, 1].copy(), full(v), full(jh), full(jx), full(jp), m.t_im)


def extended_hubbard_square(lx: int, ly: int, t: float = 1.0, u: float = 4.0, v: float = 1.0,
                            j: float = 0.3) -> HubbardModel:
    """Nearest-neighbour extended Hubbard model on the periodic square
    lattice in the form the Wannier-function input of Sec. 5 produces: one
    Coulomb V and one exchange integral J per bond, J entering the Hund,
    exchange and pair-hopping terms alike."""
    m = hubbard_square(lx, ly, t, u)
    return with_pair_terms(m, np.stack([m.hi, m.hj], axis=1), v, j, j, j,
                           f"ext_hubbard_square_{lx}x{ly}")


@dataclass
class HubbardFrames:
    """Time-dependent amplitudes of a HubbardModel (Sec. 3.4: H(t) with
    t_ij(t) and two-body terms I(t)). Frame k holds the amplitudes at time
    t_k; None keeps the model's own values in every frame."""
    n_frames: int
    hop_t: Optional[np.ndarray] = None    # (n_frames, n_hops)
    u_site: Optional[np.ndarray] = None   # (n_frames, n_sites)
    pair_v: Optional[np.ndarray] = None   # (n_frames, n_pairs, 4): v, j_hund, j_ex, j_pair
    hop_t_im: Optional[np.ndarray] = None  # (n_frames, n_hops): imaginary parts of the transfers


def model_at_frame(m: HubbardModel, fr: HubbardFrames, k: int) -> HubbardModel:
    """The model with the amplitudes of frame min(k, n_frames - 1)."""
    f = min(int(k), fr.n_frames - 1)
    t = m.t if fr.hop_t is None else np.array(fr.hop_t[f], dtype=np.float64)
    t_im = m.t_im if fr.hop_t_im is None else np.array(fr.hop_t_im[f], dtype=np.float64)
    u = m.u_site if fr.u_site is None else np.array(fr.u_site[f], dtype=np.float64)
    pv, pjh, pjx, pjp = m.pv, m.pjh, m.pjx, m.pjp
    if fr.pair_v is not None and m.n_pairs:
        pa = np.asarray(fr.pair_v[f], dtype=np.float64)
        pv, pjh, pjx, pjp = (pa[:, c].copy() for c in range(4))
    return HubbardModel(m.n_sites, m.hi, m.hj, t, u, f"{m.name}_frame{f}", m.site_x,
                        m.pi, m.pj, pv, pjh, pjx, pjp, t_im)


def interaction_ramp(m: HubbardModel, u_from: float, u_to: float, n_ramp: int, n_frames: int) -> HubbardFrames:
    """U(t_k) rising linearly from u_from at k = 0 to u_to at k = n_ramp and
    constant after: the interaction quench of Sec. 3.4 spread over n_ramp
    steps (n_ramp = 0: the sudden quench)."""
    k = np.arange(n_frames, dtype=np.float64)
    u = u_to if n_ramp <= 0 else u_from + (u_to - u_from) * np.minimum(k, n_ramp) / n_ramp
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), (n_frames,))
    return HubbardFrames(n_frames, u_site=np.repeat(u[:, None], m.n_sites, axis=1))


def hopping_drive(m: HubbardModel, amp: float, omega: float, dt: float, n_frames: int) -> HubbardFrames:
    """Periodically modulated transfers t_ij(t_k) = t_ij (1 + amp sin(omega k dt))
    (every hop scaled alike; amp > 1 makes the factor change sign)."""
    f = 1.0 + amp * np.sin(omega * dt * np.arange(n_frames))
    return HubbardFrames(n_frames, hop_t=f[:, None] * np.asarray(m.t, dtype=np.float64)[None, :])


def hop_displacements(m: HubbardModel) -> np.ndarray:
    """x_i - x_j of each hop (i, j) along the site coordinate site_x, taken
    as the nearest periodic image on a ring of max(site_x) + 1 positions."""
    x = np.asarray(m.site_x, dtype=np.int64)
    L = int(x.max()) + 1
    d = x[np.asarray(m.hi)] - x[np.asarray(m.hj)]
    return ((d + L // 2) % L) - L // 2


def with_flux(m: HubbardModel, phi: float, name: str = "") -> HubbardModel:
    """A copy of m with a uniform vector potential: t_ij -> t_ij e^{i A (x_i - x_j)},
    A = phi / L (total flux phi through the ring of L positions)."""
    x = np.asarray(m.site_x, dtype=np.int64)
    a = phi / (int(x.max()) + 1)
    tc = np.asarray(m.t, dtype=np.float64) * np.exp(1j * a * hop_displacements(m))
    return HubbardModel(m.n_sites, m.hi, m.hj, tc.real.copy(), m.u_site, name or m.name + "_flux", m.site_x,
                        m.pi, m.pj, m.pv, m.pjh, m.pjx, m.pjp, tc.imag.copy())


def peierls_pulse(m: HubbardModel, a0: float, omega: float, t_center: float, sigma: float, dt: float,
                  n_frames: int) -> HubbardFrames:
    """Transfers in a light pulse through the Peierls phase,
    t_ij(t_k) = t_ij e^{i A(t_k) (x_i - x_j)} with
    A(t) = a0 exp(-(t - t_center)^2 / (2 sigma^2)) cos(omega (t - t_center)),
    t_k = k dt."""
    tk = dt * np.arange(n_frames)
    a = a0 * np.exp(-((tk - t_center) ** 2) / (2.0 * sigma * sigma)) * np.cos(omega * (tk - t_center))
    tc = np.asarray(m.t, dtype=np.float64)[None, :] * np.exp(1j * a[:, None] * hop_displacements(m)[None, :])
    return HubbardFrames(n_frames, hop_t=tc.real.copy(), hop_t_im=tc.imag.copy())


def random_frames(m: HubbardModel, n_frames: int, seed: int, hops: bool = True, u: bool = True,
                  pairs: bool = True, repeat: int = 2) -> HubbardFrames:
    """Seeded random amplitudes around the model's, each drawn frame held
    for `repeat` consecutive frames. Transfers: t_h (1/2 + r), r uniform in
    [0, 1) per hop and frame (independent trajectories); U_i: U_i + r,
    r uniform in [-1, 1); pair coefficients: c (1/2 + r)."""
    rng = np.random.default_rng(seed)
    nd = (n_frames + repeat - 1) // repeat
    idx = np.arange(n_frames) // repeat
    ht = us = pv = None
    if hops and m.n_hops:
        ht = (np.asarray(m.t, dtype=np.float64)[None, :] * (0.5 + rng.random((nd, m.n_hops))))[idx]
    if u:
        us = (np.asarray(m.u_site, dtype=np.float64)[None, :] + rng.uniform(-1.0, 1.0, (nd, m.n_sites)))[idx]
    if pairs and m.n_pairs:
        base = np.stack([m.pv, m.pjh, m.pjx, m.pjp], axis=1).astype(np.float64)
        pv = (base[None, :, :] * (0.5 + rng.random((nd, m.n_pairs, 4))))[idx]
    return HubbardFrames(n_frames, ht, us, pv)


def random_vector(dim: int, seed: int, dtype=np.float64, nvec: int = 1) -> np.ndarray:
    """Seeded test vector (numpy PCG64), uniform in [-1/2, 1/2); complex
    dtypes get independent real and imaginary parts. Shape (dim,) or
    (dim, nvec)."""
    rng = np.random.default_rng(seed)
    shape = (dim,) if nvec == 1 else (dim, nvec)
    if np.issubdtype(np.dtype(dtype), np.complexfloating):
        v = rng.random(shape) - 0.5 + 1j * (rng.random(shape) - 0.5)
    else:
        v = rng.random(shape) - 0.5
    return v.astype(dtype)


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the replay
    kind: str               # "lanczos" or "sqw"
    lattice: str            # "chain" or "ladder"
    n_sites: int
    two_sz: int


def serving_requests(n_req: int, rate: float, seed: int = 7,
                     n_range=(12, 26), sqw_frac: float = 0.5) -> List[Request]:
    """Poisson arrivals (exponential gaps at `rate` per second); half the
    requests ask for a ground state, half for S(q, w); half chains, half
    2-leg ladders (odd sizes redrawn for ladders); 2Sz = N mod 2."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_req):
        t += rng.exponential(1.0 / rate)
        kind = "sqw" if rng.random() < sqw_frac else "lanczos"
        lattice = "ladder" if rng.random() < 0.5 else "chain"
        while True:
            n = int(rng.integers(n_range[0], n_range[1] + 1))
            if lattice == "chain" or n % 2 == 0:
                break
        out.append(Request(r, t, kind, lattice, n, n % 2))
    return out
