"""Thin Python binding over the C ABI (argument marshalling only).

Device memory and streams come from PyTorch-ROCm; every step of the hot path
runs in the HIP library. Names mirror include/hphi_mi355.h.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _lib as L
from .workloads import HubbardModel, SpinModel


class HphiError(RuntimeError):
    def __init__(self, msg: str, code: int = 0):
        super().__init__(msg)
        self.code = code


def _check(rc: int, what: str):
    if rc != 0:
        msg = L.lib().hphi_last_error()
        raise HphiError(f"{what} failed ({rc}): {msg.decode() if msg else ''}", rc)


def _torch():
    import torch
    return torch


def dtype_code(t) -> int:
    torch = _torch()
    m = {torch.float64: L.F64, torch.float32: L.F32, torch.complex128: L.C128, torch.complex64: L.C64}
    if t.dtype not in m:
        raise HphiError(f"unsupported tensor dtype {t.dtype}")
    return m[t.dtype]


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        torch = _torch()
        return torch.cuda.current_stream().cuda_stream or None
    return getattr(stream, "cuda_stream", stream) or None


def _dev_check(t, name):
    if not t.is_cuda:
        raise HphiError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise HphiError(f"{name} must be contiguous")


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        _check(L.lib().hphi_init(device, C.byref(h)), "hphi_init")
        self.h = h

    def close(self):
        if self.h:
            L.lib().hphi_fini(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Basis:
    def __init__(self, ctx: Context, handle, kind: str):
        self.ctx, self.h, self.kind = ctx, handle, kind

    @classmethod
    def spin(cls, ctx: Context, n_sites: int, two_sz: int) -> "Basis":
        h = C.c_void_p()
        _check(L.lib().hphi_basis_spin(ctx.h, n_sites, two_sz, C.byref(h)), "hphi_basis_spin")
        b = cls(ctx, h, "spin")
        b.n_sites = n_sites
        return b

    @classmethod
    def spin_s(cls, ctx: Context, n_sites: int, two_s: int, two_sz: int) -> "Basis":
        """Spin-S sector (2S = two_s) with total 2S^z = two_sz."""
        h = C.c_void_p()
        _check(L.lib().hphi_basis_spin_s(ctx.h, n_sites, two_s, two_sz, C.byref(h)), "hphi_basis_spin_s")
        b = cls(ctx, h, "spin_s")
        b.n_sites = n_sites
        return b

    @classmethod
    def spin_gc(cls, ctx: Context, n_sites: int) -> "Basis":
        """The whole 2^N spin-1/2 space (index = configuration)."""
        h = C.c_void_p()
        _check(L.lib().hphi_basis_spin_gc(ctx.h, n_sites, C.byref(h)), "hphi_basis_spin_gc")
        b = cls(ctx, h, "spin_gc")
        b.n_sites = n_sites
        return b

    @classmethod
    def hubbard(cls, ctx: Context, n_sites: int, n_up: int, n_dn: int) -> "Basis":
        h = C.c_void_p()
        _check(L.lib().hphi_basis_hubbard(ctx.h, n_sites, n_up, n_dn, C.byref(h)), "hphi_basis_hubbard")
        b = cls(ctx, h, "hubbard")
        b.n_sites = n_sites
        return b

    @property
    def dim(self) -> int:
        return int(L.lib().hphi_basis_dim(self.h))

    def states(self, first: int, count: int) -> np.ndarray:
        out = np.empty(count, dtype=np.uint64)
        _check(L.lib().hphi_basis_states(self.h, first, count, out.ctypes.data), "hphi_basis_states")
        return out

    def rank(self, states: np.ndarray) -> np.ndarray:
        s = np.ascontiguousarray(states, dtype=np.uint64)
        out = np.empty(s.shape[0], dtype=np.int64)
        _check(L.lib().hphi_basis_rank(self.h, s.ctypes.data, s.shape[0], out.ctypes.data), "hphi_basis_rank")
        return out

    def states_device(self, first: int, count: int, stream=None):
        torch = _torch()
        out = torch.empty(count, dtype=torch.int64, device=f"cuda:{self.ctx.device}")
        _check(L.lib().hphi_basis_states_device(self.h, first, count, out.data_ptr(),
                                                 _stream_ptr(stream)), "hphi_basis_states_device")
        return out

    def rank_device(self, states, stream=None):
        torch = _torch()
        _dev_check(states, "states")
        out = torch.empty(states.shape[0], dtype=torch.int64, device=states.device)
        _check(L.lib().hphi_basis_rank_device(self.h, states.data_ptr(), states.shape[0],
                                               out.data_ptr(), _stream_ptr(stream)),
               "hphi_basis_rank_device")
        return out

    def tables(self, species: int = 0):
        lo = C.POINTER(C.c_uint32)()
        hi = C.POINTER(C.c_uint64)()
        nlo, nhi = C.c_int(), C.c_int()
        _check(L.lib().hphi_basis_tables(self.h, species, C.byref(lo), C.byref(hi), C.byref(nlo),
                                         C.byref(nhi)), "hphi_basis_tables")
        lo_a = np.ctypeslib.as_array(lo, shape=(1 << nlo.value,)).copy()
        hi_a = np.ctypeslib.as_array(hi, shape=((1 << nhi.value) + 1,)).copy()
        return lo_a, hi_a, nlo.value, nhi.value

    def close(self):
        if self.h:
            L.lib().hphi_basis_free(self.h)
            self.h = None


class Hamiltonian:
    def __init__(self, basis: Basis, handle, model):
        self.basis, self.h, self.model = basis, handle, model

    @classmethod
    def spin(cls, basis: Basis, m: SpinModel) -> "Hamiltonian":
        arr = (L.SpinBond * max(1, m.n_bonds))()
        for k in range(m.n_bonds):
            arr[k] = L.SpinBond(int(m.bi[k]), int(m.bj[k]), float(m.jz[k]), float(m.jxy[k]))
        hz = None
        if m.hz is not None:
            hz_a = np.ascontiguousarray(m.hz, dtype=np.float64)
            hz = hz_a.ctypes.data_as(L.PD)
        h = C.c_void_p()
        _check(L.lib().hphi_ham_spin(basis.h, arr, m.n_bonds, hz, C.byref(h)), "hphi_ham_spin")
        return cls(basis, h, m)

    @classmethod
    def spin_s(cls, basis: Basis, m) -> "Hamiltonian":
        arr = (L.SpinBond * max(1, m.n_bonds))()
        for k in range(m.n_bonds):
            arr[k] = L.SpinBond(int(m.bi[k]), int(m.bj[k]), float(m.jz[k]), float(m.jxy[k]))
        keep = []

        def opt(x):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype=np.float64)
            keep.append(a)
            return a.ctypes.data_as(L.PD)
        h = C.c_void_p()
        _check(L.lib().hphi_ham_spin_s(basis.h, arr, m.n_bonds, opt(m.hz), opt(m.d_ion), C.byref(h)),
               "hphi_ham_spin_s")
        return cls(basis, h, m)

    @classmethod
    def spin_gc(cls, basis: Basis, m) -> "Hamiltonian":
        arr = (L.XyzBond * max(1, m.n_bonds))()
        for k in range(m.n_bonds):
            arr[k] = L.XyzBond(int(m.bi[k]), int(m.bj[k]), float(m.jx[k]), float(m.jy[k]), float(m.jz[k]))
        hx = np.ascontiguousarray(m.hx, dtype=np.float64)
        hz = np.ascontiguousarray(m.hz, dtype=np.float64)
        h = C.c_void_p()
        _check(L.lib().hphi_ham_spin_gc(basis.h, arr, m.n_bonds, hx.ctypes.data_as(L.PD), hz.ctypes.data_as(L.PD),
                                        C.byref(h)), "hphi_ham_spin_gc")
        return cls(basis, h, m)

    @classmethod
    def hubbard(cls, basis: Basis, m: HubbardModel, frames=None) -> "Hamiltonian":
        """frames: optional HubbardFrames (time-dependent amplitudes, frame 0
        in force after the build)."""
        arr = (L.Hop * max(1, m.n_hops))()
        for k in range(m.n_hops):
            arr[k] = L.Hop(int(m.hi[k]), int(m.hj[k]), float(m.t[k]))
        us = np.ascontiguousarray(m.u_site, dtype=np.float64)
        h = C.c_void_p()
        n_pairs = getattr(m, "n_pairs", 0)
        pa = (L.PairTerm * max(1, n_pairs))()
        for k in range(n_pairs):
            pa[k] = L.PairTerm(int(m.pi[k]), int(m.pj[k]), float(m.pv[k]), float(m.pjh[k]),
                               float(m.pjx[k]), float(m.pjp[k]))
        t_im = getattr(m, "t_im", None)
        if frames is None and t_im is not None and np.any(np.asarray(t_im) != 0.0):
            # complex transfers: one frame holding them
            from .workloads import HubbardFrames
            frames = HubbardFrames(1, hop_t=np.asarray(m.t, dtype=np.float64)[None, :],
                                   hop_t_im=np.asarray(t_im, dtype=np.float64)[None, :])
        if frames is not None:
            keep = []

            def arr2(x):
                if x is None:
                    return None
                a = np.ascontiguousarray(x, dtype=np.float64)
                keep.append(a)
                return a.ctypes.data_as(L.PD)
            hop_t_im = getattr(frames, "hop_t_im", None)
            if hop_t_im is None and t_im is not None:
                hop_t_im = np.tile(np.asarray(t_im, dtype=np.float64)[None, :], (int(frames.n_frames), 1))
            fr = L.HubFrames(int(frames.n_frames), arr2(frames.hop_t), arr2(hop_t_im), arr2(frames.u_site),
                             arr2(frames.pair_v))
            _check(L.lib().hphi_ham_hubbard_td(basis.h, arr, m.n_hops, us.ctypes.data_as(L.PD), pa, n_pairs,
                                               C.byref(fr), C.byref(h)), "hphi_ham_hubbard_td")
        elif n_pairs:
            _check(L.lib().hphi_ham_hubbard_ext(basis.h, arr, m.n_hops, us.ctypes.data_as(L.PD), pa, n_pairs,
                                                C.byref(h)), "hphi_ham_hubbard_ext")
        else:
            _check(L.lib().hphi_ham_hubbard(basis.h, arr, m.n_hops, us.ctypes.data_as(L.PD), C.byref(h)),
                   "hphi_ham_hubbard")
        return cls(basis, h, m)

    def set_frame(self, frame: int, stream=None):
        """Puts frame `frame` of a time-dependent Hamiltonian in force."""
        _check(L.lib().hphi_ham_set_frame(self.h, int(frame), _stream_ptr(stream)), "hphi_ham_set_frame")

    def frames(self):
        """(number of frames, frame in force); (0, 0) for fixed amplitudes."""
        n, cur = C.c_int(), C.c_int()
        _check(L.lib().hphi_ham_frames(self.h, C.byref(n), C.byref(cur)), "hphi_ham_frames")
        return n.value, cur.value

    def trace(self, stream=None) -> float:
        out = C.c_double()
        _check(L.lib().hphi_ham_trace(self.h, C.byref(out), _stream_ptr(stream)), "hphi_ham_trace")
        return out.value

    def mult(self, v, w=None, stream=None):
        """w = H v. v: (dim,) or (dim, nvec) device tensor (f64, f32, c128, c64)."""
        torch = _torch()
        _dev_check(v, "v")
        nvec = 1 if v.dim() == 1 else v.shape[1]
        if w is None:
            w = torch.empty_like(v)
        _dev_check(w, "w")
        _check(L.lib().hphi_mult(self.h, dtype_code(v), v.data_ptr(), w.data_ptr(), nvec,
                                 _stream_ptr(stream)), "hphi_mult")
        return w

    SCHEDULE_FIELDS = ("hub_slab_cols", "hub_groups", "hub_item_rows", "hub_row_cols", "spin_per_cu",
                       "spin_implicit", "hub_sweep", "hub_row_order", "spin_tables", "hub_tile_bits",
                       "spin_split", "spin_blk_lo")

    def set_schedule(self, **kw):
        s = L.Schedule(*[int(kw.get(f, 0)) for f in self.SCHEDULE_FIELDS])
        _check(L.lib().hphi_ham_set_schedule(self.h, C.byref(s)), "hphi_ham_set_schedule")

    def get_schedule(self) -> Dict[str, int]:
        s = L.Schedule()
        _check(L.lib().hphi_ham_get_schedule(self.h, C.byref(s)), "hphi_ham_get_schedule")
        return {f: getattr(s, f) for f in self.SCHEDULE_FIELDS}

    def close(self):
        if self.h:
            L.lib().hphi_ham_free(self.h)
            self.h = None


def lanczos(ham: Hamiltonian, max_iter: int, seed: int = 1, v0=None, storage: str = "f64",
            n_energies: int = 1, want_vector: bool = False, use_graph: bool = False,
            check_every: int = 0, tol: float = 1e-12, time_kernels: bool = False,
            refine: bool = False, resid_tol: float = 0.0, no_alloc: bool = False, refine_steps: int = 0,
            stream=None) -> Dict:
    """Lanczos ground state. refine: FP64 Rayleigh quotient of the Ritz
    vector (second pass accumulated in FP64), returned as energies[0] with
    its residual |H psi - rho psi| and error estimate, then refine_steps
    (0: 16; < 0: none) FP64 Lanczos steps from that vector, whose lowest
    Ritz value becomes energies[0] (polish_e0). no_alloc: the entry
    point that takes its device buffers from the library's static scratch
    (hphi_lanczos_noalloc) instead of allocating them. storage "c128" or
    "c64": complex vectors (Hermitian H with complex transfers)."""
    torch = _torch()
    o = L.LanczosOpts()
    o.max_iter, o.check_every, o.tol, o.seed = max_iter, check_every, tol, seed
    o.resid_tol = resid_tol
    codes = {"f64": (L.F64, torch.float64), "f32": (L.F32, torch.float32),
             "c128": (L.C128, torch.complex128), "c64": (L.C64, torch.complex64)}
    if storage not in codes:
        raise HphiError(f"storage {storage!r}: f64, f32, c128 or c64")
    o.storage, tdt = codes[storage]
    if v0 is not None:
        _dev_check(v0, "v0")
        if v0.dtype != tdt:
            raise HphiError("v0 must have the storage dtype")
        o.v0_dev = v0.data_ptr()
    o.stream = _stream_ptr(stream)
    alpha = np.zeros(max_iter)
    beta = np.zeros(max_iter)
    o.alpha_out = alpha.ctypes.data_as(L.PD)
    o.beta_out = beta.ctypes.data_as(L.PD)
    psi = None
    if want_vector:
        psi = torch.empty(ham.basis.dim, dtype=tdt, device=f"cuda:{ham.basis.ctx.device}")
        o.psi_dev = psi.data_ptr()
    o.use_graph = 1 if use_graph else 0
    o.time_kernels = 1 if time_kernels else 0
    o.refine = 1 if refine else 0
    o.refine_steps = refine_steps
    e = np.zeros(n_energies)
    info = L.LanczosInfo()
    fn = L.lib().hphi_lanczos_noalloc if no_alloc else L.lib().hphi_lanczos
    _check(fn(ham.h, C.byref(o), e.ctypes.data_as(L.PD), n_energies, C.byref(info)),
           "hphi_lanczos_noalloc" if no_alloc else "hphi_lanczos")
    n = info.iterations
    return {"energies": e, "alpha": alpha[:n], "beta": beta[:n], "iterations": n,
            "converged": bool(info.converged), "breakdown": bool(info.breakdown),
            "seconds": info.seconds, "hv_seconds": info.hv_seconds, "hv_calls": info.hv_calls,
            "fused_update": bool(info.fused_update),
            "hv_second_kernel_seconds": info.hv_second_kernel_seconds, "psi": psi,
            "ritz_e0": info.ritz_e0, "rq_e0": info.rq_e0, "residual": info.residual,
            "err_est": info.err_est, "polish_e0": info.polish_e0, "polish_resid": info.polish_resid}


def lanczos_batch(hams: Sequence[Hamiltonian], max_iter, seeds, keep_coefficients: bool = False,
                  stream=None):
    """Independent Lanczos ground-state solves in one launch (a team of
    workgroups per request when the launch is small, one workgroup per
    request otherwise; the same numbers either way). max_iter and seeds are
    scalars or per-request sequences."""
    n = len(hams)
    its = [max_iter] * n if np.isscalar(max_iter) else list(max_iter)
    sds = [seeds] * n if np.isscalar(seeds) else list(seeds)
    arr = (L.BatchItem * n)()
    keep = []
    for i, h in enumerate(hams):
        arr[i].ham = h.h
        arr[i].max_iter = int(its[i])
        arr[i].seed = int(sds[i])
        if keep_coefficients:
            a = np.zeros(its[i])
            b = np.zeros(its[i])
            keep.append((a, b))
            arr[i].alpha_out = a.ctypes.data_as(L.PD)
            arr[i].beta_out = b.ctypes.data_as(L.PD)
    _check(L.lib().hphi_lanczos_batch(arr, n, _stream_ptr(stream)), "hphi_lanczos_batch")
    out = []
    for i in range(n):
        d = {"energy": arr[i].energy, "iterations": arr[i].iterations, "breakdown": bool(arr[i].breakdown)}
        if keep_coefficients:
            k = arr[i].iterations
            d["alpha"], d["beta"] = keep[i][0][:k], keep[i][1][:k]
        out.append(d)
    return out


def tridiag_lowest(alpha: np.ndarray, beta: np.ndarray, k: int = 1, want_vector: bool = False):
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    ev = np.zeros(k)
    vec = np.zeros(len(a)) if want_vector else None
    _check(L.lib().hphi_tridiag_lowest(a.ctypes.data_as(L.PD), b.ctypes.data_as(L.PD), len(a), k,
                                       ev.ctypes.data_as(L.PD),
                                       vec.ctypes.data_as(L.PD) if vec is not None else None),
           "hphi_tridiag_lowest")
    return (ev, vec) if want_vector else ev


def ctpq(ham: Hamiltonian, n_vec: int, n_max: int, dtau: float, k_steps: int,
         storage: str = "c128", seed: int = 1, phi0=None, use_graph: bool = False, stream=None) -> Dict:
    torch = _torch()
    o = L.CtpqOpts()
    o.n_vec, o.n_max, o.dtau, o.k_steps, o.seed = n_vec, n_max, dtau, k_steps, seed
    o.use_graph = 1 if use_graph else 0
    o.storage = L.C128 if storage == "c128" else L.C64
    tdt = torch.complex128 if storage == "c128" else torch.complex64
    if phi0 is not None:
        _dev_check(phi0, "phi0")
        if phi0.dtype != tdt:
            raise HphiError("phi0 must have the storage dtype")
        o.phi0_dev = phi0.data_ptr()
    o.stream = _stream_ptr(stream)
    phi = torch.empty((ham.basis.dim, n_vec), dtype=tdt, device=f"cuda:{ham.basis.ctx.device}")
    D = np.zeros((k_steps + 1, n_vec))
    E = np.zeros((k_steps + 1, n_vec))
    E2 = np.zeros((k_steps + 1, n_vec))
    _check(L.lib().hphi_ctpq(ham.h, C.byref(o), phi.data_ptr(), D.ctypes.data_as(L.PD),
                             E.ctypes.data_as(L.PD), E2.ctypes.data_as(L.PD)), "hphi_ctpq")
    return {"beta": dtau * np.arange(k_steps + 1), "D": D, "E": E, "E2": E2, "phi": phi}


def time_evolve(ham: Hamiltonian, psi, n_steps: int, dt: float = 0.01, n_max: int = 10,
                double_occupancy: bool = False, use_graph: bool = False, stream=None,
                first_frame: int = 0) -> Dict:
    """Real-time evolution of psi (device tensor [dim] or [dim, n_vec],
    complex128 or complex64, updated in place) by the truncated Taylor series;
    returns per recorded time norms, energies and (Hubbard) double occupancy.
    A Hamiltonian with frames takes frame min(first_frame + k, n_frames - 1)
    at t_k."""
    _dev_check(psi, "psi")
    torch = _torch()
    if psi.dtype not in (torch.complex128, torch.complex64):
        raise HphiError("psi must be complex128 or complex64")
    nv = 1 if psi.dim() == 1 else int(psi.shape[1])
    o = L.TevolOpts()
    o.n_vec, o.n_max, o.dt, o.n_steps = nv, n_max, dt, n_steps
    o.storage = L.C128 if psi.dtype == torch.complex128 else L.C64
    o.stream = _stream_ptr(stream)
    o.use_graph = 1 if use_graph else 0
    o.first_frame = int(first_frame)
    nrm = np.zeros((n_steps + 1) * nv)
    en = np.zeros((n_steps + 1) * nv)
    dc = np.zeros(n_steps + 1) if double_occupancy else None
    _check(L.lib().hphi_time_evolve(ham.h, C.byref(o), psi.data_ptr(), nrm.ctypes.data_as(L.PD),
                                    en.ctypes.data_as(L.PD),
                                    dc.ctypes.data_as(L.PD) if dc is not None else None), "hphi_time_evolve")
    out = {"norm": nrm.reshape(n_steps + 1, nv), "energy": en.reshape(n_steps + 1, nv),
           "t": dt * np.arange(n_steps + 1)}
    if dc is not None:
        out["double_occupancy"] = dc
    return out


def lobpcg(ham: Hamiltonian, n_eig: int, max_iter: int = 500, tol: float = 1e-8, seed: int = 1,
           precond: bool = True, e_shift: float = 0.0, want_vectors: bool = False, stream=None) -> Dict:
    """Lowest n_eig eigenpairs by LOBPCG (point-Jacobi preconditioner with
    shift e_shift, 0 = a lower bound from the couplings)."""
    torch = _torch()
    o = L.LobpcgOpts()
    o.n_eig, o.max_iter, o.tol, o.seed = n_eig, max_iter, tol, seed
    o.precond, o.e_shift, o.stream = (1 if precond else 0), e_shift, _stream_ptr(stream)
    e = np.zeros(n_eig)
    res = np.zeros(n_eig)
    vecs = None
    if want_vectors:
        vecs = torch.empty((n_eig, ham.basis.dim), dtype=torch.float64, device=f"cuda:{ham.basis.ctx.device}")
    info = L.LobpcgInfo()
    _check(L.lib().hphi_lobpcg(ham.h, C.byref(o), e.ctypes.data_as(L.PD), res.ctypes.data_as(L.PD),
                               vecs.data_ptr() if vecs is not None else None, C.byref(info)), "hphi_lobpcg")
    return {"energies": e, "residuals": res, "vectors": vecs, "iterations": info.iterations,
            "converged": bool(info.converged), "hv_calls": info.hv_calls, "seconds": info.seconds}


def szq(ham: Hamiltonian, q: float, psi, stream=None):
    """b = sum_l e^{i q x_l} S^z_l psi, x_l from the model's site_x."""
    torch = _torch()
    _dev_check(psi, "psi")
    sx = getattr(ham.model, "site_x", None)
    x = np.arange(ham.basis.n_sites, dtype=np.float64) if sx is None else np.asarray(sx, dtype=np.float64)
    phase = np.empty(2 * len(x))
    phase[0::2] = np.cos(q * x)
    phase[1::2] = np.sin(q * x)
    b = torch.empty(ham.basis.dim, dtype=torch.complex128, device=psi.device)
    _check(L.lib().hphi_szq(ham.h, phase.ctypes.data_as(L.PD), psi.data_ptr(), b.data_ptr(),
                            _stream_ptr(stream)), "hphi_szq")
    return b


def sqw_batch(hams: Sequence[Hamiltonian], bs, zs, max_iter: int = 2000, tol: float = 1e-8,
              seed_shift: int = -1, stream=None) -> List[Dict]:
    """sqw for many spin requests in one launch (one workgroup per sequence):
    hams[i], excitation bs[i] (complex128 device tensor), shifts zs[i] (all
    of the same length)."""
    n = len(hams)
    if n == 0:
        return []
    zs = [np.asarray(z, dtype=np.complex128) for z in zs]
    ns = len(zs[0])
    if any(len(z) != ns for z in zs) or len(bs) != n or len(zs) != n:
        raise HphiError("sqw_batch: one excitation and one shift list of equal length per request")
    for b in bs:
        _dev_check(b, "b")
    zr = np.ascontiguousarray(np.concatenate([z.real for z in zs]))
    zi = np.ascontiguousarray(np.concatenate([z.imag for z in zs]))
    D = np.zeros(2 * ns * n)
    res = np.zeros(ns * n)
    o = L.SqwOpts()
    o.max_iter, o.tol, o.seed_shift, o.stream = max_iter, tol, seed_shift, _stream_ptr(stream)
    infos = (L.SqwInfo * n)()
    hs = (C.c_void_p * n)(*[h.h for h in hams])
    bp = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
    _check(L.lib().hphi_sqw_batch(hs, n, C.byref(o), bp, zr.ctypes.data_as(L.PD), zi.ctypes.data_as(L.PD), ns,
                                  D.ctypes.data_as(L.PD), res.ctypes.data_as(L.PD), infos), "hphi_sqw_batch")
    out = []
    for i in range(n):
        d = D[2 * ns * i:2 * ns * (i + 1)]
        out.append({"D": d[0::2] + 1j * d[1::2], "residual": res[ns * i:ns * (i + 1)].copy(),
                    "iterations": infos[i].iterations, "converged": bool(infos[i].converged),
                    "max_residual": infos[i].max_residual, "seconds": infos[i].seconds})
    return out


def sqw(ham: Hamiltonian, b, z: Sequence[complex], max_iter: int = 2000, tol: float = 1e-8,
        seed_shift: int = -1, stream=None) -> Dict:
    _dev_check(b, "b")
    z = np.asarray(z, dtype=np.complex128)
    zr, zi = np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)
    D = np.zeros(2 * len(z))
    res = np.zeros(len(z))
    o = L.SqwOpts()
    o.max_iter, o.tol, o.seed_shift, o.stream = max_iter, tol, seed_shift, _stream_ptr(stream)
    info = L.SqwInfo()
    _check(L.lib().hphi_sqw(ham.h, C.byref(o), b.data_ptr(), zr.ctypes.data_as(L.PD),
                            zi.ctypes.data_as(L.PD), len(z), D.ctypes.data_as(L.PD),
                            res.ctypes.data_as(L.PD), C.byref(info)), "hphi_sqw")
    return {"D": D[0::2] + 1j * D[1::2], "residual": res, "iterations": info.iterations,
            "converged": bool(info.converged), "max_residual": info.max_residual,
            "seconds": info.seconds}
