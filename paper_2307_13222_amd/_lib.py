"""ctypes declarations of the C ABI in include/hphi_mi355.h.

The shared library is built in-tree by paper_2307_13222_amd/build.py. There
is no fallback: if it is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "libhphi_mi355.so")

F64, F32, C128, C64 = 0, 1, 2, 3
ERR_BUSY = -7
NOALLOC_SCRATCH_BYTES = 64 << 20


class SpinBond(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("jz", C.c_double), ("jxy", C.c_double)]


class Hop(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("t", C.c_double)]


class XyzBond(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("jx", C.c_double), ("jy", C.c_double), ("jz", C.c_double)]


class PairTerm(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("v", C.c_double), ("j_hund", C.c_double),
                ("j_ex", C.c_double), ("j_pair", C.c_double)]


class HubFrames(C.Structure):
    _fields_ = [("n_frames", C.c_int), ("hop_t", C.POINTER(C.c_double)), ("hop_t_im", C.POINTER(C.c_double)),
                ("u_site", C.POINTER(C.c_double)), ("pair_v", C.POINTER(C.c_double))]


class LanczosOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("check_every", C.c_int), ("tol", C.c_double),
                ("resid_tol", C.c_double), ("seed", C.c_uint64), ("v0_dev", C.c_void_p), ("storage", C.c_int),
                ("stream", C.c_void_p), ("alpha_out", C.POINTER(C.c_double)),
                ("beta_out", C.POINTER(C.c_double)), ("psi_dev", C.c_void_p),
                ("use_graph", C.c_int), ("time_kernels", C.c_int), ("refine", C.c_int),
                ("refine_steps", C.c_int)]


class LanczosInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("breakdown", C.c_int),
                ("seconds", C.c_double), ("hv_seconds", C.c_double), ("hv_calls", C.c_int),
                ("fused_update", C.c_int), ("hv_second_kernel_seconds", C.c_double),
                ("ritz_e0", C.c_double), ("rq_e0", C.c_double), ("residual", C.c_double),
                ("err_est", C.c_double), ("polish_e0", C.c_double), ("polish_resid", C.c_double)]


class BatchItem(C.Structure):
    _fields_ = [("ham", C.c_void_p), ("max_iter", C.c_int), ("seed", C.c_uint64),
                ("alpha_out", C.POINTER(C.c_double)), ("beta_out", C.POINTER(C.c_double)),
                ("energy", C.c_double), ("iterations", C.c_int), ("breakdown", C.c_int)]


class CtpqOpts(C.Structure):
    _fields_ = [("n_vec", C.c_int), ("n_max", C.c_int), ("dtau", C.c_double),
                ("k_steps", C.c_int), ("storage", C.c_int), ("seed", C.c_uint64),
                ("phi0_dev", C.c_void_p), ("stream", C.c_void_p), ("use_graph", C.c_int)]


class TevolOpts(C.Structure):
    _fields_ = [("n_vec", C.c_int), ("n_max", C.c_int), ("dt", C.c_double), ("n_steps", C.c_int),
                ("storage", C.c_int), ("stream", C.c_void_p), ("use_graph", C.c_int), ("first_frame", C.c_int)]


class LobpcgOpts(C.Structure):
    _fields_ = [("n_eig", C.c_int), ("max_iter", C.c_int), ("tol", C.c_double), ("seed", C.c_uint64),
                ("precond", C.c_int), ("e_shift", C.c_double), ("stream", C.c_void_p)]


class LobpcgInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("hv_calls", C.c_int64),
                ("seconds", C.c_double)]


class Schedule(C.Structure):
    _fields_ = [("hub_slab_cols", C.c_int), ("hub_groups", C.c_int), ("hub_item_rows", C.c_int),
                ("hub_row_cols", C.c_int), ("spin_per_cu", C.c_int), ("spin_implicit", C.c_int),
                ("hub_sweep", C.c_int), ("hub_row_order", C.c_int), ("spin_tables", C.c_int),
                ("hub_tile_bits", C.c_int), ("spin_split", C.c_int), ("spin_blk_lo", C.c_int)]


class SqwOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("tol", C.c_double), ("seed_shift", C.c_int),
                ("stream", C.c_void_p)]


class SqwInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("max_residual", C.c_double),
                ("seconds", C.c_double)]


# name -> (restype, argtypes)
P, I, I64, U64, D = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double
PD = C.POINTER(C.c_double)
SIGNATURES = {
    "hphi_last_error": (C.c_char_p, []),
    "hphi_version": (C.c_char_p, []),
    "hphi_init": (I, [I, C.POINTER(P)]),
    "hphi_fini": (None, [P]),
    "hphi_basis_spin": (I, [P, I, I, C.POINTER(P)]),
    "hphi_basis_hubbard": (I, [P, I, I, I, C.POINTER(P)]),
    "hphi_basis_spin_gc": (I, [P, I, C.POINTER(P)]),
    "hphi_basis_spin_s": (I, [P, I, I, I, C.POINTER(P)]),
    "hphi_ham_spin_s": (I, [P, C.POINTER(SpinBond), I, PD, PD, C.POINTER(P)]),
    "hphi_ham_spin_gc": (I, [P, C.POINTER(XyzBond), I, PD, PD, C.POINTER(P)]),
    "hphi_basis_free": (None, [P]),
    "hphi_basis_dim": (I64, [P]),
    "hphi_basis_states": (I, [P, I64, I64, P]),
    "hphi_basis_rank": (I, [P, P, I64, P]),
    "hphi_basis_states_device": (I, [P, I64, I64, P, P]),
    "hphi_basis_rank_device": (I, [P, P, I64, P, P]),
    "hphi_basis_tables": (I, [P, I, C.POINTER(C.POINTER(C.c_uint32)),
                              C.POINTER(C.POINTER(C.c_uint64)), C.POINTER(I), C.POINTER(I)]),
    "hphi_ham_spin": (I, [P, C.POINTER(SpinBond), I, PD, C.POINTER(P)]),
    "hphi_ham_hubbard": (I, [P, C.POINTER(Hop), I, PD, C.POINTER(P)]),
    "hphi_ham_hubbard_ext": (I, [P, C.POINTER(Hop), I, PD, C.POINTER(PairTerm), I, C.POINTER(P)]),
    "hphi_ham_hubbard_td": (I, [P, C.POINTER(Hop), I, PD, C.POINTER(PairTerm), I, C.POINTER(HubFrames),
                                C.POINTER(P)]),
    "hphi_ham_set_frame": (I, [P, I, P]),
    "hphi_ham_frames": (I, [P, C.POINTER(I), C.POINTER(I)]),
    "hphi_ham_free": (None, [P]),
    "hphi_ham_set_schedule": (I, [P, C.POINTER(Schedule)]),
    "hphi_ham_get_schedule": (I, [P, C.POINTER(Schedule)]),
    "hphi_ham_trace": (I, [P, PD, P]),
    "hphi_mult": (I, [P, I, P, P, I64, P]),
    "hphi_lanczos": (I, [P, C.POINTER(LanczosOpts), PD, I, C.POINTER(LanczosInfo)]),
    "hphi_lanczos_noalloc": (I, [P, C.POINTER(LanczosOpts), PD, I, C.POINTER(LanczosInfo)]),
    "hphi_tridiag_lowest": (I, [PD, PD, I, I, PD, PD]),
    "hphi_lanczos_batch": (I, [C.POINTER(BatchItem), I, P]),
    "hphi_ctpq": (I, [P, C.POINTER(CtpqOpts), P, PD, PD, PD]),
    "hphi_time_evolve": (I, [P, C.POINTER(TevolOpts), P, PD, PD, PD]),
    "hphi_lobpcg": (I, [P, C.POINTER(LobpcgOpts), PD, PD, P, C.POINTER(LobpcgInfo)]),
    "hphi_szq": (I, [P, PD, P, P, P]),
    "hphi_sqw": (I, [P, C.POINTER(SqwOpts), P, PD, PD, I, PD, PD, C.POINTER(SqwInfo)]),
    "hphi_sqw_batch": (I, [C.POINTER(P), I, C.POINTER(SqwOpts), C.POINTER(P), PD, PD, I, PD, PD,
                           C.POINTER(SqwInfo)]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        # PyTorch-ROCm ships its own HIP runtime (soname libamdhip64.so.7).
        # Load it first so this library binds to that same runtime instead
        # of pulling a second copy from /opt/rocm into the process.
        import torch  # noqa: F401
        import torch.cuda  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"HIP library not built: {LIB_PATH} is missing "
                "(run python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Names the library must export (every declaration of the header)."""
    return [n for n in SIGNATURES]
