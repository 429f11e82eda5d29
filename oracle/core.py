"""Oracle for the H*v hot path -- TEST INFRASTRUCTURE ONLY.

Plain CPU reference of what the HIP path computes. Only tests/, the smoke
check and the benchmark's CPU-baseline leg may import this module; the
product path never does. It shares no code with the HIP library: the C part
(hphi_oracle.c) is compiled separately with gcc, and the iterative methods
below are written out in numpy/scipy in the paper's order and notation.

References are to the HPhi update paper (arXiv:2307.13222):
  Sec. 1      Krylov/power methods reduce to repeated H*v; Lanczos.
  Sec. 3.2    dynamical correlation D(z) = <Phi_ex|(z - H)^-1|Phi_ex>,
              S^zz(q, w) with S^z_l and phases e^{iql}, q = 2 pi m / L.
  Sec. 3.4    real-time evolution psi(t + dt) = sum_{n<=n_max} (-i H dt)^n / n!
              psi(t); norm, energy and double occupancy as its checks; a
              time-dependent H(t) held at H(t_k) over the step from t_k.
  Sec. 3.5.1  TPQ state, random vector uniform on the d_H sphere, cTPQ
              propagator U_c = sum_{n<=n_max} (-dtau H / 2)^n / n!,
              beta_k = k dtau, relative squared norms D_k = N_k / N_{k-1}.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Callable, Dict, Optional, Tuple

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hphi_oracle.c")
# HPHI_ORACLE_LIB: another build of the same source (the sanitizer test
# loads one built with -fsanitize=address,undefined)
_LIB_PATH = os.environ.get("HPHI_ORACLE_LIB") or os.path.join(_HERE, "_build", "libhphi_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part with gcc (-O2, OpenMP)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, u64, i32, p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        L.or_binom.restype = u64; L.or_binom.argtypes = [i32, i32]
        L.or_basis_fill.restype = i64; L.or_basis_fill.argtypes = [i32, i32, p, i64]
        L.or_rank_combinadic.restype = i64; L.or_rank_combinadic.argtypes = [u64]
        L.or_unrank_combinadic.restype = u64; L.or_unrank_combinadic.argtypes = [i64, i32]
        L.or_rank_search.restype = i64; L.or_rank_search.argtypes = [p, i64, u64]
        L.or_rank_search_many.restype = None; L.or_rank_search_many.argtypes = [p, i64, p, i64, p]
        L.or_rank_combinadic_many.restype = None; L.or_rank_combinadic_many.argtypes = [p, i64, p]
        L.or_spin_hv.restype = None
        L.or_spin_hv.argtypes = [i32, p, i64, i32, p, p, p, p, p, p, p]
        L.or_spin_row_by_index.restype = i32
        L.or_spin_row_by_index.argtypes = [i32, i32, i64, i32, p, p, p, p, p, p, p]
        L.or_spin_sz_table.restype = None; L.or_spin_sz_table.argtypes = [i32, p, i64, p]
        L.or_hubbard_hv.restype = None
        L.or_hubbard_hv.argtypes = [i32, p, i64, p, i64, i32, p, p, p, p, p, p]
        L.or_hubbard_hv_rows.restype = None
        L.or_hubbard_hv_rows.argtypes = [i32, p, i64, p, i64, i32, p, p, p, p, p, i64, i64, p]
        L.or_hubbard_row.restype = i32
        L.or_hubbard_row.argtypes = [i32, p, i64, p, i64, i32, p, p, p, p, i64, i64, p, p]
        L.or_splitmix_u64.restype = None; L.or_splitmix_u64.argtypes = [u64, i64, i64, p]
        L.or_splitmix_uniform.restype = None; L.or_splitmix_uniform.argtypes = [u64, i64, i64, p]
        L.or_spin_ell.restype = None
        L.or_spin_ell.argtypes = [i32, p, i64, i32, p, p, p, p, p, p, p, p]
        L.or_hubbard_ell.restype = None
        L.or_hubbard_ell.argtypes = [i32, p, i64, p, i64, i32, p, p, p, p, p, p, p]
        L.or_hubbard_pairs_row.restype = i32
        L.or_hubbard_pairs_row.argtypes = [i32, p, i64, p, i64, i32, p, p, p, p, p, p, i64, i64, p, p]
        L.or_hubbard_pairs_hv.restype = None
        L.or_hubbard_pairs_hv.argtypes = [i32, p, i64, p, i64, i32, p, p, p, p, p, p, p, p]
        L.or_hubbard_pairs_hv_rows.restype = None
        L.or_hubbard_pairs_hv_rows.argtypes = [i32, p, i64, p, i64, i32, p, p, p, p, p, p, p, i64, i64, p]
        L.or_spin_s_basis_fill.restype = i64; L.or_spin_s_basis_fill.argtypes = [i32, i32, i32, p, i64]
        L.or_spin_s_row.restype = i32
        L.or_spin_s_row.argtypes = [i32, i32, p, i64, i32, p, p, p, p, p, p, i64, p, p]
        L.or_spin_s_hv.restype = None
        L.or_spin_s_hv.argtypes = [i32, i32, p, i64, i32, p, p, p, p, p, p, p, p]
        L.or_spin_s_ell.restype = None
        L.or_spin_s_ell.argtypes = [i32, i32, p, i64, i32, p, p, p, p, p, p, p, p, p]
        L.or_spin_gc_row.restype = i32
        L.or_spin_gc_row.argtypes = [i32, i32, p, p, p, p, p, p, p, u64, p, p]
        L.or_spin_gc_hv.restype = None
        L.or_spin_gc_hv.argtypes = [i32, i32, p, p, p, p, p, p, p, p, p]
        L.or_spin_gc_hv_rows.restype = None
        L.or_spin_gc_hv_rows.argtypes = [i32, i32, p, p, p, p, p, p, p, p, i64, i64, p]
        L.or_spin_gc_ell.restype = None
        L.or_spin_gc_ell.argtypes = [i32, i32, p, p, p, p, p, p, p, p, p, p]
        L.or_hubbard_pairs_ell.restype = None
        L.or_hubbard_pairs_ell.argtypes = [i32, p, i64, p, i64, i32, p, p, p, p, p, p, p, p, p]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------------ basis --

def binom(n: int, k: int) -> int:
    return int(lib().or_binom(n, k))


def sector_popcount_spin(n_sites: int, two_sz: int) -> int:
    """Number of up spins for total 2S^z (2Sz keyword): n_up - n_dn = 2Sz."""
    if (n_sites + two_sz) % 2 or abs(two_sz) > n_sites:
        raise ValueError("2Sz must have the parity of N and |2Sz| <= N")
    return (n_sites + two_sz) // 2


def basis_list(n_bits: int, n_pop: int) -> np.ndarray:
    """All n_bits-bit configurations with n_pop set bits, ascending (uint64)."""
    dim = binom(n_bits, n_pop)
    out = np.empty(dim, dtype=np.uint64)
    got = lib().or_basis_fill(n_bits, n_pop, _p(out), dim)
    assert got == dim
    return out


def rank_search(states: np.ndarray, xs: np.ndarray) -> np.ndarray:
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    out = np.empty(xs.shape[0], dtype=np.int64)
    lib().or_rank_search_many(_p(states), states.shape[0], _p(xs), xs.shape[0], _p(out))
    return out


def rank_combinadic(xs: np.ndarray) -> np.ndarray:
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    out = np.empty(xs.shape[0], dtype=np.int64)
    lib().or_rank_combinadic_many(_p(xs), xs.shape[0], _p(out))
    return out


def unrank_combinadic(r: int, n_pop: int) -> int:
    return int(lib().or_unrank_combinadic(int(r), n_pop))


# --------------------------------------------------------------- spin H*v --

def _spin_arrays(m):
    bi = np.ascontiguousarray(m.bi, dtype=np.int32)
    bj = np.ascontiguousarray(m.bj, dtype=np.int32)
    jz = np.ascontiguousarray(m.jz, dtype=np.float64)
    jxy = np.ascontiguousarray(m.jxy, dtype=np.float64)
    hz = None if m.hz is None else np.ascontiguousarray(m.hz, dtype=np.float64)
    return bi, bj, jz, jxy, hz


def spin_hv(m, states: np.ndarray, v: np.ndarray) -> np.ndarray:
    """w = H v for the XXZ model; complex or multi-column v is handled one
    real column at a time (H is real)."""
    v = np.asarray(v)
    if np.iscomplexobj(v):
        return spin_hv(m, states, v.real) + 1j * spin_hv(m, states, v.imag)
    if v.ndim == 2:
        return np.stack([spin_hv(m, states, v[:, k]) for k in range(v.shape[1])], axis=1)
    bi, bj, jz, jxy, hz = _spin_arrays(m)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty_like(vv)
    lib().or_spin_hv(m.n_sites, _p(states), states.shape[0], bi.shape[0], _p(bi), _p(bj),
                     _p(jz), _p(jxy), None if hz is None else _p(hz), _p(vv), _p(w))
    return w


def spin_row(m, n_pop: int, row: int) -> Tuple[np.ndarray, np.ndarray]:
    """One sparse row (columns, values) of H by index (combinadic ranks)."""
    bi, bj, jz, jxy, hz = _spin_arrays(m)
    cols = np.empty(bi.shape[0] + 1, dtype=np.int64)
    vals = np.empty(bi.shape[0] + 1, dtype=np.float64)
    k = lib().or_spin_row_by_index(m.n_sites, n_pop, int(row), bi.shape[0], _p(bi), _p(bj),
                                   _p(jz), _p(jxy), None if hz is None else _p(hz),
                                   _p(cols), _p(vals))
    return cols[:k].copy(), vals[:k].copy()


def spin_sparse(m, states: np.ndarray) -> scipy.sparse.csr_matrix:
    bi, bj, jz, jxy, hz = _spin_arrays(m)
    dim, s = states.shape[0], bi.shape[0] + 1
    cols = np.zeros(dim * s, dtype=np.int64)
    vals = np.zeros(dim * s, dtype=np.float64)
    cnt = np.zeros(dim, dtype=np.int32)
    lib().or_spin_ell(m.n_sites, _p(states), dim, bi.shape[0], _p(bi), _p(bj), _p(jz),
                      _p(jxy), None if hz is None else _p(hz), _p(cols), _p(vals), _p(cnt))
    mask = (np.arange(s)[None, :] < cnt[:, None]).ravel()
    rows = np.repeat(np.arange(dim), s)[mask]
    return scipy.sparse.csr_matrix((vals[mask], (rows, cols[mask])), shape=(dim, dim))


def sz_table(n_sites: int, states: np.ndarray) -> np.ndarray:
    out = np.empty((states.shape[0], n_sites), dtype=np.float64)
    lib().or_spin_sz_table(n_sites, _p(states), states.shape[0], _p(out))
    return out


# ------------------------------------------------------------ Hubbard H*v --

def hubbard_basis(n_sites: int, n_up: int, n_dn: int):
    return basis_list(n_sites, n_up), basis_list(n_sites, n_dn)


def _hub_arrays(m):
    return (np.ascontiguousarray(m.hi, dtype=np.int32), np.ascontiguousarray(m.hj, dtype=np.int32),
            np.ascontiguousarray(m.t, dtype=np.float64),
            np.ascontiguousarray(m.u_site, dtype=np.float64))


def _pair_arrays(m):
    f = lambda x: np.ascontiguousarray(x, dtype=np.float64)
    return (np.ascontiguousarray(m.pi, dtype=np.int32), np.ascontiguousarray(m.pj, dtype=np.int32),
            f(m.pv), f(m.pjh), f(m.pjx), f(m.pjp))


def _n_pairs(m) -> int:
    return 0 if getattr(m, "pi", None) is None else int(len(m.pi))


def hubbard_pairs_hv(m, ups: np.ndarray, dns: np.ndarray, v: np.ndarray) -> np.ndarray:
    """H_2body v alone (Sec. 5, Eq. ham_general two-body terms)."""
    pa = _pair_arrays(m)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty_like(vv)
    lib().or_hubbard_pairs_hv(m.n_sites, _p(ups), ups.shape[0], _p(dns), dns.shape[0], pa[0].shape[0],
                              *[_p(x) for x in pa], _p(vv), _p(w))
    return w


def _complex_t(m):
    """The transfers as complex numbers t + i t_im, or None when the model
    has no imaginary parts."""
    t_im = getattr(m, "t_im", None)
    if t_im is None or not np.any(np.asarray(t_im) != 0.0):
        return None
    return np.asarray(m.t, dtype=np.float64) + 1j * np.asarray(t_im, dtype=np.float64)


def species_hopping_complex(n_sites: int, states: np.ndarray, hi, hj, tc) -> scipy.sparse.csr_matrix:
    """One species' transfer matrix for complex amplitudes: each hop
    (i, j, t) contributes -(t c+_i c_j + t* c+_j c_i) (the one-body term of
    the general Hamiltonian, Sec. 5, with the Hermitian partner written
    out). For a state s with exactly one of i, j occupied and s' = s with
    the electron moved, the element <s|.|s'> is -t when s holds i and -t*
    when s holds j, times (-1)^(occupied sites strictly between i and j)."""
    st = np.asarray(states, dtype=np.uint64)
    rows, cols, vals = [], [], []
    for h in range(len(hi)):
        i, j, t = int(hi[h]), int(hj[h]), complex(tc[h])
        bi = (st >> np.uint64(i)) & np.uint64(1)
        bj = (st >> np.uint64(j)) & np.uint64(1)
        act = np.nonzero(bi != bj)[0]
        if act.size == 0:
            continue
        s = st[act]
        s2 = s ^ (np.uint64(1 << i) | np.uint64(1 << j))
        r2 = np.searchsorted(st, s2)
        lo, hi_ = min(i, j), max(i, j)
        between = np.zeros(act.size, dtype=np.int64)
        for k in range(lo + 1, hi_):
            between += ((s >> np.uint64(k)) & np.uint64(1)).astype(np.int64)
        sign = np.where(between % 2 == 1, -1.0, 1.0)
        holds_i = bi[act] == np.uint64(1)
        coef = np.where(holds_i, -t, -np.conj(t)) * sign
        rows.append(act)
        cols.append(r2)
        vals.append(coef)
    d = st.shape[0]
    if not rows:
        return scipy.sparse.csr_matrix((d, d), dtype=np.complex128)
    return scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                   shape=(d, d), dtype=np.complex128)


def _hubbard_u_diag(m, ups, dns) -> np.ndarray:
    """sum_i U_i n_i,up n_i,dn on the up-major product basis."""
    u = np.asarray(ups, dtype=np.uint64)
    d = np.asarray(dns, dtype=np.uint64)
    diag = np.zeros((u.shape[0], d.shape[0]))
    for i in range(m.n_sites):
        ui = ((u >> np.uint64(i)) & np.uint64(1)).astype(np.float64)
        di = ((d >> np.uint64(i)) & np.uint64(1)).astype(np.float64)
        diag += float(m.u_site[i]) * ui[:, None] * di[None, :]
    return diag.reshape(-1)


def hubbard_sparse_complex(m, ups, dns) -> scipy.sparse.csr_matrix:
    """H with complex transfers: T_up (x) 1 + 1 (x) T_dn + U diagonal (+ the
    two-body terms). With all up orbitals before all down ones, a down hop
    passes every up electron twice, so its sign is that of the down species
    alone."""
    tc = _complex_t(m)
    if tc is None:
        tc = np.asarray(m.t, dtype=np.complex128)
    tu = species_hopping_complex(m.n_sites, ups, m.hi, m.hj, tc)
    td = species_hopping_complex(m.n_sites, dns, m.hi, m.hj, tc)
    H = (scipy.sparse.kron(tu, scipy.sparse.identity(len(dns)), format="csr")
         + scipy.sparse.kron(scipy.sparse.identity(len(ups)), td, format="csr")
         + scipy.sparse.diags(_hubbard_u_diag(m, ups, dns)))
    if _n_pairs(m):
        H = H + hubbard_pairs_sparse(m, ups, dns)
    return H.tocsr()


def hubbard_row_complex(m, ups, dns, ru: int, rd: int):
    """Row (ru, rd) of the complex-transfer H: columns and values."""
    tc = _complex_t(m)
    nd = len(dns)
    u, d = int(ups[ru]), int(dns[rd])
    cols = [ru * nd + rd]
    vals = [complex(sum(float(m.u_site[i]) for i in range(m.n_sites) if (u >> i) & (d >> i) & 1))]
    for h in range(m.n_hops):
        i, j, t = int(m.hi[h]), int(m.hj[h]), complex(tc[h])
        lo, hi_ = min(i, j), max(i, j)
        for sp, x in ((0, u), (1, d)):
            if ((x >> i) & 1) == ((x >> j) & 1):
                continue
            x2 = x ^ ((1 << i) | (1 << j))
            sign = -1.0 if bin(x & (((1 << hi_) - 1) & ~((2 << lo) - 1))).count("1") % 2 else 1.0
            c = (-t if (x >> i) & 1 else -np.conj(t)) * sign
            if sp == 0:
                cols.append(int(np.searchsorted(ups, x2)) * nd + rd)
            else:
                cols.append(ru * nd + int(np.searchsorted(dns, x2)))
            vals.append(c)
    cols, vals = np.array(cols, dtype=np.int64), np.array(vals, dtype=np.complex128)
    if _n_pairs(m):
        c2, v2 = hubbard_pairs_row(m, ups, dns, ru, rd)
        cols, vals = np.concatenate([cols, c2]), np.concatenate([vals, v2.astype(np.complex128)])
    return cols, vals


def hubbard_hv(m, ups: np.ndarray, dns: np.ndarray, v: np.ndarray) -> np.ndarray:
    v = np.asarray(v)
    if _complex_t(m) is not None:
        return hubbard_sparse_complex(m, ups, dns) @ v.astype(np.complex128)
    if np.iscomplexobj(v):
        return hubbard_hv(m, ups, dns, v.real) + 1j * hubbard_hv(m, ups, dns, v.imag)
    hi, hj, t, us = _hub_arrays(m)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty_like(vv)
    lib().or_hubbard_hv(m.n_sites, _p(ups), ups.shape[0], _p(dns), dns.shape[0], hi.shape[0],
                        _p(hi), _p(hj), _p(t), _p(us), _p(vv), _p(w))
    if _n_pairs(m):
        w += hubbard_pairs_hv(m, ups, dns, vv)
    return w


def hubbard_hv_rows(m, ups, dns, v: np.ndarray, ru_first: int, ru_count: int) -> np.ndarray:
    """Up-rows [ru_first, ru_first + ru_count) of H v (all down states)."""
    hi, hj, t, us = _hub_arrays(m)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty(ru_count * dns.shape[0])
    lib().or_hubbard_hv_rows(m.n_sites, _p(ups), ups.shape[0], _p(dns), dns.shape[0], hi.shape[0],
                             _p(hi), _p(hj), _p(t), _p(us), _p(vv), int(ru_first), int(ru_count), _p(w))
    if _n_pairs(m):
        pa = _pair_arrays(m)
        w2 = np.empty_like(w)
        lib().or_hubbard_pairs_hv_rows(m.n_sites, _p(ups), ups.shape[0], _p(dns), dns.shape[0], pa[0].shape[0],
                                       *[_p(x) for x in pa], _p(vv), int(ru_first), int(ru_count), _p(w2))
        w += w2
    return w


def hubbard_pairs_row(m, ups, dns, ru: int, rd: int):
    pa = _pair_arrays(m)
    s = 1 + 4 * pa[0].shape[0]
    cols = np.empty(s, dtype=np.int64)
    vals = np.empty(s, dtype=np.float64)
    k = lib().or_hubbard_pairs_row(m.n_sites, _p(ups), ups.shape[0], _p(dns), dns.shape[0], pa[0].shape[0],
                                   *[_p(x) for x in pa], int(ru), int(rd), _p(cols), _p(vals))
    return cols[:k].copy(), vals[:k].copy()


def hubbard_row(m, ups, dns, ru: int, rd: int):
    if _complex_t(m) is not None:
        return hubbard_row_complex(m, ups, dns, ru, rd)
    hi, hj, t, us = _hub_arrays(m)
    s = 2 * hi.shape[0] + 1
    cols = np.empty(s, dtype=np.int64)
    vals = np.empty(s, dtype=np.float64)
    k = lib().or_hubbard_row(m.n_sites, _p(ups), ups.shape[0], _p(dns), dns.shape[0],
                             hi.shape[0], _p(hi), _p(hj), _p(t), _p(us), int(ru), int(rd),
                             _p(cols), _p(vals))
    cols, vals = cols[:k].copy(), vals[:k].copy()
    if _n_pairs(m):
        c2, v2 = hubbard_pairs_row(m, ups, dns, ru, rd)
        cols, vals = np.concatenate([cols, c2]), np.concatenate([vals, v2])
    return cols, vals


def hubbard_sparse(m, ups, dns) -> scipy.sparse.csr_matrix:
    if _complex_t(m) is not None:
        return hubbard_sparse_complex(m, ups, dns)
    hi, hj, t, us = _hub_arrays(m)
    dim, s = ups.shape[0] * dns.shape[0], 2 * hi.shape[0] + 1
    cols = np.zeros(dim * s, dtype=np.int64)
    vals = np.zeros(dim * s, dtype=np.float64)
    cnt = np.zeros(dim, dtype=np.int32)
    lib().or_hubbard_ell(m.n_sites, _p(ups), ups.shape[0], _p(dns), dns.shape[0], hi.shape[0],
                         _p(hi), _p(hj), _p(t), _p(us), _p(cols), _p(vals), _p(cnt))
    mask = (np.arange(s)[None, :] < cnt[:, None]).ravel()
    rows = np.repeat(np.arange(dim), s)[mask]
    H = scipy.sparse.csr_matrix((vals[mask], (rows, cols[mask])), shape=(dim, dim))
    if _n_pairs(m):
        H = H + hubbard_pairs_sparse(m, ups, dns)
    return H


def hubbard_pairs_sparse(m, ups, dns) -> scipy.sparse.csr_matrix:
    pa = _pair_arrays(m)
    dim, s = ups.shape[0] * dns.shape[0], 1 + 4 * pa[0].shape[0]
    cols = np.zeros(dim * s, dtype=np.int64)
    vals = np.zeros(dim * s, dtype=np.float64)
    cnt = np.zeros(dim, dtype=np.int32)
    lib().or_hubbard_pairs_ell(m.n_sites, _p(ups), ups.shape[0], _p(dns), dns.shape[0], pa[0].shape[0],
                               *[_p(x) for x in pa], _p(cols), _p(vals), _p(cnt))
    mask = (np.arange(s)[None, :] < cnt[:, None]).ravel()
    rows = np.repeat(np.arange(dim), s)[mask]
    return scipy.sparse.csr_matrix((vals[mask], (rows, cols[mask])), shape=(dim, dim))


# ----------------------------------------------------------------- spin-S --

def spin_s_basis(n_sites: int, two_s: int, two_sz: int) -> np.ndarray:
    """Configurations of n spin-S sites (digit m_i = S^z_i + S in b-bit fields,
    b the fewest bits holding 2S) with total 2S^z = two_sz, ascending."""
    msum2 = two_sz + n_sites * two_s
    if msum2 % 2:
        raise ValueError("2Sz parity")
    msum = msum2 // 2
    n = lib().or_spin_s_basis_fill(n_sites, two_s, msum, None, 0)
    out = np.empty(max(n, 1), dtype=np.uint64)
    lib().or_spin_s_basis_fill(n_sites, two_s, msum, _p(out), n)
    return out[:n]


def _spin_s_arrays(m):
    f = lambda x: np.ascontiguousarray(x, dtype=np.float64)
    hz = f(m.hz) if m.hz is not None else None
    d = f(m.d_ion) if m.d_ion is not None else None
    return (np.ascontiguousarray(m.bi, dtype=np.int32), np.ascontiguousarray(m.bj, dtype=np.int32),
            f(m.jz), f(m.jxy), hz, d)


def _pn(a):
    return None if a is None else _p(a)


def spin_s_hv(m, states: np.ndarray, v: np.ndarray) -> np.ndarray:
    v = np.asarray(v)
    if np.iscomplexobj(v):
        return spin_s_hv(m, states, v.real) + 1j * spin_s_hv(m, states, v.imag)
    bi, bj, jz, jxy, hz, d = _spin_s_arrays(m)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty_like(vv)
    lib().or_spin_s_hv(m.n_sites, m.two_s, _p(states), states.shape[0], bi.shape[0], _p(bi), _p(bj), _p(jz),
                       _p(jxy), _pn(hz), _pn(d), _p(vv), _p(w))
    return w


def spin_s_row(m, states: np.ndarray, r: int):
    bi, bj, jz, jxy, hz, d = _spin_s_arrays(m)
    cols = np.empty(1 + 2 * bi.shape[0], dtype=np.int64)
    vals = np.empty(1 + 2 * bi.shape[0])
    k = lib().or_spin_s_row(m.n_sites, m.two_s, _p(states), states.shape[0], bi.shape[0], _p(bi), _p(bj),
                            _p(jz), _p(jxy), _pn(hz), _pn(d), int(r), _p(cols), _p(vals))
    return cols[:k].copy(), vals[:k].copy()


def spin_s_sparse(m, states: np.ndarray) -> scipy.sparse.csr_matrix:
    bi, bj, jz, jxy, hz, d = _spin_s_arrays(m)
    dim, s = states.shape[0], 1 + 2 * bi.shape[0]
    cols = np.zeros(dim * s, dtype=np.int64)
    vals = np.zeros(dim * s, dtype=np.float64)
    cnt = np.zeros(dim, dtype=np.int32)
    lib().or_spin_s_ell(m.n_sites, m.two_s, _p(states), dim, bi.shape[0], _p(bi), _p(bj), _p(jz), _p(jxy),
                        _pn(hz), _pn(d), _p(cols), _p(vals), _p(cnt))
    mask = (np.arange(s)[None, :] < cnt[:, None]).ravel()
    rows = np.repeat(np.arange(dim), s)[mask]
    return scipy.sparse.csr_matrix((vals[mask], (rows, cols[mask])), shape=(dim, dim))


# ---------------------------------------------------------------- SpinGC --

def _gc_arrays(m):
    f = lambda x: np.ascontiguousarray(x, dtype=np.float64)
    return (np.ascontiguousarray(m.bi, dtype=np.int32), np.ascontiguousarray(m.bj, dtype=np.int32),
            f(m.jx), f(m.jy), f(m.jz), f(m.hx), f(m.hz))


def spin_gc_hv(m, v: np.ndarray) -> np.ndarray:
    """H v on the full 2^N space (index = configuration, bit 1 = up)."""
    v = np.asarray(v)
    if np.iscomplexobj(v):
        return spin_gc_hv(m, v.real) + 1j * spin_gc_hv(m, v.imag)
    ga = _gc_arrays(m)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty_like(vv)
    lib().or_spin_gc_hv(m.n_sites, ga[0].shape[0], *[_p(x) for x in ga], _p(vv), _p(w))
    return w


def spin_gc_hv_rows(m, v: np.ndarray, first: int, count: int) -> np.ndarray:
    ga = _gc_arrays(m)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty(count)
    lib().or_spin_gc_hv_rows(m.n_sites, ga[0].shape[0], *[_p(x) for x in ga], _p(vv), int(first), int(count),
                             _p(w))
    return w


def spin_gc_row(m, x: int):
    ga = _gc_arrays(m)
    cap = 1 + 3 * ga[0].shape[0] + m.n_sites
    cols = np.empty(cap, dtype=np.int64)
    vals = np.empty(cap, dtype=np.float64)
    k = lib().or_spin_gc_row(m.n_sites, ga[0].shape[0], *[_p(a) for a in ga], ctypes.c_uint64(int(x)),
                             _p(cols), _p(vals))
    return cols[:k].copy(), vals[:k].copy()


def spin_gc_sparse(m) -> scipy.sparse.csr_matrix:
    ga = _gc_arrays(m)
    dim, s = 1 << m.n_sites, 1 + 3 * ga[0].shape[0] + m.n_sites
    cols = np.zeros(dim * s, dtype=np.int64)
    vals = np.zeros(dim * s, dtype=np.float64)
    cnt = np.zeros(dim, dtype=np.int32)
    lib().or_spin_gc_ell(m.n_sites, ga[0].shape[0], *[_p(x) for x in ga], _p(cols), _p(vals), _p(cnt))
    mask = (np.arange(s)[None, :] < cnt[:, None]).ravel()
    rows = np.repeat(np.arange(dim), s)[mask]
    return scipy.sparse.csr_matrix((vals[mask], (rows, cols[mask])), shape=(dim, dim))


# ----------------------------------------------------------------- random --

def splitmix_u64(seed: int, first: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    lib().or_splitmix_u64(ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), first, n, _p(out))
    return out


def splitmix_uniform(seed: int, first: int, n: int) -> np.ndarray:
    """Uniform [-1/2, 1/2) from SplitMix64 outputs (top 53 bits)."""
    out = np.empty(n, dtype=np.float64)
    lib().or_splitmix_uniform(ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), first, n, _p(out))
    return out


def splitmix_complex_gaussian(seed: int, n: int) -> np.ndarray:
    """Element i = sqrt(-2 ln u1) * exp(2 pi i u2) (Box-Muller), u1 in (0, 1]
    and u2 in [0, 1) from outputs 2i and 2i+1 of the stream."""
    z = splitmix_u64(seed, 0, 2 * n)
    u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2 * np.pi * u2) + 1j * r * np.sin(2 * np.pi * u2)


# ---------------------------------------------------------------- Lanczos --

def lanczos(hv: Callable[[np.ndarray], np.ndarray], v0: np.ndarray, n_iter: int,
            breakdown: float = 1e-13) -> Dict[str, np.ndarray]:
    """Plain Lanczos tridiagonalization (Sec. 1: the Krylov method built on
    repeated H*v), no reorthogonalization:
        v_0 = r / |r|, beta_0 = 0;
        w = H v_k - beta_k v_{k-1}; alpha_k = <v_k, w>; w -= alpha_k v_k;
        beta_{k+1} = |w|; stop if beta_{k+1} <= 1e-13 max(1, |alpha_k|);
        v_{k+1} = w / beta_{k+1}.
    Returns alpha (k), beta (k, beta[0] = 0 and beta[k] couples k-1, k) and
    the number of steps done."""
    v = np.asarray(v0, dtype=np.float64) / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    alpha, beta = [], [0.0]
    b = 0.0
    for k in range(n_iter):
        w = hv(v) - b * v_prev
        a = float(np.dot(v, w))
        w = w - a * v
        alpha.append(a)
        b = float(np.linalg.norm(w))
        if k + 1 == n_iter:
            break
        if b <= breakdown * max(1.0, abs(a)):
            break
        beta.append(b)
        v_prev, v = v, w / b
    # beta_full also holds the norm after the last step (a residual estimate)
    return {"alpha": np.array(alpha), "beta": np.array(beta[:len(alpha)]),
            "beta_full": np.array(beta[:len(alpha)] + [b]), "steps": len(alpha)}


def lanczos_stop(alpha: np.ndarray, beta_full: np.ndarray, check_every: int, tol: float,
                 resid_tol: float = 0.0) -> int:
    """Step count at which a checked Lanczos run stops: every check_every
    steps m the lowest Ritz value theta_m of T_m is compared with the
    previous check's, and the run stops at the first m where it moved by
    less than tol max(1, |theta_m|) and (resid_tol > 0) the residual
    estimate beta_m |s_{m-1}| of the lowest Ritz pair (s its eigenvector of
    T_m) is below resid_tol max(1, |theta_m|). beta_full[m] must be the
    norm after step m (beta_full[0] = 0). Returns len(alpha) if no check
    passes."""
    last = None
    for m in range(check_every, len(alpha) + 1, check_every):
        th, s = scipy.linalg.eigh_tridiagonal(alpha[:m], beta_full[1:m], select="i", select_range=(0, 0))
        th = float(th[0])
        ok = last is not None and abs(th - last) < tol * max(1.0, abs(th))
        if ok and resid_tol > 0:
            ok = m < len(beta_full) and beta_full[m] * abs(s[m - 1, 0]) < resid_tol * max(1.0, abs(th))
        if ok:
            return m
        last = th
    return len(alpha)


def tridiag_lowest(alpha: np.ndarray, beta: np.ndarray, k: int = 1) -> np.ndarray:
    """Lowest k eigenvalues of the Lanczos tridiagonal (LAPACK via scipy);
    beta[1:] are the off-diagonals."""
    ev = scipy.linalg.eigh_tridiagonal(alpha, beta[1:], eigvals_only=True,
                                       select="i", select_range=(0, min(k, len(alpha)) - 1))
    return np.asarray(ev)


def lanczos_ground_vector(hv, v0, alpha, beta) -> np.ndarray:
    """Second pass: repeat the recurrence with the same start vector and
    accumulate psi = sum_k s_k v_k with s the lowest eigenvector of T."""
    n = len(alpha)
    _, s = scipy.linalg.eigh_tridiagonal(alpha, beta[1:], select="i", select_range=(0, 0))
    s = s[:, 0]
    v = np.asarray(v0, dtype=np.float64) / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    psi = s[0] * v
    for k in range(n - 1):
        w = hv(v) - beta[k] * v_prev - alpha[k] * v
        v_prev, v = v, w / beta[k + 1]
        psi = psi + s[k + 1] * v
    return psi / np.linalg.norm(psi)


# ------------------------------------------------------------------- cTPQ --

def ctpq(hv: Callable[[np.ndarray], np.ndarray], phi0: np.ndarray, n_max: int,
         dtau: float, k_steps: int) -> Dict[str, np.ndarray]:
    """Canonical TPQ (Sec. 3.5.1): Phi_k = U_c(dtau)^k Phi_rand with
    U_c = sum_{n=0}^{n_max} (1/n!) (-dtau H / 2)^n applied term by term.
    Squared norms: N_0 = <Phi_rand|Phi_rand>, D_0 = N_0, D_k = N_k / N_{k-1};
    the state is renormalized after each step (so D_k is the squared norm of
    U_c applied to the normalized previous state). At each beta_k = k dtau the
    energy <H> = <Phi|H Phi> / <Phi|Phi> and <H^2> = |H Phi|^2 / <Phi|Phi> are
    recorded. Works column by column for a block (dim, B)."""
    phi = np.array(phi0, dtype=np.complex128)
    single = phi.ndim == 1
    if single:
        phi = phi[:, None]

    def H(x):
        return np.stack([hv(x[:, c]) for c in range(x.shape[1])], axis=1)

    B = phi.shape[1]
    Dk = np.zeros((k_steps + 1, B))
    E = np.zeros((k_steps + 1, B))
    E2 = np.zeros((k_steps + 1, B))
    n0 = np.sum(np.abs(phi) ** 2, axis=0).real
    Dk[0] = n0
    phi = phi / np.sqrt(n0)
    hp = H(phi)
    E[0] = np.real(np.sum(np.conj(phi) * hp, axis=0))
    E2[0] = np.sum(np.abs(hp) ** 2, axis=0).real
    for k in range(1, k_steps + 1):
        term = phi.copy()
        acc = phi.copy()
        for n in range(1, n_max + 1):
            term = (-dtau / 2.0 / n) * H(term)
            acc = acc + term
        nk = np.sum(np.abs(acc) ** 2, axis=0).real
        Dk[k] = nk
        phi = acc / np.sqrt(nk)
        hp = H(phi)
        E[k] = np.real(np.sum(np.conj(phi) * hp, axis=0))
        E2[k] = np.sum(np.abs(hp) ** 2, axis=0).real
    beta = dtau * np.arange(k_steps + 1)
    out = {"beta": beta, "D": Dk, "E": E, "E2": E2, "phi": phi[:, 0] if single else phi}
    return out


# ----------------------------------------------------- S^zz(q, w) / D(z) --

def szq_excitation(m, states: np.ndarray, q: float, psi: np.ndarray) -> np.ndarray:
    """Phi_ex = sum_l e^{i q x_l} S^z_l Phi_GS (Sec. 3.2, with S^z_l diagonal,
    +-1/2 by the bit of site l; x_l the site's coordinate along the chain or
    the ladder's legs)."""
    sz = sz_table(m.n_sites, states)
    phase = np.exp(1j * q * np.asarray(m.site_x, dtype=np.float64))
    return (sz @ phase) * psi


def hubbard_szq_excitation(m, ups: np.ndarray, dns: np.ndarray, q: float,
                           psi: np.ndarray) -> np.ndarray:
    """Phi_ex = sum_l e^{i q x_l} S^z_l Phi_GS on the Hubbard basis (Sec. 3.2),
    S^z_l = (n_l,up - n_l,dn) / 2, state index r_up * dim_dn + r_dn; x_l the
    site coordinate (site number when the model gives none)."""
    n = m.n_sites
    sx = getattr(m, "site_x", None)
    x = np.arange(n, dtype=np.float64) if sx is None else np.asarray(sx, dtype=np.float64)
    l = np.arange(n, dtype=np.uint64)
    nu = ((np.asarray(ups, dtype=np.uint64)[:, None] >> l) & np.uint64(1)).astype(np.float64)
    nd = ((np.asarray(dns, dtype=np.uint64)[:, None] >> l) & np.uint64(1)).astype(np.float64)
    sz = 0.5 * (nu[:, None, :] - nd[None, :, :]).reshape(-1, n)
    return (sz @ np.exp(1j * q * x)) * psi


def dyn_corr_direct(Hs, b: np.ndarray, zs: np.ndarray) -> np.ndarray:
    """D(z) = <b| (z I - H)^-1 |b> by one sparse direct solve per z
    (Sec. 3.2 definition; no E0 offset, no 1/pi)."""
    dim = Hs.shape[0]
    I = scipy.sparse.identity(dim, dtype=np.complex128, format="csc")
    Hc = Hs.astype(np.complex128).tocsc()
    out = np.empty(len(zs), dtype=np.complex128)
    for k, z in enumerate(zs):
        x = scipy.sparse.linalg.spsolve(z * I - Hc, b.astype(np.complex128))
        out[k] = np.vdot(b, x)
    return out


def dyn_corr_spectral(Hd: np.ndarray, b: np.ndarray, zs: np.ndarray) -> np.ndarray:
    """Same quantity from the full spectrum: sum_n |<n|b>|^2 / (z - E_n)."""
    E, U = np.linalg.eigh(Hd)
    wts = np.abs(U.T.conj() @ b) ** 2
    return np.array([np.sum(wts / (z - E)) for z in zs])


def continued_fraction(alpha: np.ndarray, beta: np.ndarray, norm2: float,
                       zs: np.ndarray) -> np.ndarray:
    """Lanczos continued fraction D(z) = |b|^2 / (z - a_0 - b_1^2 / (z - a_1 - ...))
    (Sec. 3.2, method="Lanczos")."""
    out = np.empty(len(zs), dtype=np.complex128)
    for k, z in enumerate(zs):
        g = 0.0 + 0.0j
        for j in range(len(alpha) - 1, 0, -1):
            g = beta[j] ** 2 / (z - alpha[j] - g)
        out[k] = norm2 / (z - alpha[0] - g)
    return out


def lanczos_complex(hv, b: np.ndarray, n_iter: int):
    """Hermitian Lanczos on a complex start vector (for the continued
    fraction); returns alpha, beta with beta[0] = 0."""
    v = b / np.linalg.norm(b)
    v_prev = np.zeros_like(v)
    alpha, beta = [], [0.0]
    bb = 0.0
    for k in range(n_iter):
        w = hv(v) - bb * v_prev
        a = float(np.real(np.vdot(v, w)))
        w = w - a * v
        alpha.append(a)
        bb = float(np.linalg.norm(w))
        if k + 1 == n_iter or bb < 1e-14:
            break
        beta.append(bb)
        v_prev, v = v, w / bb
    return np.array(alpha), np.array(beta[:len(alpha)])


def taylor_evolve(hv: Callable[[np.ndarray], np.ndarray], psi0: np.ndarray, n_max: int, dt: float,
                  n_steps: int, weight: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Real-time evolution (Sec. 3.4): psi(t + dt) = sum_{n=0}^{n_max}
    (1/n!) (-i H dt)^n psi(t), summed term by term (t_n = (-i dt / n) H t_{n-1}).
    Records at t_k = k dt the norm <psi|psi>, the energy <psi|H|psi> / <psi|psi>
    and, with a diagonal weight w_x (e.g. the count of doubly occupied sites
    divided by N_s), <psi|w|psi> / <psi|psi>. psi0: (dim,) or (dim, B)."""
    return taylor_evolve_td(lambda k: hv, psi0, n_max, dt, n_steps, weight)


def taylor_evolve_td(hv_at: Callable[[int], Callable[[np.ndarray], np.ndarray]], psi0: np.ndarray, n_max: int,
                     dt: float, n_steps: int, weight: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """The same with a time-dependent H (Sec. 3.4, H(t) in the Schroedinger
    equation): hv_at(k) applies H(t_k). The step from t_k to t_{k+1} sums the
    Taylor series of exp(-i H(t_k) dt), i.e. H is held at its value at the
    start of the step, and the energy recorded at t_k is <H(t_k)>."""
    psi = np.array(psi0, dtype=np.complex128)
    if psi.ndim == 1:
        psi = psi[:, None]
    nrm, en, ob = [], [], []
    for k in range(n_steps + 1):
        hv = hv_at(k)
        hp = np.stack([hv(psi[:, j]) for j in range(psi.shape[1])], axis=1)
        n2 = np.real(np.sum(np.conj(psi) * psi, axis=0))
        nrm.append(n2)
        en.append(np.real(np.sum(np.conj(psi) * hp, axis=0)) / n2)
        if weight is not None:
            ob.append(np.real(np.sum(weight[:, None] * np.abs(psi) ** 2, axis=0)) / n2)
        if k == n_steps:
            break
        term = psi.copy()
        new = psi.copy()
        for n in range(1, n_max + 1):
            term = np.stack([hv(term[:, j]) for j in range(term.shape[1])], axis=1) * (-1j * dt / n)
            new = new + term
        psi = new
    out = {"norm": np.array(nrm), "energy": np.array(en), "psi": psi}
    if weight is not None:
        out["obs"] = np.array(ob)
    return out


def hubbard_double_occupancy_weight(ups: np.ndarray, dns: np.ndarray, n_sites: int) -> np.ndarray:
    """Diagonal of (1/N_s) sum_i n_i,up n_i,dn on the up-major product basis."""
    cnt = np.array([[bin(int(u) & int(d)).count("1") for d in dns] for u in ups], dtype=np.float64)
    return cnt.reshape(-1) / n_sites


def canonical_thermo(evals: np.ndarray, betas: np.ndarray, n_sites: int) -> Dict[str, np.ndarray]:
    """Exact canonical energy, specific heat and entropy per site from a full
    spectrum (the quantities the TPQ states estimate, Sec. 3.5.1):
    Z = sum_n e^{-beta E_n}, E = <E>, C = beta^2 (<E^2> - <E>^2), S = ln Z + beta E."""
    ev = np.asarray(evals, dtype=np.float64)
    e0 = ev.min()
    out = {"E": [], "C": [], "S": []}
    for b in np.asarray(betas, dtype=np.float64):
        wts = np.exp(-b * (ev - e0))
        z = wts.sum()
        e = float((wts * ev).sum() / z)
        e2 = float((wts * ev * ev).sum() / z)
        out["E"].append(e / n_sites)
        out["C"].append(b * b * (e2 - e * e) / n_sites)
        out["S"].append((np.log(z) - b * e0 + b * e) / n_sites)
    return {k: np.array(v) for k, v in out.items()}
