"""Finite-temperature and spectral post-processing of the device results.

Everything here works on the scalars the C ABI returns (relative squared
norms D_k, <H>, <H^2> per TPQ vector; Lanczos alpha/beta); the vectors stay
on the device and every H*v runs in the HIP library.

  * tpq_bootstrap / tpq_thermo: the bootstrap of the HPhi update paper
    (Sec. 3.5.1): M samples of P of the N initial vectors drawn with
    replacement; sample m gives <A>_m(beta_k) = sum_p N_k^p <A>^p_k /
    sum_p N_k^p with the squared norms N_k = prod_{l<=k} D_l, normalized by
    the zeroth vector's norm to stay finite; mean and standard deviation
    over the M samples. Energy E = <H>, specific heat C = beta^2 (<H^2> -
    <H>^2), entropy S = ln Z + beta E with Z(beta_k) = d_H sum_p N_k^p /
    sum_p N_0^p.
  * mtpq: microcanonical TPQ states (Sec. 3.5.1): U_m = 1 - (dtau/2) H with
    dtau = 2 / (l N_s) is the first-order canonical step, so the states come
    from the device cTPQ routine with n_max = 1; beta_k = k dtau / (1 - u_k / l)
    with u_k = <H>_k / N_s (per vector).
  * lanczos_spectrum: the Lanczos continued fraction for D(z) =
    <b|(z - H)^-1|b> from a real excitation b (Sec. 3.2, method "Lanczos").
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np


def _log_norms(D: np.ndarray) -> np.ndarray:
    """log N_k per vector from the relative squared norms (rows k, columns j)."""
    return np.cumsum(np.log(np.asarray(D, dtype=np.float64)), axis=0)


def tpq_bootstrap(D: np.ndarray, A: np.ndarray, n_boot: int = 200, n_pick: Optional[int] = None,
                  seed: int = 0) -> Dict[str, np.ndarray]:
    """Bootstrap mean and error of <A>(beta_k) from per-vector normalized
    expectations A[k, j] and relative squared norms D[k, j]."""
    D = np.asarray(D, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    n = D.shape[1]
    p = n if n_pick is None else int(n_pick)
    logn = _log_norms(D)
    w = np.exp(logn - logn[:, :1])          # N_k^j / N_k^0
    rng = np.random.default_rng(seed)
    samples = np.empty((n_boot, D.shape[0]))
    for m in range(n_boot):
        idx = rng.integers(0, n, p)
        samples[m] = np.sum(w[:, idx] * A[:, idx], axis=1) / np.sum(w[:, idx], axis=1)
    return {"mean": samples.mean(axis=0), "err": samples.std(axis=0, ddof=1) if n_boot > 1 else
            np.zeros(D.shape[0]), "all": np.sum(w * A, axis=1) / np.sum(w, axis=1)}


def tpq_thermo(beta: np.ndarray, D: np.ndarray, E: np.ndarray, E2: np.ndarray, dim: int, n_sites: int,
               n_boot: int = 200, n_pick: Optional[int] = None, seed: int = 0) -> Dict[str, np.ndarray]:
    """Energy, specific heat and entropy per site with bootstrap errors from
    canonical TPQ results (beta_k common to all vectors)."""
    D = np.asarray(D, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    E2 = np.asarray(E2, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    n = D.shape[1]
    p = n if n_pick is None else int(n_pick)
    logn = _log_norms(D)
    ref = logn[:, :1]
    w = np.exp(logn - ref)
    rng = np.random.default_rng(seed)
    es, cs, ss = [], [], []
    for m in range(n_boot):
        idx = rng.integers(0, n, p)
        z = np.sum(w[:, idx], axis=1)
        e = np.sum(w[:, idx] * E[:, idx], axis=1) / z
        e2 = np.sum(w[:, idx] * E2[:, idx], axis=1) / z
        # ln Z(beta_k) = ln d_H + ln(sum_p N_k^p) - ln(sum_p N_0^p)
        lnz = np.log(dim) + np.log(z) + ref[:, 0] - (np.log(z[0]) + ref[0, 0])
        es.append(e / n_sites)
        cs.append(beta ** 2 * (e2 - e * e) / n_sites)
        ss.append((lnz + beta * e) / n_sites)
    out = {"beta": beta}
    for key, arr in (("E", es), ("C", cs), ("S", ss)):
        a = np.array(arr)
        out[key] = a.mean(axis=0)
        out[key + "_err"] = a.std(axis=0, ddof=1) if n_boot > 1 else np.zeros(len(beta))
    return out


def mtpq(api, ham, n_vec: int, l: float, k_steps: int, n_sites: int, storage: str = "c128", seed: int = 1,
         phi0=None) -> Dict[str, np.ndarray]:
    """Microcanonical TPQ sequence: states from the device (first-order
    canonical steps with dtau = 2 / (l N_s)), inverse temperatures per
    vector beta_k = k dtau / (1 - u_k / l)."""
    if not l > 0:
        raise ValueError("l must be positive and above the largest energy per site")
    dtau = 2.0 / (l * n_sites)
    r = api.ctpq(ham, n_vec, 1, dtau, k_steps, storage=storage, seed=seed, phi0=phi0)
    u = r["E"] / n_sites
    k = np.arange(k_steps + 1, dtype=np.float64)[:, None]
    beta = k * dtau / (1.0 - u / l)
    return {"beta": beta, "u": u, "D": r["D"], "E": r["E"], "E2": r["E2"], "dtau": dtau, "phi": r["phi"]}


def continued_fraction(alpha: Sequence[float], beta: Sequence[float], norm2: float,
                       z: Sequence[complex]) -> np.ndarray:
    """D(z) = |b|^2 / (z - a_0 - b_1^2 / (z - a_1 - ...)) from a Lanczos
    tridiagonal started at b / |b| (beta[0] unused)."""
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    z = np.asarray(z, dtype=np.complex128)
    g = np.zeros_like(z)
    for j in range(len(a) - 1, 0, -1):
        g = b[j] ** 2 / (z - a[j] - g)
    return norm2 / (z - a[0] - g)


def lanczos_spectrum(api, ham, b, n_iter: int, z: Sequence[complex]) -> Dict[str, np.ndarray]:
    """D(z) for a real excitation b (device FP64 vector): Lanczos from
    b / |b| on the device, continued fraction on the host."""
    import torch
    if b.dtype != torch.float64:
        raise ValueError("the Lanczos continued fraction takes a real FP64 excitation")
    norm2 = float(torch.dot(b, b))
    if norm2 == 0.0:
        return {"D": np.zeros(len(z), dtype=np.complex128), "iterations": 0}
    r = api.lanczos(ham, n_iter, v0=b)
    return {"D": continued_fraction(r["alpha"], r["beta"], norm2, z), "iterations": r["iterations"],
            "alpha": r["alpha"], "beta": r["beta"]}
