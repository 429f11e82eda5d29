"""Benchmark: matrix-free H*v inside plain Lanczos on one MI355X.

Workload (default): Fermi-Hubbard model on the 4x4 periodic square lattice,
t = 1, U = 4, N_up = N_dn = 8 (dim 12870^2 = 165,636,900), real FP64
vectors, Lanczos ground state with 300 iterations from a seeded uniform
[-1/2, 1/2) start vector. One step = one full Lanczos solve (start vector,
300 fused H*v + update iterations, host tridiagonal eigensolve). Basis,
tables and vectors are resident on the device before the timed region.

Prints one JSON line: value = effective H*v bandwidth (algorithmic bytes:
read v + write w, 16 B per state) over the H*v launches timed with HIP
events inside the timed solves; Lanczos solves/s and per-solve p50/p99;
roofline of the H*v; the oracle's CPU rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--iters", type=int, default=300)
    p.add_argument("--workload", default="hubbard4x4", choices=["hubbard4x4", "heisenberg16"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-tune", action="store_true", help="keep the default launch schedule")
    p.add_argument("--retune", action="store_true", help="sweep schedules even if one is recorded")
    p.add_argument("--cpu-sample-rows", type=int, default=0,
                   help="oracle sample size in up-rows (0 = all rows, one full H*v)")
    return p.parse_args()


def cpu_baseline(workload: str, sample_rows: int):
    """The oracle's row-wise H*v (plain C, OpenMP) on a bounded sample of
    the same workload, reported in the same unit as `value` (GB/s of
    algorithmic H*v bytes)."""
    from oracle import core as O
    from paper_2307_13222_amd import workloads as W
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    if workload == "hubbard4x4":
        m = W.hubbard_square(4, 4, 1.0, 4.0)
        ups, dns = O.hubbard_basis(16, 8, 8)
        # rows of the sample: all down states of the first nu up states; the
        # gathers still read the whole vector
        nu = sample_rows if sample_rows > 0 else 3000
        nu = min(nu, len(ups))
        v = np.random.default_rng(0).random(len(ups) * len(dns)) - 0.5
        t0 = time.perf_counter()
        w = O.hubbard_hv_rows(m, ups, dns, v, 0, nu)
        dt = time.perf_counter() - t0
        states = nu * len(dns)
        del w
        sample = (f"oracle Hubbard H*v over up-rows [0, {nu}) of {len(ups)} "
                  f"({states} of {len(ups) * len(dns)} states)")
    else:
        m = W.heisenberg_chain(16)
        s = O.basis_list(16, 8)
        v = np.random.default_rng(0).random(len(s)) - 0.5
        reps = 50
        t0 = time.perf_counter()
        for _ in range(reps):
            O.spin_hv(m, s, v)
        dt = time.perf_counter() - t0
        states = reps * len(s)
        sample = f"oracle spin H*v x{reps} on dim {len(s)}"
    gbs = 16.0 * states / dt / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": sample, "seconds": round(dt, 3)}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {a.gpus} is not supported by this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2307_13222_amd import api, workloads as W

    ctx = api.Context(0)
    if a.workload == "hubbard4x4":
        m = W.hubbard_square(4, 4, 1.0, 4.0)
        basis = api.Basis.hubbard(ctx, 16, 8, 8)
        ham = api.Hamiltonian.hubbard(basis, m)
        wl = {"workload": "hubbard_4x4_pbc_t1_U4_half_filling", "dim": basis.dim, "lanczos_iters": a.iters,
              "storage": "f64", "lattice": "square 4x4", "n_up": 8, "n_dn": 8}
    else:
        m = W.heisenberg_chain(16)
        basis = api.Basis.spin(ctx, 16, 0)
        ham = api.Hamiltonian.spin(basis, m)
        wl = {"workload": "heisenberg_chain16_sz0", "dim": basis.dim, "lanczos_iters": a.iters,
              "storage": "f64"}
    dim = basis.dim
    stream = torch.cuda.current_stream()
    tuned = None
    if not a.no_tune:
        # schedule sweep (or cached lookup) outside the timed region
        from paper_2307_13222_amd import autotune
        tuned = autotune.tune(ham, "f64", 1, force=a.retune)
        wl["schedule"] = tuned["schedule"]
        if tuned.get("swept"):
            print(json.dumps({"autotune": tuned}), file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        api.lanczos(ham, a.iters, seed=1, stream=stream)
    torch.cuda.synchronize()
    lat, hv_s, hv_n, energies = [], 0.0, 0, []
    t0 = time.perf_counter()
    for k in range(a.steps):
        s0 = time.perf_counter()
        r = api.lanczos(ham, a.iters, seed=1 + k, stream=stream, time_kernels=True)
        lat.append(time.perf_counter() - s0)
        hv_s += r["hv_seconds"]
        hv_n += r["hv_calls"]
        energies.append(float(r["energies"][0]))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    hv_avg = hv_s / max(1, hv_n)
    alg_bytes = 16.0 * dim                      # read v + write w, FP64
    gbs = alg_bytes / hv_avg / 1e9
    out = {
        "metric": "H·v HBM GB/s (% peak) + Lanczos solves/s, p50/p99; batched/FP32 vs plain FP64",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * total / a.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": wl,
        "hbm_peak_frac": round(gbs / HBM_PEAK_GBS, 4),
        "lanczos_solves_per_s": round(a.steps / total, 4),
        "solve_ms_p50": round(1e3 * float(np.percentile(lat, 50)), 3),
        "solve_ms_p99": round(1e3 * float(np.percentile(lat, 99)), 3),
        "hv_ms_avg": round(1e3 * hv_avg, 5),
        "e0": energies[0],
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "H*v (k_hub_rows + k_hub_cols)", "alg_bytes_per_launch": alg_bytes},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.workload, a.cpu_sample_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
