"""Benchmark: matrix-free H*v inside plain Lanczos / cTPQ on one MI355X.

Default workload (the headline configuration): Fermi-Hubbard model on the 4x4
periodic square lattice, t = 1, U = 4, N_up = N_dn = 8 (dim 12870^2 =
165,636,900), real FP64 vectors, Lanczos ground state with 300 iterations
from a seeded uniform [-1/2, 1/2) start vector. One step = one full Lanczos
solve (start vector, 300 fused H*v + update iterations, host tridiagonal
eigensolve). Basis, tables and vectors are resident on the device before the
timed region.

Prints one JSON line: value = effective H*v bandwidth (algorithmic bytes:
read v + write w, 16 B per state in FP64) over the H*v launches timed with
HIP events inside the timed solves; Lanczos solves/s and per-solve p50/p99;
the roofline of the H*v; the oracle's CPU rate on a bounded sample.

Other workloads (--workload), reported the same way:
  heisenberg16  spin-1/2 Heisenberg ring N = 16 (dim 12870), 200 iterations
  ctpq_xxz28    16 TPQ vectors, XXZ (1.0, 0.8) + J2 (0.5, 0.4) ring N = 28
                (dim 40,116,600), complex FP32 storage, n_max 6, dtau 0.02;
                error vs the same run in complex FP64
  j1j2_6x6      J1-J2 Heisenberg 6x6 (J2 = 0.5), dim 9,075,135,300, FP32
                Lanczos vectors (36.3 GB each); E0 vs an FP64-storage run
  tevol_hubbard16  interaction quench of the half-filled 16-site Hubbard ring
                (dim 165,636,900): U = 0 ground state (Lanczos), then real-time
                steps with U = 8 (Taylor order 10, dt 0.01), complex FP64;
                one step = 10 complex H*v; norm and energy drift reported
  tevol_ramp_hubbard16  the same with a time-dependent H: U(t) rising
                linearly from 0 to 8 over the warmup and timed steps (one
                frame per step); the energy change checked against the
                work (U_k+1 - U_k) N_s <D>, and the cost of the frame
                switches against the same steps with one frame held
  tevol_pulse_hubbard16  the U = 4 ring's ground state driven by a light
                pulse: Peierls phases e^{i A(t)(x_i - x_j)} on the transfers
                (complex amplitudes, one frame per step)
  lobpcg_hubbard3x4  lowest 4 (+2 guard) eigenpairs of the 3x4 periodic Hubbard
                lattice at half filling (U = 4, dim 853,776) by LOBPCG with the
                point-Jacobi preconditioner; energies vs a long Lanczos
  ext_hubbard4x4  the 4x4 workload with the two-body terms of the general
                Hamiltonian in Wannier form (nearest-neighbour V = 1 and
                J = 0.3 in the Hund, exchange and pair-hopping terms), Lanczos
                300 iterations, FP64; the pair-term kernel's share reported
  tfim_ring28   transverse-field Ising ring N = 28 at g = 1 on the full 2^28
                space (SpinGC), Lanczos 100 iterations, FP64
  spin1_chain18 S = 1 Heisenberg ring N = 18, S^z = 0 (spin-S basis),
                Lanczos 200 iterations, FP64
  serving_mix   continuous batching of a request stream: half ground states,
                half S(q, w) (64 shifts, eta 0.05); Heisenberg chains and
                2-leg ladders, N in 12..26, random bonds J ~ U[0.5, 1.5];
                capacity (all requests queued at t = 0), then Poisson
                arrivals at 0.5 / 0.8 / 0.95 of it: p50/p99 latency
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
METRIC = "H·v HBM GB/s (% peak) + Lanczos solves/s, p50/p99; batched/FP32 vs plain FP64"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--iters", type=int, default=0, help="Krylov / TPQ steps per solve (0 = workload default)")
    p.add_argument("--workload", default="hubbard4x4",
                   choices=["hubbard4x4", "heisenberg16", "ctpq_xxz28", "j1j2_6x6", "serving_mix", "tevol_hubbard16",
                            "tevol_ramp_hubbard16", "tevol_pulse_hubbard16",
                            "lobpcg_hubbard3x4", "copy_probe", "ext_hubbard4x4", "tfim_ring28", "spin1_chain18"])
    p.add_argument("--requests", type=int, default=64, help="requests per serving run (serving_mix)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-refine", action="store_true",
                   help="j1j2_6x6: skip the untimed FP32 solve with the FP64 Rayleigh quotient")
    p.add_argument("--tune", action="store_true",
                   help="run the schedule autotuner first (default: the built-in schedule)")
    p.add_argument("--no-tune", action="store_true", help="keep the built-in launch schedule (the default)")
    p.add_argument("--retune", action="store_true", help="with --tune: sweep even if a schedule is recorded")
    p.add_argument("--cpu-sample-rows", type=int, default=0,
                   help="oracle sample size in up-rows (hubbard4x4)")
    p.add_argument("--schedule", default="",
                   help='JSON launch-schedule fields applied before timing, e.g. \'{"hub_sweep": 5}\'')
    a = p.parse_args()
    a.no_tune = a.no_tune or not a.tune
    return a


# HBM traffic of one Lanczos step of the 4x4 Hubbard workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch of the
# column kernel and of the rows kernel) scaled by the factors a plain 2 GiB device copy gives for the same
# counters (fetch 2.000, write 1.000). Valid only for the kernel sources and
# schedule it was taken with; anything else reports null.
HUB_TRAFFIC = {
    "sources_sha256": {"kern_hub.hip": "42fc06a1a42b002c35186ffd15f1f1b753f7627bbc42aa52d0d887972d392111",
                       "kern_common.h": "82a4da084e46d3f069fff2bbec75262cce5cf6131077ca6b4d166d41e8c25fce"},
    "schedule": {"hub_slab_cols": 128, "hub_groups": 128, "hub_item_rows": 16, "hub_row_cols": 6, "hub_sweep": 7,
                 "hub_row_order": 2, "hub_tile_bits": 0},
    "cols_fetch_kib": 3.359620e+06, "cols_write_kib": 1.361091e+06,
    "rows_fetch_kib": 1.456485e+06, "rows_write_kib": 2.588495e+06,
    "fetch_factor": 2.0, "write_factor": 1.0,
}

def hub_traffic(schedule, which: str = "pair") -> float:
    """Measured HBM bytes per launch of the column kernel ("cols") or of the
    rows + column launch pair ("pair"), or None when the kernel sources or
    the schedule differ from those the counters were taken on."""
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2307_13222_amd", "csrc")
    for f, h in HUB_TRAFFIC["sources_sha256"].items():
        with open(os.path.join(src, f), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != h:
                return None
    if any(schedule.get(k) != v for k, v in HUB_TRAFFIC["schedule"].items()):
        return None
    t = HUB_TRAFFIC
    fetch = t["cols_fetch_kib"] + (t["rows_fetch_kib"] if which == "pair" else 0.0)
    write = t["cols_write_kib"] + (t["rows_write_kib"] if which == "pair" else 0.0)
    return 1024.0 * (fetch * t["fetch_factor"] + write * t["write_factor"])


def omp_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()


def cpu_baseline(workload: str, sample_rows: int):
    """The oracle's row-wise H*v (plain C, OpenMP) on a bounded sample of
    the same workload, in the same unit as `value` (GB/s of algorithmic H*v
    bytes)."""
    from oracle import core as O
    from paper_2307_13222_amd import workloads as W
    if workload == "hubbard4x4":
        m = W.hubbard_square(4, 4, 1.0, 4.0)
        ups, dns = O.hubbard_basis(16, 8, 8)
        # all down states of the first nu up states (default: every up
        # state, one whole H*v, about 11 s on 16 threads); gathers read the
        # whole vector
        nu = min(sample_rows if sample_rows > 0 else len(ups), len(ups))
        v = np.random.default_rng(0).random(len(ups) * len(dns)) - 0.5
        t0 = time.perf_counter()
        w = O.hubbard_hv_rows(m, ups, dns, v, 0, nu)
        dt = time.perf_counter() - t0
        states, bytes_per = nu * len(dns), 16.0
        sample = (f"oracle Hubbard H*v over up-rows [0, {nu}) of {len(ups)} "
                  f"({states} of {len(ups) * len(dns)} states)")
        # the vector work of one oracle Lanczos step on full-size vectors
        # (numpy), for the time-to-E0 extrapolation
        u = np.random.default_rng(1).random(len(v)) - 0.5
        t1 = time.perf_counter()
        w -= 0.5 * u
        al = float(np.dot(v, w))
        w -= al * v
        bt = float(np.linalg.norm(w))
        u = w / bt
        t_vec = time.perf_counter() - t1
        del w, u
        t_hv_full = dt * len(ups) / nu
        # one core: the same row formula over a sixteenth of the rows
        n1 = max(1, len(ups) // 16)
        try:
            import ctypes
            gomp = ctypes.CDLL("libgomp.so.1")
            gomp.omp_set_num_threads(1)
            t2 = time.perf_counter()
            O.hubbard_hv_rows(m, ups, dns, v, 0, n1)
            dt1 = time.perf_counter() - t2
            gomp.omp_set_num_threads(omp_threads())
            one_core = {"value": round(16.0 * n1 * len(dns) / dt1 / 1e9, 4), "unit": "GB/s", "cores": 1,
                        "sample": f"up-rows [0, {n1}), {n1 * len(dns)} states", "seconds": round(dt1, 3)}
        except OSError:
            one_core = None
        extra = {"one_core": one_core,
                 "time_to_e0_s": {"value": round(300 * (t_hv_full + t_vec), 1), "kind": "extrapolated",
                                  "how": "300 x (one full oracle H*v on all cores + one step's numpy vector "
                                         "work on full-size vectors), both timed here"}}
    elif workload in ("heisenberg16", "ctpq_xxz28"):
        n = 16 if workload == "heisenberg16" else 20
        m = W.heisenberg_chain(16) if n == 16 else W.xxz_chain_j2(20)
        s = O.basis_list(n, n // 2)
        v = np.random.default_rng(0).random(len(s)) - 0.5
        reps = 50 if n == 16 else 3
        t0 = time.perf_counter()
        for _ in range(reps):
            O.spin_hv(m, s, v)
        dt = time.perf_counter() - t0
        states, bytes_per = reps * len(s), 16.0
        sample = f"oracle spin H*v x{reps} on N={n} (dim {len(s)}), FP64 real"
    elif workload == "ext_hubbard4x4":
        m = W.extended_hubbard_square(4, 4, 1.0, 4.0, 1.0, 0.3)
        ups, dns = O.hubbard_basis(16, 8, 8)
        nu = min(sample_rows if sample_rows > 0 else 800, len(ups))
        v = np.random.default_rng(0).random(len(ups) * len(dns)) - 0.5
        t0 = time.perf_counter()
        O.hubbard_hv_rows(m, ups, dns, v, 0, nu)
        dt = time.perf_counter() - t0
        states, bytes_per = nu * len(dns), 16.0
        sample = f"oracle extended-Hubbard H*v over up-rows [0, {nu}) of {len(ups)}"
    elif workload == "tevol_pulse_hubbard16":
        # complex transfers: the oracle's complex row formula (Python),
        # row by row on a bounded sample of rows
        m = W.with_flux(W.hubbard_chain(16, 1.0, 4.0), 0.7)
        ups, dns = O.hubbard_basis(16, 8, 8)
        rows = sample_rows if sample_rows > 0 else 100000
        rng = np.random.default_rng(0)
        dim = len(ups) * len(dns)
        v = (rng.random(dim) - 0.5) + 1j * (rng.random(dim) - 0.5)
        t0 = time.perf_counter()
        for r in range(rows):
            cols, vals = O.hubbard_row(m, ups, dns, r // len(dns), r % len(dns))
            complex(np.dot(vals, v[cols]))
        dt = time.perf_counter() - t0
        del v
        states, bytes_per = rows, 32.0
        sample = f"oracle complex-transfer Hubbard rows [0, {rows}) of the 16-site ring (row formula, one thread)"
    elif workload in ("tevol_hubbard16", "tevol_ramp_hubbard16"):
        # the complex product a Taylor order applies, on the 16-site ring
        # at U = 8 (the ramp's frames differ only in U, a diagonal term)
        m = W.hubbard_chain(16, 1.0, 8.0)
        ups, dns = O.hubbard_basis(16, 8, 8)
        nu = min(sample_rows if sample_rows > 0 else len(ups), len(ups))
        rng = np.random.default_rng(0)
        dim = len(ups) * len(dns)
        vr, vi = rng.random(dim) - 0.5, rng.random(dim) - 0.5
        t0 = time.perf_counter()
        O.hubbard_hv_rows(m, ups, dns, vr, 0, nu)
        O.hubbard_hv_rows(m, ups, dns, vi, 0, nu)
        dt = time.perf_counter() - t0
        states, bytes_per = nu * len(dns), 32.0
        sample = (f"oracle complex Hubbard H*v (real and imaginary parts) over up-rows [0, {nu}) "
                  f"of {len(ups)} on the 16-site ring")
    elif workload == "tfim_ring28":
        m = W.tfim_chain(28, 1.0, 1.0)
        count = sample_rows if sample_rows > 0 else 1 << 26
        v = np.random.default_rng(0).random(1 << 28) - 0.5
        t0 = time.perf_counter()
        O.spin_gc_hv_rows(m, v, 0, count)
        dt = time.perf_counter() - t0
        states, bytes_per = count, 16.0
        sample = f"oracle SpinGC H*v over rows [0, {count}) of 2^28"
    elif workload == "spin1_chain18":
        # the full 18-site sector takes the oracle minutes to list; the
        # 14-site ring (same row formula) stands in
        m = W.spin_s_model(14, 2, W.chain_pairs(14), 1.0, 1.0)
        s = O.spin_s_basis(14, 2, 0)
        v = np.random.default_rng(0).random(len(s)) - 0.5
        t0 = time.perf_counter()
        O.spin_s_hv(m, s, v)
        dt = time.perf_counter() - t0
        states, bytes_per = len(s), 16.0
        sample = f"oracle spin-1 H*v on the 14-site ring (dim {len(s)}) standing in for 18 sites"
    else:
        m = W.j1j2_square(6, 6, 1.0, 0.5)
        rows = 20000
        t0 = time.perf_counter()
        for r in np.random.default_rng(1).integers(0, 9075135300, rows):
            O.spin_row(m, 18, int(r))
        dt = time.perf_counter() - t0
        states, bytes_per = rows, 8.0
        sample = f"oracle sparse rows of the 6x6 J1-J2 sector, {rows} random rows (row formula only)"
    gbs = bytes_per * states / dt / 1e9
    cores = 1 if workload == "tevol_pulse_hubbard16" else omp_threads()
    out = {"value": round(gbs, 4), "unit": "GB/s", "cores": cores, "kind": "oracle",
           "sample": sample, "seconds": round(dt, 3)}
    if workload == "hubbard4x4":
        out.update(extra)
    return out


def roofline(gbs: float, alg_bytes: float, kernel: str, traffic=None):
    return {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None if traffic is None else round(traffic),
            "kernel": kernel, "alg_bytes_per_launch": alg_bytes}


def base_line(a, value, ms_per_step, dtype, config):
    return {"metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def run_lanczos(a, api, ham, dim, iters, storage, wl, kernel, tune_dtype, hv_events=True, check_every=0):
    """Timed solves; with hv_events the HIP events around every product are
    recorded inside them, otherwise (products of a few microseconds, where
    the events themselves would lengthen the solves) in two extra solves
    after the timed ones."""
    import torch
    stream = torch.cuda.current_stream()
    if a.schedule:
        ham.set_schedule(**json.loads(a.schedule))
    if not a.no_tune:
        from paper_2307_13222_amd import autotune
        tuned = autotune.tune(ham, tune_dtype, 1, force=a.retune)
        if tuned.get("swept"):
            print(json.dumps({"autotune": tuned}), file=sys.stderr, flush=True)
    sched = ham.get_schedule()
    wl["schedule"] = ({k: v for k, v in sched.items() if k.startswith("hub_")} if ham.basis.kind == "hubbard"
                      else {k: v for k, v in sched.items() if k.startswith("spin_")})
    for _ in range(a.warmup):
        api.lanczos(ham, iters, seed=1, storage=storage, stream=stream)
    torch.cuda.synchronize()
    lat, hv_s, hv_n, k2_s, energies, fused, hv_solves = [], 0.0, 0, 0.0, [], False, 0
    t0 = time.perf_counter()
    for k in range(a.steps):
        s0 = time.perf_counter()
        r = api.lanczos(ham, iters, seed=1 + k, storage=storage, stream=stream, time_kernels=hv_events,
                        check_every=check_every, tol=0.0)
        lat.append(time.perf_counter() - s0)
        hv_s += r["hv_seconds"]
        hv_n += r["hv_calls"]
        k2_s += r["hv_second_kernel_seconds"]
        hv_solves += 1 if hv_events else 0
        fused = r["fused_update"]
        energies.append(float(r["energies"][0]))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    if not hv_events:
        for k in range(2):
            r = api.lanczos(ham, iters, seed=1 + k, storage=storage, stream=stream, time_kernels=True)
            hv_s += r["hv_seconds"]
            hv_n += r["hv_calls"]
            k2_s += r["hv_second_kernel_seconds"]
            hv_solves += 1
    hv_avg = hv_s / max(1, hv_n)
    esize = 8.0 if storage == "f64" else 4.0
    # algorithmic bytes per timed product: H*v reads v and writes w; with the
    # fused update, every product but a solve's first also reads q_{k-1}
    # and writes q_k back (the read of w_k is shared with the product's)
    frac_fused = (1.0 - hv_solves / max(1, hv_n)) if fused else 0.0
    alg_bytes = esize * dim * (2.0 + 2.0 * frac_fused)
    gbs = alg_bytes / hv_avg / 1e9
    hub = ham.basis.kind == "hubbard"
    if hub and k2_s > 0.0:
        # dominant kernel: the T_up column kernel. Algorithmic bytes: what
        # its part of the method must move -- read V (the T_up gathers,
        # once), read u = q_{k-1} (the epilogue; none in a solve's first
        # product), write W. The partial W the rows kernel hands it (written
        # there, read here: 16 B per state) is an intermediate of the
        # two-kernel split, reported beside the measured traffic, not counted
        k2_avg = k2_s / max(1, hv_n)
        cols_bytes = esize * dim * (3.0 - hv_solves / max(1, hv_n))
        kname = ("k_hub_up_tile (T_up block tiles in LDS, Lanczos epilogue and FP64 dots" if
                 wl["schedule"].get("hub_sweep") == 7 else
                 "k_hub_cols_f (T_up slab kernel with the Lanczos epilogue and FP64 dots")
        roof = roofline(cols_bytes / k2_avg / 1e9, cols_bytes, f"{kname}; {100 * k2_avg / hv_avg:.0f} % of a step)",
                        hub_traffic(wl["schedule"], "cols"))
        roof["ms"] = round(1e3 * k2_avg, 5)
        roof["split_overhead_bytes_per_launch"] = 2.0 * esize * dim
        pair = roofline(gbs, alg_bytes, kernel, hub_traffic(wl["schedule"], "pair"))
    else:
        roof = roofline(gbs, alg_bytes, kernel, None)
        pair = None
    out = base_line(a, gbs, 1e3 * total / a.steps, storage, wl)
    out.update({"hbm_peak_frac": round(gbs / HBM_PEAK_GBS, 4),
                "lanczos_solves_per_s": round(a.steps / total, 4),
                "solve_ms_p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                "solve_ms_p99": round(1e3 * float(np.percentile(lat, 99)), 3),
                "hv_ms_avg": round(1e3 * hv_avg, 5), "e0": energies[0],
                "fused_lanczos_update": fused,
                "hv_only_gbs": round(2 * esize * dim / hv_avg / 1e9, 2),
                "roofline": roof})
    if pair is not None:
        out["launch_pair"] = pair
    return out, energies


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {a.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2307_13222_amd import api, workloads as W

    if a.workload == "copy_probe":
        copy_probe(a)
        return
    if a.workload in ("tevol_hubbard16", "tevol_ramp_hubbard16", "tevol_pulse_hubbard16"):
        mode = {"tevol_hubbard16": "quench", "tevol_ramp_hubbard16": "ramp",
                "tevol_pulse_hubbard16": "pulse"}[a.workload]
        out = run_tevol(a, api, W, mode)
        if not a.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(a.workload, a.cpu_sample_rows)
        print(json.dumps(out), flush=True)
        return
    if a.workload == "lobpcg_hubbard3x4":
        out = run_lobpcg(a, api, W)
        print(json.dumps(out), flush=True)
        return
    if a.workload == "serving_mix":
        out = run_serving(a, W)
        if not a.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_serving(a.requests)
        print(json.dumps(out), flush=True)
        return
    ctx = api.Context(0)
    if a.workload == "hubbard4x4":
        iters = a.iters or 300
        m = W.hubbard_square(4, 4, 1.0, 4.0)
        basis = api.Basis.hubbard(ctx, 16, 8, 8)
        ham = api.Hamiltonian.hubbard(basis, m)
        wl = {"workload": "hubbard_4x4_pbc_t1_U4_half_filling", "dim": basis.dim, "lanczos_iters": iters,
              "storage": "f64", "lattice": "square 4x4", "n_up": 8, "n_dn": 8}
        out, e64 = run_lanczos(a, api, ham, basis.dim, iters, "f64", wl,
                               "H*v launch pair = k_hub_rows_fz (previous step's Lanczos update fused into the T_dn/U "
                               "rows kernel) + the T_up kernel (epilogue and FP64 dots)", "f64")
        # the same solves with FP32 vector storage (FP64 alpha/beta, dots
        # and tridiagonal), outside the timed FP64 region
        ts, hv32, e32 = [], [], []
        for k in range(max(1, min(a.steps, 3))):
            r = api.lanczos(ham, iters, seed=1 + k, storage="f32", time_kernels=True)
            ts.append(r["seconds"])
            hv32.append(r["hv_seconds"] / max(1, r["hv_calls"]))
            e32.append(float(r["energies"][0]))
        # refined: the FP32 run's Ritz vector rebuilt in FP64 (second pass),
        # its FP64 Rayleigh quotient and residual, then 16 FP64 Lanczos
        # steps from it (the reported energy)
        rr = api.lanczos(ham, iters, seed=1, storage="f32", refine=True)
        rr64 = api.lanczos(ham, iters, seed=1, storage="f64", refine=True)
        out["fp32_storage"] = {"solve_ms_p50": round(1e3 * float(np.median(ts)), 3),
                               "lanczos_solves_per_s": round(1.0 / float(np.median(ts)), 4),
                               "hv_ms_avg": round(1e3 * float(np.mean(hv32)), 5),
                               "e0_ritz": e32[0], "abs_dE0_ritz_vs_fp64_same_seed": abs(e32[0] - e64[0]),
                               "refined": {"e0": float(rr["energies"][0]),
                                           "abs_dE0_vs_fp64_same_seed": abs(float(rr["energies"][0]) - e64[0]),
                                           "rayleigh_quotient": rr["rq_e0"], "residual": rr["residual"],
                                           "err_est": rr["err_est"], "fp64_restart_steps": 16,
                                           "fp64_restart_resid_est": rr["polish_resid"],
                                           "solve_ms": round(1e3 * rr["seconds"], 3),
                                           "fp64_refined_e0": float(rr64["energies"][0]),
                                           "fp64_refined_residual": rr64["residual"]}}
    elif a.workload == "heisenberg16":
        iters = a.iters or 200
        m = W.heisenberg_chain(16)
        basis = api.Basis.spin(ctx, 16, 0)
        ham = api.Hamiltonian.spin(basis, m)
        wl = {"workload": "heisenberg_chain16_sz0", "dim": basis.dim, "lanczos_iters": iters, "storage": "f64"}
        out, _ = run_lanczos(a, api, ham, basis.dim, iters, "f64", wl, "H*v = k_spin_hv<double,1>", "f64",
                             hv_events=False)
        # many independent solves per call (B = 1: the request on a team of
        # workgroups; larger B: one workgroup per request)
        hams = [ham] * 256
        rates, lat_b = {}, {}
        for B in (1, 16, 64, 256):
            api.lanczos_batch(hams[:B], iters, list(range(1, B + 1)))
            torch.cuda.synchronize()
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                res = api.lanczos_batch(hams[:B], iters, list(range(1, B + 1)))
                ts.append(time.perf_counter() - t0)
            rates[str(B)] = round(B / float(np.median(ts)), 2)
            lat_b[str(B)] = round(1e3 * float(np.median(ts)), 3)
            assert abs(res[0]["energy"] - out["e0"]) < 1e-9
        out["batched_solves_per_s"] = rates
        out["batched_launch_ms"] = lat_b
    elif a.workload == "ext_hubbard4x4":
        iters = a.iters or 300
        m = W.extended_hubbard_square(4, 4, 1.0, 4.0, 1.0, 0.3)
        basis = api.Basis.hubbard(ctx, 16, 8, 8)
        ham = api.Hamiltonian.hubbard(basis, m)
        wl = {"workload": "extended_hubbard_4x4_pbc_t1_U4_V1_J0.3_half_filling", "dim": basis.dim,
              "lanczos_iters": iters, "storage": "f64", "pair_terms": m.n_pairs}
        a.no_tune = True
        out, _ = run_lanczos(a, api, ham, basis.dim, iters, "f64", wl,
                             "H*v = k_hub_rows_fz + k_hub_pairs (two-body terms) + the T_up tile kernel", "f64")
        # the two-body kernel runs between the rows kernel and the T_up
        # kernel: its time is the first-kernel time beyond the plain model's
        plain = api.Hamiltonian.hubbard(basis, W.hubbard_square(4, 4, 1.0, 4.0))
        rp = api.lanczos(plain, iters, seed=1, time_kernels=True)
        re_ = api.lanczos(ham, iters, seed=1, time_kernels=True)
        first = lambda r: (r["hv_seconds"] - r["hv_second_kernel_seconds"]) / max(1, r["hv_calls"])
        t_pairs = first(re_) - first(rp)
        # its algorithmic bytes: read v, read and write the partial w
        pair_bytes = 24.0 * basis.dim
        out["pair_kernel"] = {"ms_est": round(1e3 * t_pairs, 4), "alg_bytes_per_launch": pair_bytes,
                              "gbs_est": round(pair_bytes / t_pairs / 1e9, 2) if t_pairs > 0 else None,
                              "plain_model_hv_ms": round(1e3 * rp["hv_seconds"] / max(1, rp["hv_calls"]), 4)}
    elif a.workload == "tfim_ring28":
        iters = a.iters or 100
        n = 28
        m = W.tfim_chain(n, 1.0, 1.0)
        basis = api.Basis.spin_gc(ctx, n)
        ham = api.Hamiltonian.spin_gc(basis, m)
        wl = {"workload": "tfim_ring28_g1_full_space", "dim": basis.dim, "lanczos_iters": iters, "storage": "f64"}
        a.no_tune = True
        out, e = run_lanczos(a, api, ham, basis.dim, iters, "f64", wl,
                             "H*v = k_spin_gc bit-window passes (3 passes at 28 sites)", "f64")
        ks = np.pi * (2 * np.arange(n) + 1) / n
        out["e0_free_fermion"] = float(-np.sum(np.sqrt(2.0 - 2.0 * np.cos(ks))))
        out["e0_abs_diff_vs_free_fermion"] = abs(e[0] - out["e0_free_fermion"])
    elif a.workload == "spin1_chain18":
        iters = a.iters or 200
        m = W.spin_s_model(18, 2, W.chain_pairs(18), 1.0, 1.0)
        basis = api.Basis.spin_s(ctx, 18, 2, 0)
        ham = api.Hamiltonian.spin_s(basis, m)
        wl = {"workload": "spin1_heisenberg_ring18_sz0", "dim": basis.dim, "lanczos_iters": iters, "storage": "f64"}
        a.no_tune = True
        out, _ = run_lanczos(a, api, ham, basis.dim, iters, "f64", wl,
                             "H*v = k_spin_s_hv<double,1,true> (one row per thread, fused epilogue and dots)", "f64")
    elif a.workload == "j1j2_6x6":
        iters = a.iters or 100
        m = W.j1j2_square(6, 6, 1.0, 0.5)
        basis = api.Basis.spin(ctx, 36, 0)
        ham = api.Hamiltonian.spin(basis, m)
        wl = {"workload": "j1j2_square_6x6_J2_0.5_sz0", "dim": basis.dim, "lanczos_iters": iters,
              "storage": "f32 vectors, f64 alpha/beta"}
        a.no_tune = True
        if not a.schedule:
            # block-staged product: a block of states in LDS per workgroup
            ham.set_schedule(spin_split=2)
        # a product takes about a second here: every tenth step reports on stderr
        os.environ["HPHI_PROGRESS"] = "1"
        kname = ("H*v = k_spin_blk<float> (implicit basis, blocks of one high pattern staged in LDS, "
                 "partner positions from tables) + k_dots_xy_yy<float>" if ham.get_schedule()["spin_split"] in (2, 3)
                 else "H*v = k_spin_hv_implicit<float> (implicit basis, 64-bit indices)")
        out, e32 = run_lanczos(a, api, ham, basis.dim, iters, "f32", wl, kname, "f32", check_every=10)
        torch.cuda.empty_cache()
        # untimed: the same FP32 solve with its Ritz vector rebuilt in FP64
        # (second pass) and its FP64 Rayleigh quotient (no FP64 restart:
        # three FP32 and two FP64 vectors, 254 GB, fit; five FP64 do not)
        rr = None
        if not a.no_refine:
            print("j1j2: FP32 solve with FP64 Rayleigh quotient", file=sys.stderr, flush=True)
            rr = api.lanczos(ham, iters, seed=1, storage="f32", check_every=10, tol=0.0, refine=True,
                             refine_steps=-1)
        r64 = api.lanczos(ham, iters, seed=1, storage="f64", check_every=10, tol=0.0)
        out["e0_fp64_storage"] = float(r64["energies"][0])
        out["e0_abs_diff_fp32_vs_fp64"] = abs(e32[0] - float(r64["energies"][0]))
        if rr is not None:
            out["fp32_refined"] = {"rq_e0": float(rr["rq_e0"]), "ritz_e0": float(rr["ritz_e0"]),
                                   "residual": float(rr["residual"]), "err_est": float(rr["err_est"]),
                                   "abs_dE0_vs_fp64_storage": abs(float(rr["rq_e0"]) - float(r64["energies"][0]))}
    else:
        out = run_ctpq(a, api, ctx, W)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.workload, a.cpu_sample_rows)
    print(json.dumps(out), flush=True)


def run_tevol(a, api, W, mode="quench"):
    """Real-time evolution after an interaction quench (the example of the
    paper's real-time section, on 16 sites). ramp: U(t) rises linearly from
    0 to 8 over the warmup and timed steps (a time-dependent H, one frame
    per step). pulse: the U = 4 ground state driven by a light pulse through
    Peierls phases on the transfers (complex amplitudes, one frame per
    step, the pulse centred in the timed steps)."""
    import torch
    ramp = mode != "quench"
    ctx = api.Context(0)
    n, n_max, dt = 16, 10, 0.01
    basis = api.Basis.hubbard(ctx, n, 8, 8)
    u_init = 4.0 if mode == "pulse" else 0.0
    h0 = api.Hamiltonian.hubbard(basis, W.hubbard_chain(n, 1.0, u_init))
    r = api.lanczos(h0, a.iters or 150, seed=1, want_vector=True)
    psi = r["psi"].to(torch.complex128)
    del r
    h0.close()
    n_fr = a.warmup + a.steps + 1
    if mode == "pulse":
        m8 = W.hubbard_chain(n, 1.0, 4.0)
        t_c = dt * (a.warmup + a.steps / 2.0)
        fr = W.peierls_pulse(m8, 1.0, 6.0, t_c, max(dt, dt * a.steps / 4.0), dt, n_fr)
    else:
        m8 = W.hubbard_chain(n, 1.0, 8.0)
        fr = W.interaction_ramp(m8, 0.0, 8.0, n_fr - 1, n_fr) if ramp else None
    h = api.Hamiltonian.hubbard(basis, m8, frames=fr)
    print("tevol: initial state ready", file=sys.stderr, flush=True)
    api.time_evolve(h, psi, a.warmup, dt=dt, n_max=n_max)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = api.time_evolve(h, psi, a.steps, dt=dt, n_max=n_max, double_occupancy=True,
                        first_frame=a.warmup if ramp else 0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    dim = basis.dim
    alg = 2.0 * 16 * dim * n_max * a.steps          # complex FP64: read v + write w per H*v
    gbs = alg / total / 1e9
    wl = {"quench": "tevol_hubbard_ring16_half_filling_quench_U0_to_U8",
          "ramp": "tevol_hubbard_ring16_half_filling_ramp_U0_to_U8",
          "pulse": "tevol_hubbard_ring16_half_filling_U4_peierls_pulse"}[mode]
    cfg = {"workload": wl, "dim": dim, "n_max": n_max, "dt": dt, "steps": a.steps,
           "initial": f"U = {u_init:g} ground state (Lanczos)"}
    if mode == "ramp":
        cfg.update({"frames": n_fr, "ramp": f"U(t_k) = 8 k / {n_fr - 1}, one frame per step"})
    if mode == "pulse":
        cfg.update({"frames": n_fr, "pulse": "t_ij e^{i A(t)(x_i - x_j)}, A(t) = exp(-(t - t_c)^2 / 2 s^2) "
                                             "cos(6 (t - t_c)), t_c at the middle of the timed steps"})
    out = base_line(a, gbs, 1e3 * total / a.steps, "c128", cfg)
    out.update({"hbm_peak_frac": round(gbs / HBM_PEAK_GBS, 4), "time_steps_per_s": round(a.steps / total, 4),
                "hv_per_step": n_max,
                "norm_drift": float(np.max(np.abs(g["norm"] / g["norm"][0] - 1))),
                "energy": float(g["energy"][0, 0]),
                "double_occupancy": [round(float(x), 8) for x in g["double_occupancy"]],
                "roofline": roofline(gbs, 2.0 * 16 * dim,
                                     "complex H*v = Hubbard rows + cols kernels, complex epilogue "
                                     "(rate from wall time of whole steps)")})
    if mode == "ramp":
        # exact evolution under H(t_k) conserves <H(t_k)>: the energy steps
        # by the work (U_k+1 - U_k) N_s <D>(t_k+1)
        u = fr.u_site[a.warmup:a.warmup + a.steps + 1, 0]
        de = np.diff(g["energy"][:, 0])
        work = np.diff(u) * n * np.asarray(g["double_occupancy"][1:])
        out["ramp_work_residual"] = float(np.max(np.abs(de - work)))
    if ramp:
        out["energy_last"] = float(g["energy"][-1, 0])
        # the same steps with the last frame held (no frame switches)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        api.time_evolve(h, psi, a.steps, dt=dt, n_max=n_max, double_occupancy=True, first_frame=n_fr - 1)
        torch.cuda.synchronize()
        fixed = time.perf_counter() - t1
        out["ms_per_step_fixed_frame"] = round(1e3 * fixed / a.steps, 3)
        out["frame_switch_overhead"] = round(total / fixed - 1.0, 4)
    else:
        out["energy_drift"] = float(np.max(np.abs(g["energy"] - g["energy"][0])))
    return out


def run_lobpcg(a, api, W):
    """LOBPCG (block 6, lowest 4 reported) on a Hubbard sector."""
    import torch
    ctx = api.Context(0)
    basis = api.Basis.hubbard(ctx, 12, 6, 6)
    h = api.Hamiltonian.hubbard(basis, W.hubbard_square(3, 4, 1.0, 4.0))
    for _ in range(a.warmup):
        api.lobpcg(h, 6, max_iter=20, tol=1e-8)
    torch.cuda.synchronize()
    lat, r = [], None
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s0 = time.perf_counter()
        r = api.lobpcg(h, 6, max_iter=a.iters or 2000, tol=1e-7)
        lat.append(time.perf_counter() - s0)
        print(f"lobpcg: {r['iterations']} iterations, {lat[-1]:.2f} s", file=sys.stderr, flush=True)
    total = time.perf_counter() - t0
    lz = api.lanczos(h, 400, seed=2)
    dim = basis.dim
    per_hv = (total / a.steps) / max(1, r["hv_calls"])
    out = base_line(a, 16.0 * dim / per_hv / 1e9, 1e3 * total / a.steps, "f64",
                    {"workload": "lobpcg_hubbard_3x4_pbc_U4_half_filling", "dim": dim, "block": 6,
                     "reported": 4, "tol": 1e-7, "precond": "point Jacobi, shift = coupling lower bound"})
    out.update({"iterations": r["iterations"], "converged": r["converged"], "hv_calls": r["hv_calls"],
                "solve_s_p50": round(float(np.percentile(lat, 50)), 3),
                "energies": [float(x) for x in r["energies"][:4]],
                "e0_minus_lanczos": float(r["energies"][0] - lz["energies"][0]),
                "residual_max": float(np.max(r["residuals"][:4])),
                "roofline": roofline(16.0 * dim / per_hv / 1e9, 16.0 * dim,
                                     "whole LOBPCG iteration per H*v (H*v, Gram products, combinations)")})
    return out


def run_serving(a, W):
    """Continuous batching (serve.Server over serve.GpuExecutor): one step =
    one open-loop pass over the request list."""
    import torch
    from paper_2307_13222_amd import serve as S
    n_req = a.requests
    ex = S.GpuExecutor(0, n_workers=4, batch_max_dim=20000, lanczos_iters=200)
    budget = 200 * 10 ** 9
    def note(msg):
        print(msg, file=sys.stderr, flush=True)

    for _ in range(a.warmup):
        S.Server(ex, budget, max_active=64).run(W.serving_requests(16, 1e9, seed=11, n_range=(12, 20)))
    torch.cuda.synchronize()
    note("serving: warm-up done")
    # capacity: the whole list queued at t = 0
    cap_run = S.Server(ex, budget, max_active=64).run(W.serving_requests(n_req, 1e9, seed=7))
    cap = cap_run["throughput_per_s"]
    note(f"serving: capacity {cap:.3f} requests/s over {cap_run['span_s']:.1f} s")
    loads = {}
    t_total, steps = 0.0, 0
    fracs = (0.5, 0.8, 0.95)
    for k in range(max(1, a.steps)):
        frac = fracs[k % len(fracs)]
        reqs = W.serving_requests(n_req, frac * cap, seed=7 + k // len(fracs))
        t0 = time.perf_counter()
        r = S.Server(ex, budget, max_active=64).run(reqs)
        t_total += time.perf_counter() - t0
        steps += 1
        note(f"serving: load {frac} done, p50 {r['p50_latency_s']:.3f} s, p99 {r['p99_latency_s']:.3f} s")
        loads[str(frac)] = {"rate_per_s": round(frac * cap, 3), "completed": r["completed"], "failed": r["failed"],
                            "p50_latency_ms": round(1e3 * r["p50_latency_s"], 2),
                            "p99_latency_ms": round(1e3 * r["p99_latency_s"], 2),
                            "throughput_per_s": round(r["throughput_per_s"], 3),
                            "busy_fraction": round(r["busy_fraction"], 3), "peak_active": r["peak_active"],
                            "peak_gb": round(r["peak_bytes"] / 1e9, 3)}
    kinds = {}
    for res in cap_run["results"]:
        kinds.setdefault(res.kind, []).append(res)
    out = {"metric": METRIC, "value": round(cap, 3), "unit": "requests/s", "n_gpus": 1, "steps": steps,
           "warmup": a.warmup, "ms_per_step": round(1e3 * t_total / max(1, steps), 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "serving_mix_heisenberg_chains_ladders_N12-26", "requests": n_req,
                      "kinds": {k: len(v) for k, v in kinds.items()}, "lanczos_small_batch_max_dim": 20000,
                      "sqw_shifts": 64, "eta": 0.05, "sqw_tol": ex.sqw_tol, "sqw_max_iter": ex.sqw_max_iter,
                      "sqw_group_max_dim": ex.sqw_batch_max_dim, "workers": 4},
           "capacity": {"throughput_per_s": round(cap, 3), "span_s": round(cap_run["span_s"], 3),
                        "completed": cap_run["completed"], "failed": cap_run["failed"],
                        "p50_latency_ms": round(1e3 * cap_run["p50_latency_s"], 2),
                        "p99_latency_ms": round(1e3 * cap_run["p99_latency_s"], 2),
                        "busy_fraction": round(cap_run["busy_fraction"], 3)},
           "open_loop": loads,
           "roofline": None}
    return out


def cpu_baseline_serving(n_req: int):
    """The oracle on a bounded sample of the same request list: the requests
    with N <= 18 among the first ones, run one after another (ground state
    by plain Lanczos with the oracle's C H*v; S(q, w) by the Lanczos continued
    fraction from the excitation, 200 steps)."""
    import math as _m
    from oracle import core as O
    from paper_2307_13222_amd import workloads as W
    from paper_2307_13222_amd import serve as S
    reqs = [r for r in W.serving_requests(n_req, 1e9, seed=7) if r.n_sites <= 18]
    done, t0 = 0, time.perf_counter()
    for r in reqs:
        m = W.random_heisenberg(r.n_sites, r.lattice, seed=r.rid)
        st = O.basis_list(r.n_sites, O.sector_popcount_spin(r.n_sites, r.two_sz))
        hv = lambda x, m=m, st=st: O.spin_hv(m, st, x)
        v0 = np.random.default_rng(r.rid).random(len(st)) - 0.5
        lz = O.lanczos(hv, v0, 200)
        if r.kind == "sqw":
            psi = O.lanczos_ground_vector(hv, v0, lz["alpha"], lz["beta"])
            e0 = float(O.tridiag_lowest(lz["alpha"], lz["beta"])[0])
            b = O.szq_excitation(m, st, _m.pi, psi)
            al, be = O.lanczos_complex(lambda x: hv(x.real) + 1j * hv(x.imag), b, 200)
            O.continued_fraction(al, be, float(np.vdot(b, b).real),
                                 e0 + S.sqw_grid(float(np.max(m.jz)), 64) + 0.05j)
        done += 1
        if time.perf_counter() - t0 > 20.0:
            break
    dt = time.perf_counter() - t0
    return {"value": round(done / dt, 4), "unit": "requests/s", "cores": omp_threads(), "kind": "oracle",
            "sample": f"first {done} requests with N <= 18 of the same list, sequential", "seconds": round(dt, 3)}


def copy_probe(a):
    """A plain device copy of known size (2 GiB read + 2 GiB written per
    launch): run under the FETCH_SIZE / WRITE_SIZE counters, it gives the
    factor between those counters and bytes moved."""
    import torch
    n = 1 << 28
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(a.warmup):
        y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    print(json.dumps({"workload": "copy_probe", "bytes_read_per_launch": 8 * n, "bytes_written_per_launch": 8 * n,
                      "ms_per_launch": round(1e3 * dt, 4), "GB_per_s": round(16 * n / dt / 1e9, 1)}), flush=True)


def run_ctpq(a, api, ctx, W):
    """Batched cTPQ: 16 vectors advanced together by block H*V."""
    import torch
    from paper_2307_13222_amd import autotune
    k_steps = a.iters or 250
    m = W.xxz_chain_j2(28)
    basis = api.Basis.spin(ctx, 28, 0)
    ham = api.Hamiltonian.spin(basis, m)
    dim, nv = basis.dim, 16
    wl = {"workload": "ctpq_xxz_j2_chain28_sz0_16vec", "dim": dim, "n_vec": nv, "n_max": 6, "dtau": 0.02,
          "k_steps": k_steps, "storage": "c64 (FP32 complex), f64 norms"}
    if a.schedule:
        ham.set_schedule(**json.loads(a.schedule))
    else:
        # block-staged product: the block of one high pattern in LDS per
        # workgroup (the stored list's default is the one-pass kernel)
        ham.set_schedule(spin_split=2)
    if not a.no_tune:
        wl["schedule"] = autotune.tune(ham, "c64", nv, force=a.retune)["schedule"]
    else:
        wl["schedule"] = {k: v for k, v in ham.get_schedule().items() if k.startswith("spin_")}
    # block H*V time with HIP events (the kernel the propagator runs)
    v = (torch.rand((dim, nv), dtype=torch.complex64, device="cuda") - (0.5 + 0.5j)).contiguous()
    w = torch.empty_like(v)
    hv_ms = autotune.time_mult(ham, v, w, reps=10)
    del v, w
    print(f"ctpq: block H*V {hv_ms:.3f} ms", file=sys.stderr, flush=True)
    alg_bytes = 2.0 * dim * nv * 8
    gbs = alg_bytes / (hv_ms * 1e-3) / 1e9
    for _ in range(a.warmup):
        api.ctpq(ham, nv, 6, 0.02, 2, storage="c64", seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = []
    res = None
    for k in range(a.steps):
        s0 = time.perf_counter()
        res = api.ctpq(ham, nv, 6, 0.02, k_steps, storage="c64", seed=1)
        lat.append(time.perf_counter() - s0)
        print(f"ctpq: run {k} {lat[-1]:.2f} s", file=sys.stderr, flush=True)
    total = time.perf_counter() - t0
    del res["phi"]
    torch.cuda.empty_cache()
    ref = api.ctpq(ham, nv, 6, 0.02, k_steps, storage="c128", seed=1)
    del ref["phi"]
    print("ctpq: FP64 reference done", file=sys.stderr, flush=True)
    dE = float(np.max(np.abs(res["E"] - ref["E"])))
    dlogN = float(np.max(np.abs(np.cumsum(np.log(res["D"]), 0) - np.cumsum(np.log(ref["D"]), 0))))
    from paper_2307_13222_amd import thermo
    th = thermo.tpq_thermo(res["beta"], res["D"], res["E"], res["E2"], dim, 28, n_boot=200)
    out = base_line(a, gbs, 1e3 * total / a.steps, "c64", wl)
    out.update({"thermo_final_beta": {"beta": float(th["beta"][-1]),
                                      "E_per_site": [float(th["E"][-1]), float(th["E_err"][-1])],
                                      "C_per_site": [float(th["C"][-1]), float(th["C_err"][-1])],
                                      "S_per_site": [float(th["S"][-1]), float(th["S_err"][-1])]}})
    out.update({"hbm_peak_frac": round(gbs / HBM_PEAK_GBS, 4), "block_hv_ms": round(hv_ms, 4),
                "ctpq_steps_per_s": round(a.steps * k_steps / total, 3),
                "ctpq_run_ms_p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                "max_abs_dE_fp32_vs_fp64": dE, "max_abs_dlogN_fp32_vs_fp64": dlogN,
                "E_beta_final_mean": float(np.mean(res["E"][-1])),
                "roofline": roofline(gbs, alg_bytes, ("block H*V = k_spin_blk_v<float,32> (16 complex vectors; blocks of one "
                                                      "high pattern staged in LDS)") if wl["schedule"].get("spin_split") == 2
                                     else "block H*V = k_spin_hv<float,32> (16 complex vectors)")})
    return out


if __name__ == "__main__":
    main()
