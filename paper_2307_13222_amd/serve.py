"""Continuous-batching request server for ground-state and S(q, w) solves.

Requests (Poisson arrivals, chains and 2-leg ladders of mixed size) are
admitted as soon as a slot is free, their device-memory footprint fits the
budget and the device's free memory (as the device reports it, less what
admitted requests have yet to allocate) can hold it; admitted requests run
concurrently on the device, and new arrivals join while others are in
flight (not a queue drained one request at a time):

  * small ground-state requests (sector dimension <= batch_max_dim) are
    grouped: whatever is admitted while the previous group runs goes into
    the next single call of the batched Lanczos (a team of workgroups per
    request when the group is small, one workgroup per request otherwise;
    the same numbers either way);
  * larger ground-state requests and S(q, w) requests each run on a worker
    thread with its own HIP stream (Lanczos with a convergence check every
    10 steps -- for S(q, w) on the Ritz residual estimate as well, since the
    ground vector's error carries into D(z) -- ground vector from a second
    pass, S^z(q) excitation), so their kernels overlap on the device;
  * the shifted COCG over the shift grid of a large S(q, w) request runs on
    its worker's stream; small ones (sector dimension <= sqw_batch_max_dim)
    hand their excitation to a grouping thread, which runs every excitation
    that arrived while the previous group ran as one launch (one workgroup
    per COCG sequence; a request alone takes the same launch, so its numbers
    are the same alone and grouped).

Every path uses fixed-order reductions, so a request's numbers are the same
alone and in any mix. The server records arrival, admission and completion
times and reports p50 / p99 latency next to throughput.

`FakeExecutor` is a deterministic simulated device (configurable memory and
service times, injectable failures) used to test admission and accounting
without a GPU.
"""
from __future__ import annotations

import heapq
import math
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

from .workloads import Request, random_heisenberg


@dataclass
class Result:
    rid: int
    kind: str
    lattice: str
    n_sites: int
    dim: int
    arrival: float
    admit: float = math.nan
    finish: float = math.nan
    ok: bool = True
    error: str = ""
    energy: float = math.nan
    iterations: int = 0
    omega: Optional[np.ndarray] = None
    D: Optional[np.ndarray] = None
    path: str = ""

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def sector_dim(n_sites: int, two_sz: int) -> int:
    return math.comb(n_sites, (n_sites + two_sz) // 2)


def footprint_bytes(req: Request) -> int:
    """Device memory a request holds while active: basis states (4 B per
    state), Lanczos vectors (3 x 8 B) and, for S(q, w), the ground vector and
    four complex FP64 work vectors."""
    d = sector_dim(req.n_sites, req.two_sz)
    per = 4 + 3 * 8
    if req.kind == "sqw":
        per += 8 + 16 + 4 * 16
    return d * per + (1 << 20)


# ------------------------------------------------------------------ server --

class Server:
    def __init__(self, executor, hbm_budget: int, max_active: int = 64):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)

    def run(self, requests: List[Request]) -> Dict:
        ex = self.ex
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        waiting: List[Request] = []
        active: Dict[int, Tuple[Request, int]] = {}
        results: Dict[int, Result] = {}
        used = 0
        peak_used = 0
        peak_active = 0
        busy = 0.0
        last_t = ex.now()
        ex.begin()
        i = 0
        while i < len(pending) or waiting or active:
            now = ex.now()
            if active:
                busy += now - last_t
            last_t = now
            while i < len(pending) and pending[i].arrival <= now:
                r = pending[i]
                waiting.append(r)
                results[r.rid] = Result(r.rid, r.kind, r.lattice, r.n_sites, sector_dim(r.n_sites, r.two_sz),
                                        r.arrival)
                i += 1
            # admission: every waiting request that fits, in arrival order
            still = []
            for r in waiting:
                fp = footprint_bytes(r)
                res = results[r.rid]
                if fp > self.budget:
                    res.ok, res.error, res.finish, res.admit = False, "footprint above the memory budget", now, now
                    continue
                if len(active) < self.max_active and used + fp <= self.budget and ex.can_start(r):
                    try:
                        ex.start(r)
                    except MemoryError as e:       # allocation failure: stay queued
                        res.error = f"deferred: {e}"
                        still.append(r)
                        continue
                    res.admit = now
                    active[r.rid] = (r, fp)
                    used += fp
                    peak_used = max(peak_used, used)
                    peak_active = max(peak_active, len(active))
                else:
                    still.append(r)
            waiting = still
            if not active and not waiting and i >= len(pending):
                break
            next_arr = pending[i].arrival if i < len(pending) else math.inf
            timeout = max(0.0, next_arr - ex.now()) if active or waiting else max(0.0, next_arr - now)
            for rid, out in ex.poll(timeout if math.isfinite(timeout) else None):
                r, fp = active.pop(rid)
                used -= fp
                res = results[rid]
                res.finish = ex.now()
                for k, v in out.items():
                    setattr(res, k, v)
        ex.end()
        done = [results[k] for k in sorted(results)]
        ok = [r for r in done if r.ok]
        lat = np.array([r.latency for r in ok]) if ok else np.array([math.nan])
        t_end = max((r.finish for r in done), default=0.0)
        t_start = min((r.arrival for r in done), default=0.0)
        span = max(t_end - t_start, 1e-12)
        return {"results": done,
                "completed": len(ok), "failed": len(done) - len(ok),
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_latency_s": float(np.mean(lat)),
                "throughput_per_s": len(ok) / span, "span_s": span,
                "busy_fraction": busy / span, "peak_bytes": peak_used, "peak_active": peak_active}


# ------------------------------------------------------- simulated device --

class FakeExecutor:
    """Simulated device clock: service time from `service(req)`, with a
    concurrency slowdown `1 + slow * (active - 1)` frozen at start;
    `fail(req)` may return 'alloc' (start raises MemoryError once),
    'breakdown' (the solve reports a breakdown) or None. With `device_bytes`
    the device has that much memory, of which `external(t)` is held by
    others at time t; a request starts only when its footprint fits what
    the running requests and the others leave free (as GpuExecutor asks the
    device)."""

    def __init__(self, service: Callable[[Request], float], slow: float = 0.0,
                 fail: Optional[Callable[[Request], Optional[str]]] = None,
                 device_bytes: Optional[int] = None, external: Optional[Callable[[float], int]] = None):
        self.service, self.slow, self.fail = service, slow, fail
        self.device_bytes, self.external = device_bytes, external
        self.t = 0.0
        self.heap: List[Tuple[float, int]] = []
        self.out: Dict[int, Dict] = {}
        self.held: Dict[int, int] = {}
        self.failed_once = set()
        self.admit_free: List[Tuple[int, int]] = []   # (free bytes seen, footprint) at each start

    def begin(self):
        pass

    def end(self):
        pass

    def now(self) -> float:
        return self.t

    def free_bytes(self) -> Optional[int]:
        if self.device_bytes is None:
            return None
        ext = self.external(self.t) if self.external else 0
        return self.device_bytes - ext - sum(self.held.values())

    def can_start(self, req) -> bool:
        free = self.free_bytes()
        return free is None or footprint_bytes(req) <= free

    def start(self, req):
        mode = self.fail(req) if self.fail else None
        if mode == "alloc" and req.rid not in self.failed_once:
            self.failed_once.add(req.rid)
            raise MemoryError("injected allocation failure")
        free = self.free_bytes()
        if free is not None:
            self.admit_free.append((free, footprint_bytes(req)))
        self.held[req.rid] = footprint_bytes(req)
        dt = self.service(req) * (1.0 + self.slow * len(self.heap))
        heapq.heappush(self.heap, (self.t + dt, req.rid))
        self.out[req.rid] = {"energy": -float(req.n_sites), "iterations": 1, "path": "fake",
                             "ok": mode != "breakdown",
                             "error": "breakdown" if mode == "breakdown" else ""}

    def poll(self, timeout: Optional[float]):
        if not self.heap:
            if timeout is not None:
                self.t += timeout
            return []
        t_next = self.heap[0][0]
        if timeout is not None and self.t + timeout < t_next:
            self.t += timeout
            return []
        self.t = t_next
        done = []
        while self.heap and self.heap[0][0] <= self.t:
            _, rid = heapq.heappop(self.heap)
            self.held.pop(rid, None)
            done.append((rid, self.out.pop(rid)))
        return done


# ------------------------------------------------------------ GPU device --

def sqw_grid(j_max: float, n: int = 64) -> np.ndarray:
    """Frequencies w_j uniform in [0, 4 J_max] (64 shifts)."""
    return np.linspace(0.0, 4.0 * j_max, n)


class GpuExecutor:
    """Runs requests on the GPU through the C ABI (see module docstring)."""

    def __init__(self, device: int = 0, n_workers: int = 4, batch_max_dim: int = 20000,
                 max_batch: int = 512, lanczos_iters: int = 200, max_iter: int = 500, eta: float = 0.05,
                 n_shift: int = 64, sqw_tol: float = 1e-8, sqw_max_iter: int = 6000,
                 gs_resid_tol: float = 1e-9, reserve_bytes: int = 512 << 20, sqw_batch_max_dim: int = 20000):
        from . import api
        self.api = api
        self.ctx = api.Context(device)
        self.n_workers = n_workers
        self.batch_max_dim = batch_max_dim
        self.max_batch = max_batch
        self.lanczos_iters = lanczos_iters
        self.max_iter = max_iter
        self.eta = eta
        self.n_shift = n_shift
        self.sqw_tol = sqw_tol
        self.sqw_max_iter = sqw_max_iter
        self.gs_resid_tol = gs_resid_tol
        self.sqw_batch_max_dim = sqw_batch_max_dim
        self.device = device
        self.pending_bytes = 0
        self.reserve_bytes = reserve_bytes
        self.t0 = time.perf_counter()
        self.work: "queue.Queue" = queue.Queue()
        self.batchq: "queue.Queue" = queue.Queue()
        self.cocgq: "queue.Queue" = queue.Queue()
        self.done: "queue.Queue" = queue.Queue()
        self.bases: Dict[Tuple[int, int], object] = {}
        self.lock = threading.Lock()
        self.threads: List[threading.Thread] = []

    # -- model construction (bases shared per sector) --
    def _basis(self, n, two_sz):
        with self.lock:
            key = (n, two_sz)
            if key not in self.bases:
                self.bases[key] = self.api.Basis.spin(self.ctx, n, two_sz)
            return self.bases[key]

    def _ham(self, req):
        m = random_heisenberg(req.n_sites, req.lattice, seed=req.rid)
        return self.api.Hamiltonian.spin(self._basis(req.n_sites, req.two_sz), m), m

    # -- lifecycle --
    def begin(self):
        import torch
        self.t0 = time.perf_counter()
        self.stop = False
        for k in range(self.n_workers):
            t = threading.Thread(target=self._worker, args=(torch.cuda.Stream(),), daemon=True)
            t.start()
            self.threads.append(t)
        t = threading.Thread(target=self._batcher, args=(torch.cuda.Stream(),), daemon=True)
        t.start()
        self.threads.append(t)
        self.cocg_thread = threading.Thread(target=self._cocg_grouper, args=(torch.cuda.Stream(),), daemon=True)
        self.cocg_thread.start()

    def end(self):
        for _ in range(self.n_workers):
            self.work.put(None)
        self.batchq.put(None)
        for t in self.threads:
            t.join()
        # the workers have handed over their last excitations
        self.cocgq.put(None)
        self.cocg_thread.join()
        self.threads = []

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def can_start(self, req) -> bool:
        """Admit only what the device can still hold: its free memory now
        (other processes and the allocator's cache included), less the
        footprints of requests admitted but not yet running (their buffers
        are not allocated yet), less a reserve."""
        import torch
        free, _ = torch.cuda.mem_get_info(self.device)
        with self.lock:
            pending = self.pending_bytes
        return footprint_bytes(req) + pending + self.reserve_bytes <= free

    def _begin_request(self, req):
        with self.lock:
            self.pending_bytes -= footprint_bytes(req)

    def start(self, req):
        with self.lock:
            self.pending_bytes += footprint_bytes(req)
        if req.kind == "lanczos" and sector_dim(req.n_sites, req.two_sz) <= self.batch_max_dim:
            self.batchq.put(req)
        else:
            self.work.put(req)

    def poll(self, timeout: Optional[float]):
        out = []
        try:
            out.append(self.done.get(timeout=timeout if timeout is None or timeout > 0 else 1e-4))
            while True:
                out.append(self.done.get_nowait())
        except queue.Empty:
            pass
        return out

    # -- execution --
    def _prepare_sqw(self, req, stream=None) -> Dict:
        """Ground state, excitation and shift grid of an S(q, w) request."""
        api = self.api
        ham, m = self._ham(req)
        # the excitation is built from the ground vector, so its error (about
        # the Ritz residual over the gap) sets D(z)'s: stop on the residual
        # estimate too, not on the energy alone
        r = api.lanczos(ham, self.max_iter, seed=req.rid + 1, check_every=10, tol=1e-12,
                        resid_tol=self.gs_resid_tol, want_vector=True, stream=stream)
        e0 = float(r["energies"][0])
        b = api.szq(ham, math.pi, r["psi"], stream=stream)
        omega = sqw_grid(float(np.max(m.jz)), self.n_shift)
        return {"ham": ham, "b": b, "z": e0 + omega + 1j * self.eta, "energy": e0, "iterations": r["iterations"],
                "omega": omega}

    @staticmethod
    def _sqw_result(prep, d, path) -> Dict:
        return {"energy": prep["energy"], "iterations": prep["iterations"], "omega": prep["omega"], "D": d["D"],
                "path": path, "ok": bool(d["converged"]), "error": "" if d["converged"] else "COCG not converged"}

    def run_sqw_group(self, preps, stream=None) -> List[Dict]:
        """The COCG stage of small S(q, w) requests in one launch."""
        out = self.api.sqw_batch([p["ham"] for p in preps], [p["b"] for p in preps], [p["z"] for p in preps],
                                 max_iter=self.sqw_max_iter, tol=self.sqw_tol, stream=stream)
        return [self._sqw_result(p, d, f"cocg_group{len(preps)}") for p, d in zip(preps, out)]

    def run_one(self, req, stream=None) -> Dict:
        """One request on one stream (also used to run a request alone)."""
        api = self.api
        if req.kind == "lanczos":
            ham, _ = self._ham(req)
            r = api.lanczos(ham, self.max_iter, seed=req.rid + 1, check_every=10, tol=1e-12, stream=stream)
            return {"energy": float(r["energies"][0]), "iterations": r["iterations"], "path": "stream"}
        prep = self._prepare_sqw(req, stream)
        if sector_dim(req.n_sites, req.two_sz) <= self.sqw_batch_max_dim:
            return self.run_sqw_group([prep], stream)[0]
        d = api.sqw(prep["ham"], prep["b"], prep["z"], max_iter=self.sqw_max_iter, tol=self.sqw_tol, stream=stream)
        return self._sqw_result(prep, d, "stream")

    def run_batch(self, reqs, stream=None) -> List[Dict]:
        hams = [self._ham(r)[0] for r in reqs]
        out = self.api.lanczos_batch(hams, self.lanczos_iters, [r.rid + 1 for r in reqs], stream=stream)
        return [{"energy": o["energy"], "iterations": o["iterations"], "path": f"batch{len(reqs)}"}
                for o in out]

    def _worker(self, stream):
        while True:
            req = self.work.get()
            if req is None:
                return
            self._begin_request(req)
            try:
                if req.kind == "sqw" and sector_dim(req.n_sites, req.two_sz) <= self.sqw_batch_max_dim:
                    prep = self._prepare_sqw(req, stream)
                    # the excitation must be complete before another stream reads it
                    stream.synchronize()
                    self.cocgq.put((req, prep))
                    continue
                res = self.run_one(req, stream)
            except Exception as e:  # report, keep serving
                res = {"ok": False, "error": repr(e)}
            self.done.put((req.rid, res))

    def _cocg_grouper(self, stream):
        """Runs the excitations handed over while the previous group ran as
        one batched COCG launch."""
        while True:
            item = self.cocgq.get()
            if item is None:
                return
            group = [item]
            stop = False
            while len(group) < self.max_batch:
                try:
                    it = self.cocgq.get_nowait()
                except queue.Empty:
                    break
                if it is None:
                    stop = True
                    break
                group.append(it)
            try:
                outs = self.run_sqw_group([p for _, p in group], stream)
            except Exception as e:
                outs = [{"ok": False, "error": repr(e)}] * len(group)
            for (r, _), o in zip(group, outs):
                self.done.put((r.rid, o))
            if stop:
                return

    def _batcher(self, stream):
        while True:
            req = self.batchq.get()
            if req is None:
                return
            group = [req]
            stop = False
            while len(group) < self.max_batch:
                try:
                    r = self.batchq.get_nowait()
                except queue.Empty:
                    break
                if r is None:
                    stop = True
                    break
                group.append(r)
            for r in group:
                self._begin_request(r)
            try:
                outs = self.run_batch(group, stream)
            except Exception as e:
                outs = [{"ok": False, "error": repr(e)}] * len(group)
            for r, o in zip(group, outs):
                self.done.put((r.rid, o))
            if stop:
                return
