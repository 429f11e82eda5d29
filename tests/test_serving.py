"""Continuous-batching server on a simulated device (no GPU): admission by
memory footprint, slot reuse, latency accounting, Poisson replay, and the
failure paths (allocation failure, solver breakdown, oversized request)."""
import math

import numpy as np
import pytest

from paper_2307_13222_amd import serve as S
from paper_2307_13222_amd import workloads as W


def service(req):
    # simulated seconds: proportional to the sector dimension
    return 1e-7 * S.sector_dim(req.n_sites, req.two_sz) + 2e-3


def test_poisson_replay_is_seeded():
    a = W.serving_requests(100, 50.0, seed=7)
    b = W.serving_requests(100, 50.0, seed=7)
    c = W.serving_requests(100, 50.0, seed=8)
    assert [(r.arrival, r.kind, r.lattice, r.n_sites) for r in a] == \
           [(r.arrival, r.kind, r.lattice, r.n_sites) for r in b]
    assert [r.arrival for r in a] != [r.arrival for r in c]
    assert all(12 <= r.n_sites <= 26 for r in a)
    assert all(r.n_sites % 2 == 0 for r in a if r.lattice == "ladder")
    assert all(r.two_sz == r.n_sites % 2 for r in a)
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert abs(np.mean(gaps) - 1 / 50.0) < 0.3 / 50.0


def test_admission_respects_budget_and_slots():
    reqs = W.serving_requests(300, 400.0, seed=1)
    budget = 3 * 10 ** 9
    out = S.Server(S.FakeExecutor(service, slow=0.05), budget, max_active=6).run(reqs)
    assert out["completed"] == 300 and out["failed"] == 0
    assert out["peak_bytes"] <= budget
    assert out["peak_active"] <= 6
    for r in out["results"]:
        assert r.arrival <= r.admit <= r.finish
    assert out["p50_latency_s"] <= out["p99_latency_s"]


def test_requests_overlap_and_join_while_others_run():
    reqs = W.serving_requests(80, 1000.0, seed=2)
    out = S.Server(S.FakeExecutor(service), 10 ** 12, max_active=64).run(reqs)
    res = out["results"]
    # some request is admitted while another admitted earlier is still running
    overlaps = sum(1 for a in res for b in res if a.rid != b.rid and a.admit < b.admit < a.finish)
    assert overlaps > 10
    assert out["peak_active"] > 1


def test_memory_pressure_queues_instead_of_failing():
    reqs = W.serving_requests(60, 1000.0, seed=3, n_range=(24, 26))
    big = max(S.footprint_bytes(r) for r in reqs)
    out = S.Server(S.FakeExecutor(service), int(1.5 * big), max_active=64).run(reqs)
    assert out["completed"] == 60
    assert out["peak_bytes"] <= 1.5 * big
    # room for about one of the largest at a time: later arrivals wait
    waited = [r for r in out["results"] if r.admit > r.arrival]
    assert len(waited) > 10


def test_injected_allocation_failure_is_retried():
    reqs = W.serving_requests(30, 200.0, seed=4)
    bad = {reqs[3].rid, reqs[10].rid}
    ex = S.FakeExecutor(service, fail=lambda r: "alloc" if r.rid in bad else None)
    out = S.Server(ex, 10 ** 12).run(reqs)
    assert out["completed"] == 30
    assert ex.failed_once == bad


def test_breakdown_reported_not_hidden():
    reqs = W.serving_requests(20, 200.0, seed=5)
    ex = S.FakeExecutor(service, fail=lambda r: "breakdown" if r.rid == 7 else None)
    out = S.Server(ex, 10 ** 12).run(reqs)
    r7 = [r for r in out["results"] if r.rid == 7][0]
    assert not r7.ok and r7.error == "breakdown"
    assert out["completed"] == 19 and out["failed"] == 1


def test_oversized_request_rejected():
    reqs = W.serving_requests(10, 100.0, seed=6, n_range=(26, 26))
    out = S.Server(S.FakeExecutor(service), 10 ** 6).run(reqs)
    assert out["failed"] == 10
    assert all("budget" in r.error for r in out["results"])


def test_footprint_model():
    r = W.Request(0, 0.0, "sqw", "chain", 26, 0)
    fp = S.footprint_bytes(r)
    d = math.comb(26, 13)
    assert fp > 100 * d and fp < 140 * d
    assert S.footprint_bytes(W.Request(0, 0.0, "lanczos", "chain", 26, 0)) < fp


def test_admission_follows_device_free_memory():
    # the device (8 GB) is half held by another user for the first 0.05 s:
    # requests that fit the budget but not the free memory wait, none is
    # started on memory the device does not have, and all complete
    reqs = W.serving_requests(60, 2000.0, seed=9, n_range=(22, 26))
    dev_bytes = 8 * 10 ** 9
    ex = S.FakeExecutor(service, device_bytes=dev_bytes,
                        external=lambda t: 4 * 10 ** 9 if t < 0.05 else 0)
    out = S.Server(ex, 10 ** 12, max_active=64).run(reqs)
    assert out["completed"] == 60
    assert ex.admit_free and all(fp <= free for free, fp in ex.admit_free)
    early = [r for r in out["results"] if r.arrival < 0.02]
    assert any(r.admit > r.arrival for r in early)
    # with the device all free the same list waits less
    out2 = S.Server(S.FakeExecutor(service, device_bytes=dev_bytes), 10 ** 12, max_active=64).run(reqs)
    assert out2["mean_latency_s"] < out["mean_latency_s"]
