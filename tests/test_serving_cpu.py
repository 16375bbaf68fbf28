"""Host logic of the continuous-batching request loop (no GPU): admission in
arrival order, at most `slots` requests at once, the device-memory budget,
and latency accounting, with a stand-in executor."""
import threading
import time

import pytest

from paper_1010_0762_amd import serving
from paper_1010_0762_amd import workloads as wl


def _reqs(arrivals, edges):
    return [wl.Request(i, a, e, (1.0, 1.0, 1.0), 4, 10, 7 + i) for i, (a, e) in
            enumerate(zip(arrivals, edges))]


def test_slots_bound_concurrency_and_fifo():
    active, peak, order = [0], [0], []
    lock = threading.Lock()

    def execute(r):
        with lock:
            active[0] += 1
            peak[0] = max(peak[0], active[0])
            order.append(r.rid)
        time.sleep(0.05)
        with lock:
            active[0] -= 1
        return [{"status": 0}] * r.nsys, None

    reqs = _reqs([0.0] * 8, [16] * 8)
    srv = serving.Server(slots=3, hbm_budget=1 << 40, execute=execute)
    res = srv.run(reqs)
    assert peak[0] == 3
    assert order == sorted(order)            # admitted in arrival order
    assert [r.rid for r in res] == list(range(8))
    assert all(r.latency >= 0.05 for r in res)
    summ = serving.latency_summary(res)
    assert summ["p99_s"] >= summ["p50_s"] > 0 and summ["all_converged"]


def test_memory_budget_limits_admission():
    active, peak = [0], [0]
    lock = threading.Lock()

    def execute(r):
        with lock:
            active[0] += 1
            peak[0] = max(peak[0], active[0])
        time.sleep(0.03)
        with lock:
            active[0] -= 1
        return [{"status": 0}] * r.nsys, None

    reqs = _reqs([0.0] * 6, [32] * 6)
    one = serving.request_bytes(reqs[0])
    srv = serving.Server(slots=6, hbm_budget=2 * one + 1, execute=execute)
    srv.run(reqs)
    assert peak[0] == 2
    with pytest.raises(ValueError):
        serving.Server(slots=2, hbm_budget=one // 2, execute=execute).run(reqs[:1])


def test_arrivals_are_respected():
    seen = {}

    def execute(r):
        seen[r.rid] = time.perf_counter()
        return [{"status": 0}], None

    reqs = _reqs([0.0, 0.1, 0.2], [16, 16, 16])
    t0 = time.perf_counter()
    res = serving.Server(slots=2, hbm_budget=1 << 40, execute=execute).run(reqs)
    for r in reqs:
        assert seen[r.rid] - t0 >= r.arrival - 0.01
    assert all(x.admitted >= x.arrival - 1e-3 for x in res)
