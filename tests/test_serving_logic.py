"""CPU tests of the serving scheduler with a fake executor and a fake HBM budget."""

import threading
import time

import pytest

from paper_1305_6497_amd.serving import Request, Server, summarize


class FakeExecutor:
    """Footprint = shpar[0] bytes; runtime = x * 10 ms; records concurrency."""

    def __init__(self):
        self.lock = threading.Lock()
        self.running = 0
        self.used = 0
        self.max_running = 0
        self.max_used = 0
        self.order = []

    def prepare(self, req):
        return dict(sites=[0] * 8), int(req.shpar[0])

    def __call__(self, req, prep):
        with self.lock:
            self.order.append(req.id)
            self.running += 1
            self.used += int(req.shpar[0])
            self.max_running = max(self.max_running, self.running)
            self.max_used = max(self.max_used, self.used)
        time.sleep(req.x * 0.01)
        with self.lock:
            self.running -= 1
            self.used -= int(req.shpar[0])
        return [dict(qext=1.0, qabs=0.5, qsca=0.5)] * 2, [dict(status=0, iters=1)] * 2


def _req(i, t, fp, dur):
    return Request(id=i, arrival=t, shape="ELLIPSOID", shpar=(fp, fp, fp), m=1.5, x=dur)


def test_slots_and_budget_respected_and_fifo():
    ex = FakeExecutor()
    reqs = [_req(i, 0.0, 40 + 10 * (i % 3), 2) for i in range(12)]
    res = Server(ex, slots=3, hbm_budget=120).run(reqs)
    assert len(res) == 12
    assert ex.max_running <= 3
    assert ex.max_used <= 120
    assert ex.order == sorted(ex.order)            # admitted in arrival order


def test_continuous_batching_admits_arrivals_while_others_run():
    ex = FakeExecutor()
    # a long request first, then short ones arriving while it runs
    reqs = [_req(0, 0.0, 10, 20)] + [_req(i, 0.02 * i, 10, 1) for i in range(1, 6)]
    res = Server(ex, slots=4, hbm_budget=100).run(reqs)
    long_done = res[0].done
    assert all(res[i].done < long_done for i in range(1, 6))
    assert all(res[i].admitted < long_done for i in range(1, 6))


def test_memory_blocks_admission_until_freed():
    ex = FakeExecutor()
    reqs = [_req(0, 0.0, 80, 5), _req(1, 0.0, 50, 1)]
    res = Server(ex, slots=4, hbm_budget=100).run(reqs)
    assert res[1].admitted >= res[0].done - 1e-3      # waited for the first to free memory
    assert ex.max_used <= 100


def test_request_larger_than_budget_is_rejected():
    with pytest.raises(ValueError):
        Server(FakeExecutor(), slots=2, hbm_budget=10).run([_req(0, 0.0, 50, 1)])


def test_summary_latency_percentiles():
    ex = FakeExecutor()
    reqs = [_req(i, 0.0, 1, 1) for i in range(8)]
    t0 = time.perf_counter()
    res = Server(ex, slots=8, hbm_budget=100).run(reqs)
    s = summarize(res, time.perf_counter() - t0)
    assert s["requests"] == 8 and s["solves"] == 16 and s["converged"] == 8
    assert 0 < s["p50_ms"] <= s["p99_ms"]
