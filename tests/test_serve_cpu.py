"""Scheduler logic of the serving loop on the CPU, with a fake executor that
models device memory and run time (no GPU): FIFO admission by HBM footprint,
rejection of oversize requests, continuous admission as slots free up,
isolation of a failing request, and that every request completes."""
import threading
import time

import numpy as np
import pytest

from paper_2511_18233_amd.serve import Request, Server, latency_stats


class FakeExec:
    def __init__(self, k, log):
        self.k = k
        self.held = 0
        self.log = log

    def held_bytes(self):
        return self.held

    def release(self):
        self.log.append(("release", -1, self.k, time.perf_counter()))
        self.held = 0

    def need_bytes(self, r):
        return int(r.shell_exp[0])          # the test encodes the footprint here

    def run(self, r):
        self.held = max(self.held, self.need_bytes(r))
        self.log.append(("start", r.rid, self.k, time.perf_counter()))
        if r.nocc < 0:
            raise RuntimeError("planted failure")
        time.sleep(r.C[0, 0])
        self.log.append(("end", r.rid, self.k, time.perf_counter()))
        return np.full((1, 2, 3), float(r.rid)), None


def req(rid, arrival, need, dur, fail=False):
    z = np.zeros(2, dtype=np.int32)
    return Request(rid, arrival, z, np.zeros((2, 3)), z, z, np.array([float(need), 1.0]), np.array([[dur]]),
                   np.zeros(1), -1 if fail else 1, np.zeros((1, 1, 1)), None, [0], [])


def make(nslots, budget, log):
    return Server([FakeExec(k, log) for k in range(nslots)], budget)


def test_all_requests_complete_and_results_route_back():
    log = []
    s = make(3, 100, log)
    reqs = [req(k, 0.002 * k, 10, 0.01) for k in range(20)]
    res = s.run_trace(reqs)
    s.close()
    assert sorted(res) == list(range(20))
    for k, r in res.items():
        assert r.error is None and r.grad[0, 0, 0] == k and r.done >= r.admitted >= r.arrival - 1e-9
    st = latency_stats(res)
    assert st["n"] == 20 and st["p99_ms"] >= st["p50_ms"] > 0


def test_oversize_request_is_rejected_and_others_continue():
    log = []
    s = make(2, 50, log)
    res = s.run_trace([req(0, 0.0, 10, 0.01), req(1, 0.0, 80, 0.01), req(2, 0.0, 10, 0.01)])
    s.close()
    assert res[1].error is not None and "budget" in res[1].error
    assert res[0].error is None and res[2].error is None


def test_memory_admission_limits_concurrency():
    # each request needs 40 of a 100 budget: at most 2 run at once even with 4 slots
    log = []
    s = make(4, 100, log)
    res = s.run_trace([req(k, 0.0, 40, 0.03) for k in range(6)])
    s.close()
    events = sorted([(t, 1 if e == "start" else -1) for (e, _, _, t) in log])
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    assert peak == 2
    assert all(r.error is None for r in res.values())


def test_fifo_order_of_admission():
    log = []
    s = make(1, 100, log)
    res = s.run_trace([req(k, 0.0, 10, 0.005) for k in range(5)])
    s.close()
    starts = [rid for (e, rid, _, _) in log if e == "start"]
    assert starts == [0, 1, 2, 3, 4]
    assert [res[k].admitted for k in range(5)] == sorted(res[k].admitted for k in range(5))


def test_failing_request_is_isolated():
    log = []
    s = make(2, 100, log)
    res = s.run_trace([req(0, 0.0, 10, 0.01), req(1, 0.0, 10, 0.01, fail=True), req(2, 0.001, 10, 0.01)])
    s.close()
    assert res[1].error and "planted" in res[1].error
    assert res[0].error is None and res[2].error is None


def test_continuous_admission_while_others_run():
    # a long request keeps slot 0 busy; later arrivals start before it ends
    log = []
    s = make(2, 100, log)
    res = s.run_trace([req(0, 0.0, 10, 0.2)] + [req(k, 0.01 * k, 10, 0.01) for k in range(1, 5)])
    s.close()
    end0 = [t for (e, rid, _, t) in log if e == "end" and rid == 0][0]
    later = [t for (e, rid, _, t) in log if e == "end" and rid > 0]
    assert all(t < end0 for t in later)


def test_idle_regions_are_released_for_the_head():
    # two 40-byte requests leave both slots holding 40 of a 100 budget; a
    # 70-byte request fits only once an idle slot gives its region back
    log = []
    s = make(2, 100, log)
    res = s.run_trace([req(0, 0.0, 40, 0.01), req(1, 0.0, 40, 0.01), req(2, 0.05, 70, 0.01)], timeout=10.0)
    s.close()
    assert all(r.error is None for r in res.values())
    assert any(e == "release" for (e, _, _, _) in log)
    assert res[2].grad[0, 0, 0] == 2


def test_scheduler_reads_no_context_of_a_busy_slot():
    # held bytes come from each slot's own thread: the executor records the
    # threads that asked, and only its worker (or the constructor) may ask
    log = []

    class Strict(FakeExec):
        def __init__(self, k, log):
            super().__init__(k, log)
            self.askers = set()

        def held_bytes(self):
            self.askers.add(threading.get_ident())
            return self.held

    ex = [Strict(k, log) for k in range(2)]
    main = threading.get_ident()
    s = Server(ex, 100)
    s.run_trace([req(k, 0.0, 10, 0.01) for k in range(6)])
    s.close()
    for e, w in zip(ex, s.workers):
        assert e.askers <= {main, w.ident}
