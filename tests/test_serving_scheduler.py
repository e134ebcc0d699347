"""Admission logic of the serving loop, with the GPU work replaced by a sleep."""
import threading
import time

import numpy as np

from paper_2304_05460_amd import serving


class FakeServer(serving.Server):
    """Setup sleeps; a solve takes 2 + rid % 3 steps."""

    def __init__(self, slots, budget, sizes):
        super().__init__(slots=slots, hbm_budget=budget, device="cpu")
        self.sizes = sizes
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.started = []

    def _make_stream(self):
        return None

    def footprint(self, r):
        return self.sizes[r.rid]

    def _prepare(self, job):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            self.started.append(job.req.rid)
        time.sleep(0.001)

    def _begin(self, job):
        job.state = 2 + job.req.rid % 3

    def _step(self, jobs):
        time.sleep(0.0005)
        done = []
        for j in jobs:
            j.state -= 1
            if j.state == 0:
                j.res.status = 0
                done.append(j)
        return done

    def _release(self, job):
        with self.lock:
            self.running -= 1
        job.state = None


def _reqs(count, rate, seed=3):
    arr = np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=count))
    X = np.zeros((4, 1))
    return [serving.Request(i, X, np.zeros(4), 1.0, 1.0, arrival=float(arr[i]))
            for i in range(count)]


def test_fifo_slots_and_budget():
    reqs = _reqs(40, 2000.0)
    sizes = {i: 10 + (7 * i) % 30 for i in range(40)}
    srv = FakeServer(slots=3, budget=60, sizes=sizes)
    res = srv.run(reqs)
    assert all(r.status == 0 for r in res)
    assert srv.max_running <= 3 and srv.peak_active <= 3
    assert srv.peak_committed <= 60
    assert srv.started == sorted(srv.started)         # first come, first served
    for q, r in zip(reqs, res):
        assert q.arrival <= r.admitted + 1e-9 <= r.done + 1e-9
    s = serving.summarize(res)
    assert s["completed"] == 40 and s["p99_s"] >= s["p50_s"] > 0


def test_oversized_request_rejected_others_served():
    reqs = _reqs(6, 5000.0)
    sizes = {i: 5 for i in range(6)}
    sizes[2] = 100
    srv = FakeServer(slots=2, budget=20, sizes=sizes)
    res = srv.run(reqs)
    assert [r.status for r in res] == [0, 0, serving.REJECTED, 0, 0, 0]
    s = serving.summarize(res)
    assert s["rejected"] == 1 and s["completed"] == 5
