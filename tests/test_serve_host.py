"""The serving loop's scheduling on the host, with stand-in batches whose
steps only take time (no device): every request runs exactly its steps,
the HBM budget holds, classes advance independently, and requests that do
not fit the budget wait for an idle class to close."""
import threading
import time

import numpy as np

from paper_1805_03155_amd import serve, spstd
from paper_1805_03155_amd import workloads as W


class FakeStream:
    def synchronize(self):
        pass


class FakeBatch:
    """Slots of one class; a step of the batch takes step_s seconds."""

    def __init__(self, key, capacity, step_s, log):
        self.key, self.capacity, self.step_s, self.log = key, capacity, step_s, log
        self.npoints = int(np.prod(key[0]))
        self.steps = {}
        self.lock = threading.Lock()     # only the class's worker may touch it

    def load(self, s, dx, V, psiR, psiI, probes, cfl_fraction=0.5, hbar=1.0, mass=1.0):
        assert self.lock.acquire(blocking=False)
        try:
            assert 0 <= s < self.capacity and s not in self.steps
            self.steps[s] = 0
            self.log.append(("load", self.key, s))
            return 0.05
        finally:
            self.lock.release()

    def slot_info(self, s):
        return s in self.steps, self.steps.get(s, 0), 0.05

    def step(self, k):
        assert self.lock.acquire(blocking=False)
        try:
            time.sleep(k * self.step_s)
            for s in self.steps:
                self.steps[s] += k
            self.log.append(("step", self.key, k, len(self.steps)))
        finally:
            self.lock.release()

    def read(self, s, state=False):
        n = self.steps[s]
        t = np.arange(n + 1) * 0.05
        ser = np.zeros((n + 1, 1, 2))
        ser[:, 0, 0], ser[:, 0, 1] = np.cos(3.0 * t), -np.sin(3.0 * t)
        return ser, None, None, n

    def release(self, s):
        del self.steps[s]


def _requests(spec):
    """spec: (arrival, n, steps) triples; tiny wells of the given shape."""
    out = []
    for i, (arr, n, steps) in enumerate(spec):
        N = int(np.prod(n))
        w = W.Workload(f"r{i}", tuple(n), (0.1,) * len(n), (0.0,) * len(n), np.zeros(N), np.ones(N),
                       np.zeros(N), np.array([0], np.int64), steps, W.PAPER)
        out.append(serve.Request(i, w, steps, spstd.FP64, arrival=arr))
    return out


def _server(budget, step_s, log, per_slot=100, base=1000, **kw):
    return serve.Server(hbm_budget=budget, max_steps=5000, keep_series=True,
                        batch_factory=lambda key, cap, st: FakeBatch(key, cap, step_s[key[0]], log),
                        stream_factory=FakeStream,
                        workspace_bytes=lambda key, cap: base + per_slot * cap, **kw)


def test_every_request_runs_its_steps_within_the_budget():
    log = []
    spec = [(0.002 * i, (64,) if i % 3 else (8, 8, 8), 200 + 37 * i) for i in range(24)]
    reqs = _requests(spec)
    srv = _server(budget=1000 + 100 * 4 + 1000 + 100 * 3, step_s={(64,): 2e-5, (8, 8, 8): 5e-5}, log=log,
                  max_slots=4)
    srv.run(reqs)
    assert all(r.status == "done" for r in reqs)
    assert srv.peak_used <= srv.budget and srv.used == 0
    for r in reqs:
        assert r.series.shape == (r.steps + 1, 1, 2)          # exactly its steps
        assert r.admitted >= r.arrival and r.done >= r.admitted
        assert len(r.E) >= 1 and abs(r.E[0] - 3.0) < 0.5      # the stand-in's level
    # no chunk overshoots a slot's remaining steps; slots never exceed the capacity
    assert all(e[3] <= 4 for e in log if e[0] == "step")


def test_a_slow_class_does_not_hold_back_a_fast_one():
    log = []
    slow = [(0.0, (4, 4, 4), 400)]                            # 400 x 3 ms = 1.2 s
    fast = [(0.01 * (i + 1), (32,), 300) for i in range(20)]  # 300 x 20 us = 6 ms each
    reqs = _requests(slow + fast)
    srv = _server(budget=1 << 20, step_s={(4, 4, 4): 3e-3, (32,): 2e-5}, log=log, max_slots=2)
    srv.run(reqs)
    lat_fast = [r.latency for r in reqs[1:]]
    assert reqs[0].latency >= 1.2
    assert max(lat_fast) < 0.5, lat_fast
    assert max(r.done for r in reqs[1:]) < reqs[0].done


def test_requests_wait_for_budget_and_an_idle_class_closes():
    log = []
    # room for one class with one slot: the second class opens only after
    # the first one has emptied and closed
    reqs = _requests([(0.0, (16,), 300), (0.001, (8, 8, 8), 200), (0.002, (16,), 100)])
    srv = _server(budget=1000 + 100, step_s={(16,): 1e-4, (8, 8, 8): 1e-4}, log=log, idle_close_s=0.01)
    srv.run(reqs)
    assert all(r.status == "done" for r in reqs)
    assert srv.peak_used <= srv.budget
    a, b, c = reqs
    # first come, first served across classes: b (blocked behind a) starts
    # after a is done, c (a's class, arriving later) after b's class closed
    assert b.admitted >= a.done and c.admitted >= b.done


class FailingBatch(FakeBatch):
    def step(self, k):
        raise RuntimeError("device step failed")


def test_a_worker_error_reaches_the_caller():
    log = []
    reqs = _requests([(0.0, (64,), 100), (0.0, (8, 8, 8), 100)])
    srv = serve.Server(hbm_budget=1 << 20, max_steps=5000,
                       batch_factory=lambda key, cap, st: (FailingBatch if key[0] == (8, 8, 8) else FakeBatch)(
                           key, cap, 1e-5, log),
                       stream_factory=FakeStream, workspace_bytes=lambda key, cap: 1000 + 100 * cap)
    try:
        srv.run(reqs)
    except RuntimeError as e:
        assert "device step failed" in str(e)
    else:
        raise AssertionError("the worker's error was not raised")
    assert all(not c.thread.is_alive() for c in srv.classes.values())


def test_time_limit_stops_the_workers():
    log = []
    reqs = _requests([(0.0, (4, 4, 4), 4000)])               # 4000 x 1 ms: 4 s
    srv = _server(budget=1 << 20, step_s={(4, 4, 4): 1e-3}, log=log)
    t0 = time.perf_counter()
    srv.run(reqs, time_limit=0.3)
    assert time.perf_counter() - t0 < 2.0
    assert reqs[0].status == "running" and reqs[0].done is None
