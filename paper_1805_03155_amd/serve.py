"""Serving loop: eigenvalue-solve requests with continuous batching.

Requests of one grid shape and precision form a class; each class owns one
batch (``spstd.Batch``) whose slots hold the wavefunctions of its admitted
requests on the device for their whole run, one stream and one worker
thread.  A worker repeatedly

1. admits the class's routed requests into free slots, first come first
   served (loading a slot synchronises the class's own stream only);
2. advances the batch by K steps and waits for them on its stream:
   K = min(the smallest remaining step count among its active slots, the
   steps that fill the chunk's time budget at the class's measured step
   time, the chunk cap), so that every request of the class shares every
   launch and a chunk never holds an arrival back for long;
3. finishes the requests whose step count is reached: reads their probe
   series, extracts eigenvalues with ``spstd.spectrum`` and frees their
   slots.

The library calls and the stream waits release the interpreter lock, so
the classes advance independently: a copy, a long chunk or the host's
spectrum in one class never holds back another.  The dispatcher (the
caller's thread) routes arrivals to their classes, opens a class when its
workspace fits the HBM budget, and closes idle classes while requests wait
for budget.  Latency is measured from arrival to the result; throughput is
counted in grid-point stage updates.

Host code only orchestrates; every step of the solver runs in the
library's kernels.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass

import numpy as np

from . import spstd
from . import workloads as W


@dataclass
class Request:
    rid: int
    work: W.Workload          # grid, spacing, V, initial state, probes
    steps: int
    precision: int = spstd.FP64
    nlevels: int = 4
    arrival: float = 0.0       # seconds, on the server's clock
    admitted: float = None
    done: float = None
    dt: float = None
    E: np.ndarray = None
    series: np.ndarray = None
    status: str = "waiting"

    @property
    def key(self):
        return (tuple(self.work.n), self.precision)

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


class _Class:
    """One class: its routed requests, its slots and its worker's state."""

    def __init__(self, key, capacity, nbytes):
        self.key = key
        self.capacity = capacity
        self.bytes = nbytes
        self.queue = deque()        # routed to the class, not yet admitted (server lock)
        self.slots = {}             # slot -> Request (worker only)
        self.step_s = None          # measured seconds per step
        self.idle_since = None      # server clock time the class became empty
        self.closing = False
        self.finished = False       # the worker has exited and freed the batch
        self.error = None
        self.thread = None


class Server:
    """Continuous-batching eigenvalue server on one GPU.

    chunk: the most steps per launch chunk; chunk_ms: the chunk's time
    budget at the class's measured step time; max_slots: slots per class
    (fewer when the HBM budget is short); max_steps: the longest request
    (it sizes the probe buffers); max_concurrent: classes stepping at once
    (None: all).  batch_factory(key, capacity, stream) and stream_factory()
    replace the device batch and stream (host tests of the scheduling)."""

    def __init__(self, hbm_budget, coeffs=W.PAPER, chunk=4096, chunk_ms=25.0, max_slots=64,
                 max_steps=20000, nprobes=1, device="cuda", keep_series=True, max_concurrent=None,
                 idle_close_s=0.05, batch_factory=None, stream_factory=None, workspace_bytes=None):
        self.budget = int(hbm_budget)
        self.coeffs = coeffs
        self.chunk = int(chunk)
        self.chunk_s = float(chunk_ms) * 1e-3
        self.max_slots = int(max_slots)
        self.max_steps = int(max_steps)
        self.nprobes = int(nprobes)
        self.device = device
        self.keep_series = keep_series
        self.idle_close_s = float(idle_close_s)
        self._gate = threading.BoundedSemaphore(max_concurrent) if max_concurrent else None
        self._batch_factory = batch_factory or self._device_batch
        self._stream_factory = stream_factory or self._device_stream
        self._workspace_bytes = workspace_bytes or self._device_workspace_bytes
        self.subs = sum(1 for x in coeffs[0] if x) + sum(1 for x in coeffs[1] if x)
        self.classes = {}
        self.blocked = deque()      # requests whose class cannot open yet (budget)
        self.finished = []
        self.used = 0
        self.peak_used = 0
        self.stage_updates = 0.0
        self.cv = threading.Condition()
        self.stopping = False
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    # -- device hooks --------------------------------------------------------
    def _device_stream(self):
        import torch
        return torch.cuda.Stream(device=self.device)

    def _device_batch(self, key, capacity, stream):
        n, prec = key
        # 1D classes choose between the resident kernel and the pass kernels
        # by timing both (up to 25% apart); for 3D classes only the block
        # size is open (about 2%), and timing a full 128^3 class takes a second
        flags = spstd.AUTOTUNE if len(n) == 1 else 0
        return spstd.Batch(n, self.coeffs, capacity=capacity, nprobes=self.nprobes,
                           nsteps_max=self.max_steps, precision=prec, device=self.device,
                           stream=stream, flags=flags)

    def _device_workspace_bytes(self, key, capacity):
        n, prec = key
        d = spstd.make_batch_desc(n, self.coeffs, capacity, self.nprobes, self.max_steps, prec)
        return spstd.batch_workspace_size(d) + 256       # Batch aligns its base to 256 bytes

    # -- dispatcher: routing, budget -----------------------------------------
    def _open_class(self, key):
        """Open a class with as many slots (up to max_slots) as the budget
        leaves room for; None if not even one fits."""
        one, two = self._workspace_bytes(key, 1), self._workspace_bytes(key, 2)
        per, base = two - one, one - (two - one)
        room = self.budget - self.used - base
        cap = min(self.max_slots, room // per) if per > 0 else 0
        if cap < 1:
            return None
        nbytes = self._workspace_bytes(key, int(cap))
        c = _Class(key, int(cap), nbytes)
        self.classes[key] = c
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        c.thread = threading.Thread(target=self._worker, args=(c,), daemon=True)
        c.thread.start()
        return c

    def _reap(self):
        """Drop classes whose workers have exited, returning their budget."""
        for key in [k for k, c in self.classes.items() if c.finished]:
            c = self.classes.pop(key)
            c.thread.join()
            self.used -= c.bytes
            if c.error is not None:
                raise c.error

    def _route(self):
        """Move blocked requests into their classes in arrival order,
        opening classes as the budget allows; a request that cannot be
        placed holds back every later one (no overtaking, so no class
        starves).  While requests wait, close classes that have been empty
        for idle_close_s."""
        with self.cv:
            self._reap()
            still = deque()
            while self.blocked:
                r = self.blocked.popleft()
                c = None
                if not still:
                    c = self.classes.get(r.key)
                    if c is None:
                        c = self._open_class(r.key)
                    elif c.closing:
                        c = None
                if c is None:
                    still.append(r)
                    continue
                c.queue.append(r)
            self.blocked = still
            if self.blocked:
                t = self.now()
                for c in self.classes.values():
                    if (not c.closing and not c.queue and not c.slots and c.idle_since is not None
                            and t - c.idle_since >= self.idle_close_s):
                        c.closing = True
            self.cv.notify_all()

    def submit(self, req: Request):
        if req.steps > self.max_steps:
            raise ValueError("request has more steps than the server's probe buffers hold")
        with self.cv:
            self.blocked.append(req)

    # -- worker: one class ----------------------------------------------------
    def _admit(self, c, batch):
        with self.cv:
            free = [s for s in range(c.capacity) if s not in c.slots]
            take = []
            while c.queue and free:
                take.append((free.pop(0), c.queue.popleft()))
        for s, r in take:
            w = r.work
            r.dt = batch.load(s, w.dx, w.V, w.psiR, w.psiI, w.probes[: self.nprobes],
                              cfl_fraction=w.cfl_fraction, hbar=w.hbar, mass=w.mass)
            c.slots[s] = r
            r.admitted = self.now()
            r.status = "running"

    def _chunk_steps(self, c, batch):
        left = min(r.steps - batch.slot_info(s)[1] for s, r in c.slots.items())
        if c.step_s is None:
            k = 16                          # first chunk: measures the step time
        else:
            k = int(self.chunk_s / max(c.step_s, 1e-7))
        return max(1, min(k, left, self.chunk))

    def _harvest(self, c, batch):
        for s, r in list(c.slots.items()):
            if batch.slot_info(s)[1] < r.steps:
                continue
            ser, _, _, _ = batch.read(s, state=False)
            E, _ = spstd.spectrum(ser, r.dt, hbar=r.work.hbar, nlevels=r.nlevels)
            r.E = E
            if self.keep_series:
                r.series = ser
            batch.release(s)
            del c.slots[s]
            r.done = self.now()
            r.status = "done"
            with self.cv:
                self.finished.append(r)
                self.cv.notify_all()

    def _worker(self, c):
        batch = None
        try:
            stream = self._stream_factory()
            batch = self._batch_factory(c.key, c.capacity, stream)
            while True:
                with self.cv:
                    while not c.queue and not c.slots and not (c.closing or self.stopping):
                        if c.idle_since is None:
                            c.idle_since = self.now()
                        self.cv.wait(timeout=0.05)
                    if self.stopping or (not c.queue and not c.slots):
                        break                       # stopped, or closing with nothing left
                    c.idle_since = None
                self._admit(c, batch)
                k = self._chunk_steps(c, batch)
                if self._gate:
                    self._gate.acquire()
                try:
                    t0 = time.perf_counter()
                    batch.step(k)
                    stream.synchronize()
                    el = time.perf_counter() - t0
                finally:
                    if self._gate:
                        self._gate.release()
                c.step_s = el / k if c.step_s is None else 0.5 * c.step_s + 0.5 * el / k
                with self.cv:
                    self.stage_updates += len(c.slots) * batch.npoints * k * self.subs / 2.0
                self._harvest(c, batch)
        except BaseException as e:          # reported by the dispatcher
            c.error = e
        finally:
            del batch
            with self.cv:
                c.finished = True
                self.cv.notify_all()

    # -- the loop ---------------------------------------------------------------
    def run(self, requests, time_limit=None, progress=None, progress_every=20.0):
        """Serve requests whose ``arrival`` times are offsets on the server's
        clock; returns them when all have finished (or at the time limit:
        the workers stop after their current chunk).
        ``progress(now, finished, total)`` is called every ``progress_every``
        seconds if given."""
        if self._batch_factory == self._device_batch:
            spstd.lib()                     # loaded once, before the workers start
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        total = len(pending)
        start_done = len(self.finished)
        self.t0 = time.perf_counter()
        self.stopping = False
        next_report = progress_every
        try:
            while True:
                t = self.now()
                while pending and pending[0].arrival <= t:
                    self.submit(pending.popleft())
                self._route()
                with self.cv:
                    if len(self.finished) - start_done >= total:
                        break
                    wait = 0.005
                    if pending:
                        wait = min(wait, max(0.0, pending[0].arrival - self.now()))
                    self.cv.wait(timeout=wait)
                if progress is not None and self.now() >= next_report:
                    progress(self.now(), len(self.finished) - start_done, total)
                    next_report += progress_every
                if time_limit is not None and self.now() > time_limit:
                    break
        finally:
            with self.cv:
                self.stopping = True
                for c in self.classes.values():
                    c.closing = True
                self.cv.notify_all()
            for c in list(self.classes.values()):
                c.thread.join()
            with self.cv:
                self._reap()
        return requests

    def busy(self):
        with self.cv:
            return bool(self.blocked) or any(c.slots or c.queue for c in self.classes.values())


def latency_summary(reqs, elapsed, stage_updates):
    lat = np.array([r.latency for r in reqs if r.latency is not None])
    return {"requests": int(len(lat)),
            "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_s": float(lat.mean()) if len(lat) else None,
            "stage_updates_per_s": stage_updates / elapsed if elapsed > 0 else None,
            "completed_per_s": len(lat) / elapsed if elapsed > 0 else None}


def request_mix(count, rate, seed=0, steps=(2000, 20000), p1d=0.8,
                sizes_1d=(1024, 2048, 4096, 8192, 16384), sizes_3d=((32, 0.6), (64, 0.3), (128, 0.1)),
                p_fp32=0.5, box=20.0):
    """Seeded requests: Poisson arrivals at `rate` per second; 1D (prob.
    p1d) or 3D grids; square or harmonic wells as in the batching workload;
    FP32 or FP64; step counts uniform in `steps`."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < p1d:
            n = int(rng.choice(sizes_1d))
            shape = (n,)
        else:
            ns, ps = zip(*sizes_3d)
            n = int(rng.choice(ns, p=np.asarray(ps) / sum(ps)))
            shape = (n, n, n)
        w = _well_instance(shape, int(rng.integers(1 << 30)), box)
        prec = spstd.FP32 if rng.uniform() < p_fp32 else spstd.FP64
        st = int(rng.integers(steps[0], steps[1] + 1))
        out.append(Request(i, w, st, prec, arrival=t))
    return out


def _well_instance(shape, seed, box):
    """A square or harmonic well on [-box, box)^dim with a Gaussian start
    (the instance recipe of the batching workload, any dimension)."""
    rng = np.random.default_rng(seed)
    dim = len(shape)
    n = shape[0]
    d = 2.0 * box / n
    x = W.axis_coords(n, -box, box)
    grids = np.meshgrid(*([x] * dim), indexing="ij")[::-1]
    if rng.uniform() < 0.5:
        width, depth = rng.uniform(2.0, 20.0), rng.uniform(1.0, 50.0)
        inside = np.ones_like(grids[0], dtype=bool)
        for g in grids:
            inside &= np.abs(g) < width / 2
        V = np.where(inside, 0.0, depth)
        spread = width / 2
    else:
        om = rng.uniform(0.5, 2.0)
        V = 0.5 * om ** 2 * sum(g ** 2 for g in grids)
        spread = min(box / 2, 2.0 / np.sqrt(om))
    psi = np.zeros(V.shape)
    centres = []
    for _ in range(3):
        c = rng.uniform(-spread, spread, dim) * 0.6
        centres.append(c)
        psi += rng.normal() * np.exp(-sum((g - cc) ** 2 for g, cc in zip(grids, c)) / 0.5)
    # probe half a width from the first Gaussian, where the state has weight
    pc = centres[0] + 0.3
    idx = [min(n - 1, max(0, W.snap(v, -box, d))) for v in pc]
    lin = 0
    for k in reversed(range(dim)):
        lin = lin * n + idx[k]
    return W.Workload(f"req_{seed}", shape, (d,) * dim, (-box,) * dim,
                      np.ascontiguousarray(V.ravel(), np.float64),
                      np.ascontiguousarray(psi.ravel(), np.float64), np.zeros(V.size),
                      np.array([lin], np.int64), 0, W.PAPER)
