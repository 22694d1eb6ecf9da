"""Serving loop: eigenvalue-solve requests with continuous batching.

Requests of one grid shape and precision form a class; each class owns one
batch (``spstd.Batch``) whose slots hold the wavefunctions of its admitted
requests on the device for their whole run.  A tick of the loop

1. admits waiting requests (first come, first served) into free slots of
   their class, creating the class's batch on first use when its workspace
   fits the HBM budget;
2. advances every class that has active slots and no chunk in flight by K
   steps, K = min(chunk, the smallest remaining step count among its active
   slots), each class on its own stream so that classes run concurrently on
   the device and all requests of a class share every launch;
3. polls each class's last chunk (a HIP event, no device-wide wait); when it
   has completed, finishes the requests whose step count is reached: reads
   their probe series, extracts eigenvalues with ``spstd.spectrum`` and
   frees their slots.  Classes advance independently: a slow class never
   holds back a fast one.

Requests that arrive while others are running are admitted at the next
tick as slots and budget allow.  Latency is measured from arrival to the
result; throughput is counted in grid-point stage updates.

The loop itself is host orchestration (Python); every step of the solver
runs in the library's kernels.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

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


@dataclass
class _Class:
    key: tuple
    batch: spstd.Batch
    stream: object
    bytes: int
    slots: dict = field(default_factory=dict)   # slot -> Request
    idle_ticks: int = 0
    event: object = None                        # completion of the chunk in flight

    def free_slots(self):
        return [s for s in range(self.batch.capacity) if s not in self.slots]


class Server:
    """Continuous-batching eigenvalue server on one GPU."""

    def __init__(self, hbm_budget, coeffs=W.PAPER, chunk=512, max_slots=64, max_steps=20000,
                 nprobes=1, device="cuda", keep_series=True, resident_chunk=2048,
                 max_concurrent=6):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget)
        self.coeffs = coeffs
        self.chunk = int(chunk)
        # 1D classes run a whole chunk in one launch; longer chunks cost them
        # nothing, shorter ones bound how long an arrival waits for a slot
        self.resident_chunk = int(resident_chunk)
        # classes stepping at once: small latency-bound classes slow each
        # other down when too many share the device, so the classes holding
        # the oldest requests go first
        self.max_concurrent = int(max_concurrent)
        self.max_slots = int(max_slots)
        self.max_steps = int(max_steps)
        self.nprobes = int(nprobes)
        self.device = device
        self.keep_series = keep_series
        self.classes = {}
        self.waiting = deque()
        self.finished = []
        self.used = 0
        self.stage_updates = 0.0
        self.peak_used = 0
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    # -- admission ---------------------------------------------------------
    def _slot_bytes(self, key):
        n, prec = key
        d1 = spstd.make_batch_desc(n, self.coeffs, 1, self.nprobes, self.max_steps, prec)
        d2 = spstd.make_batch_desc(n, self.coeffs, 2, self.nprobes, self.max_steps, prec)
        b1, b2 = spstd.batch_workspace_size(d1), spstd.batch_workspace_size(d2)
        return b2 - b1, b1 - (b2 - b1)

    def _open_class(self, key):
        per, base = self._slot_bytes(key)
        room = self.budget - self.used - base - 256
        cap = min(self.max_slots, room // per) if per > 0 else 0
        if cap < 1:
            return None
        n, prec = key
        stream = self.torch.cuda.Stream(device=self.device)
        # 1D classes choose between the resident kernel and the pass kernels
        # by timing both (up to 25% apart); for 3D classes only the block
        # size is open (about 2%), and timing a full 128^3 class takes a
        # second during which the loop does not tick
        flags = spstd.AUTOTUNE if len(n) == 1 else 0
        b = spstd.Batch(n, self.coeffs, capacity=int(cap), nprobes=self.nprobes,
                        nsteps_max=self.max_steps, precision=prec, device=self.device,
                        stream=stream, flags=flags)
        nbytes = b.ws.numel()
        c = _Class(key, b, stream, nbytes)
        self.classes[key] = c
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        return c

    def _close_idle_classes(self):
        """Free the batches of classes that are empty while requests wait
        for budget."""
        if not self.waiting:
            return
        for key in list(self.classes):
            c = self.classes[key]
            if not c.slots and c.idle_ticks > 0 and c.event is None:
                self.used -= c.bytes
                del self.classes[key]

    def submit(self, req: Request):
        if req.steps > self.max_steps:
            raise ValueError("request has more steps than the server's probe buffers hold")
        self.waiting.append(req)

    def _admit(self):
        still = deque()
        while self.waiting:
            r = self.waiting.popleft()
            c = self.classes.get(r.key) or self._open_class(r.key)
            free = c.free_slots() if (c is not None and c.event is None) else []
            if not free:
                still.append(r)
                continue
            s = free[0]
            w = r.work
            r.dt = c.batch.load(s, w.dx, w.V, w.psiR, w.psiI, w.probes[: self.nprobes],
                                cfl_fraction=w.cfl_fraction, hbar=w.hbar, mass=w.mass)
            c.slots[s] = r
            r.admitted = self.now()
            r.status = "running"
        self.waiting = still

    # -- one tick ------------------------------------------------------------
    def _harvest(self, c):
        done = []
        for s, r in list(c.slots.items()):
            if c.batch.slot_info(s)[1] >= r.steps:
                ser, _, _, _ = c.batch.read(s, state=False)
                E, _ = spstd.spectrum(ser, r.dt, hbar=r.work.hbar, nlevels=r.nlevels)
                r.E = E
                if self.keep_series:
                    r.series = ser
                c.batch.release(s)
                del c.slots[s]
                r.done = self.now()
                r.status = "done"
                done.append(r)
        return done

    def tick(self):
        """One pass over the classes; returns the requests finished in it."""
        done = []
        # classes whose chunk has completed: finish their requests
        for c in self.classes.values():
            if c.event is not None and c.event.query():
                c.event = None
                done.extend(self._harvest(c))
        self._close_idle_classes()
        # admission only into classes with nothing in flight (loading a slot
        # synchronises the class's stream)
        if self.waiting:
            self._admit()
        subs = sum(1 for x in self.coeffs[0] if x) + sum(1 for x in self.coeffs[1] if x)
        running = sum(1 for c in self.classes.values() if c.event is not None)
        ready = []
        for c in self.classes.values():
            if c.event is not None:
                continue
            if not c.slots:
                c.idle_ticks += 1
                continue
            c.idle_ticks = 0
            ready.append(c)
        ready.sort(key=lambda c: min(r.arrival for r in c.slots.values()))
        for c in ready[: max(0, self.max_concurrent - running)]:
            left = min(r.steps - c.batch.slot_info(s)[1] for s, r in c.slots.items())
            cap = self.resident_chunk if len(c.key[0]) == 1 else self.chunk
            k = max(1, min(cap, left))
            c.batch.step(k)
            c.event = self.torch.cuda.Event()
            c.event.record(c.stream)
            self.stage_updates += len(c.slots) * c.batch.npoints * k * subs / 2.0
        self.finished.extend(done)
        return done

    def busy(self):
        return bool(self.waiting) or any(c.slots for c in self.classes.values())

    def run(self, requests, time_limit=None, progress=None, progress_every=20.0):
        """Serve requests whose ``arrival`` times are offsets on the server's
        clock; returns them when all have finished (or at the time limit).
        ``progress(now, finished, total)`` is called every ``progress_every``
        seconds if given."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        self.t0 = time.perf_counter()
        next_report = progress_every
        while pending or self.busy():
            if progress is not None and self.now() >= next_report:
                progress(self.now(), len(self.finished), len(requests))
                next_report += progress_every
            t = self.now()
            while pending and pending[0].arrival <= t:
                self.submit(pending.popleft())
            if not self.busy():
                time.sleep(max(0.0, min(0.01, pending[0].arrival - t)))
                continue
            if not self.tick():
                time.sleep(2e-4)        # nothing finished: let the device work
            if time_limit is not None and self.now() > time_limit:
                break
        return requests


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
