"""Batching form: many independent instances of uneven sizes advanced together.

Instances are grouped by grid shape; each group is one ``spstd.Batch``
(one launch per pass for the whole group, or one resident launch for short
1D grids), and every group runs on its own stream so that groups overlap on
the device.  Host code only orchestrates; the solver runs in the library.
"""
from __future__ import annotations

import time
from collections import defaultdict

import numpy as np

from . import spstd


def run_instances(instances, steps, precision=spstd.FP32, coeffs=None, nprobes=1,
                  device="cuda", dt=None, warmup=0):
    """Advance every instance by `warmup` untimed and then `steps` timed
    steps; returns (results, stats).

    results[i] = (probe series [(warmup+steps+1), nprobes, 2], dt); stats
    holds the elapsed device time of the timed steps (wall clock around the
    stepping, inputs resident; warm-up steps capture the step graphs), the
    stage updates done in them and the group layout."""
    import torch
    groups = defaultdict(list)
    for i, w in enumerate(instances):
        groups[tuple(w.n)].append(i)
    coeffs = coeffs if coeffs is not None else instances[0].coeffs
    subs = sum(1 for x in coeffs[0] if x) + sum(1 for x in coeffs[1] if x)
    batches, dts = {}, {}
    for shape, idx in groups.items():
        st = torch.cuda.Stream(device=device)
        b = spstd.Batch(shape, coeffs, capacity=len(idx), nprobes=nprobes, nsteps_max=steps + warmup,
                        precision=precision, device=device, stream=st, flags=spstd.AUTOTUNE)
        for s, i in enumerate(idx):
            w = instances[i]
            dts[i] = b.load(s, w.dx, w.V, w.psiR, w.psiI, w.probes[:nprobes],
                            dt=0.0 if dt is None else dt[i], cfl_fraction=w.cfl_fraction,
                            hbar=w.hbar, mass=w.mass)
        batches[shape] = (b, st, idx)
    if warmup > 0:
        for b, st, _ in batches.values():
            b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, st, _ in batches.values():
        b.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    results = {}
    for b, st, idx in batches.values():
        for s, i in enumerate(idx):
            ser, _, _, _ = b.read(s, state=False)
            results[i] = (ser, dts[i])
    su = sum(np.prod(w.n) for w in instances) * steps * subs / 2.0
    stats = {"elapsed_s": el, "stage_updates": su, "stage_updates_per_s": su / el,
             "groups": {str(k): len(v[2]) for k, v in batches.items()},
             "schedules": {str(k): v[0].schedule()[:2] for k, v in batches.items()},
             "points": int(sum(np.prod(w.n) for w in instances))}
    return results, stats
