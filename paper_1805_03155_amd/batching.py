"""Batching form: many independent instances of uneven sizes advanced together.

Instances are grouped by grid shape into ``spstd.Batch`` objects.  The 2D
shapes that the pass kernels step (128 to 512 points per axis) form one
``spstd.BatchGroup``: every pass of a stage is one persistent launch over
all of them, with the schedule the group's tuner picked.  1D and small 2D
shapes run their resident kernels (a whole chunk of steps per launch), each
on its own stream so that they overlap with the group on the device.  Host
code only orchestrates; the solver runs in the library.
"""
from __future__ import annotations

import time
from collections import defaultdict

import numpy as np

from . import spstd


def run_instances(instances, steps, precision=spstd.FP32, coeffs=None, nprobes=1,
                  device="cuda", dt=None, warmup=0, group="auto", trial=64):
    """Advance every instance by `warmup` untimed and then `steps` timed
    steps; returns (results, stats).

    The 2D shapes that the pass kernels step (128 to 512 points per axis)
    either form one ``spstd.BatchGroup`` (one persistent launch per pass for
    all of them) or step on their own streams beside the others.  group:
    True or False fixes that; "auto" times `trial` steps of each on the
    loaded workload after the warm-up and keeps the faster for the timed
    steps (the trial steps are untimed steps of every instance, like the
    warm-up).

    results[i] = (probe series [(untimed + steps + 1), nprobes, 2], dt);
    stats holds the elapsed device time of the timed steps (wall clock
    around the stepping, inputs resident; warm-up steps capture the step
    graphs), the stage updates done in them, the layout and the schedules."""
    import torch
    shapes = defaultdict(list)
    for i, w in enumerate(instances):
        shapes[tuple(w.n)].append(i)
    coeffs = coeffs if coeffs is not None else instances[0].coeffs
    subs = sum(1 for x in coeffs[0] if x) + sum(1 for x in coeffs[1] if x)
    npts = sum(np.prod(w.n) for w in instances)
    untimed = warmup + (2 * trial if group == "auto" else 0)
    batches, dts = {}, {}
    for shape, idx in shapes.items():
        st = torch.cuda.Stream(device=device)
        # long 1D rows keep one workgroup per row pair: their four-step form
        # (five launches per x pass over many workgroups) is the faster alone
        # but takes more of the device from the group beside it (512
        # instances: 1.29e11 against 1.35e11 stage updates/s)
        flags = spstd.AUTOTUNE | (spstd.NO_FOURSTEP if len(shape) == 1 else 0)
        b = spstd.Batch(shape, coeffs, capacity=len(idx), nprobes=nprobes, nsteps_max=steps + untimed,
                        precision=precision, device=device, stream=st, flags=flags)
        batches[shape] = (b, st, idx)
    gshapes = [k for k, v in batches.items()
               if group is not False and spstd.group_ok(k) and v[0].schedule()[0] == "passes"]
    grp = None
    gstream = torch.cuda.Stream(device=device)
    if gshapes:
        # tuned on the empty members
        grp = spstd.BatchGroup([batches[k][0] for k in gshapes], flags=spstd.AUTOTUNE, device=device,
                               stream=gstream)
    gsched = None if grp is None else grp.schedule()
    for shape, (b, st, idx) in batches.items():
        for s, i in enumerate(idx):
            w = instances[i]
            dts[i] = b.load(s, w.dx, w.V, w.psiR, w.psiI, w.probes[:nprobes],
                            dt=0.0 if dt is None else dt[i], cfl_fraction=w.cfl_fraction,
                            hbar=w.hbar, mass=w.mass)

    def advance(n, use_group, chunk=16):
        # resident batches step the whole run in one launch each; the
        # graph-replayed pass batches and the group are enqueued a chunk
        # (one step graph) at a time in turn, so that every stream has work
        # from the start instead of the last one waiting for the host to
        # enqueue all of the others' graphs first (512 instances, 5000
        # steps: 1.35e11 against 1.21e11 stage updates/s)
        looped = []
        for k, (b, _, _) in batches.items():
            if use_group and k in gshapes:
                continue
            if b.schedule()[0] == "resident":
                b.step(n)
            else:
                looped.append(b)
        if use_group:
            looped.append(grp)
        done = 0
        while done < n:
            k = min(chunk, n - done)
            for b in looped:
                b.step(k)
            done += k

    def timed(n, use_group):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        advance(n, use_group)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    use_group = grp is not None
    if warmup > 0:
        advance(warmup, use_group)
    trials = None
    if grp is not None and group == "auto":
        t_group = timed(trial, True)
        grp.close()                  # the members step on their own streams again
        grp = None
        # the per-shape streams warm their graphs inside this trial's first chunk
        t_alone = timed(trial, False)
        trials = {"group_us_per_step": 1e6 * t_group / trial, "per_shape_streams_us_per_step": 1e6 * t_alone / trial}
        use_group = t_group < t_alone
        if use_group:
            grp = spstd.BatchGroup([batches[k][0] for k in gshapes], device=device, stream=gstream)
            grp.set_schedule(gsched[0])
    el = timed(steps, use_group)
    results = {}
    for b, st, idx in batches.values():
        for s, i in enumerate(idx):
            ser, _, _, _ = b.read(s, state=False)
            results[i] = (ser, dts[i])
    su = npts * steps * subs / 2.0
    stats = {"elapsed_s": el, "stage_updates": su, "stage_updates_per_s": su / el,
             "groups": {str(k): len(v[2]) for k, v in batches.items()},
             "schedules": {str(k): v[0].schedule()[:2] for k, v in batches.items()
                           if not (use_group and k in gshapes)},
             "points": int(npts),
             "workload_schedule": "group" if use_group else "per-shape streams",
             "trials": trials,
             "mixed_group": None if gsched is None else {
                 "shapes": [list(k) for k in gshapes],
                 "instances": int(sum(len(batches[k][2]) for k in gshapes)),
                 "schedule": gsched[0], "tuned_us_per_step": list(gsched[1])}}
    if grp is not None:
        grp.close()
    return results, stats
