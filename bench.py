#!/usr/bin/env python3
"""SPSTD throughput on one MI355X: grid-point stage updates per second.

Workload: the 3D isotropic harmonic oscillator on a 256^3 periodic grid over
[-12, 12)^3 (hbar = m* = 1, omega = 1), seeded off-centre Gaussian start,
Yoshida sixth-order 8-stage symplectic set (15 non-zero substeps per step),
dt = 0.5 x the stability limit, 3 probes.  One "step" is one full time step
of the hot path (every directional pass of every stage plus the probe
sample); the set's last stage has no B half, so within each chunk of 16
steps the A half ending one step and the A half opening the next run as one
(exact: they see the same psi_I).  A stage update is one A plus one B
substep at one grid point, so a step is 7.5 stage updates per point.

The timed region runs with per-pass HIP events on the plan's stream; the
dominant kernel's average duration gives the roofline entry.  The CPU oracle
is timed on a bounded sample of the same workload (rank 0, N = 1 only).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the serving and batching legs run one stream per request class or shape;
# with fewer hardware queues than streams, streams share in-order queues and
# a long chunk on one holds back the others' launches and copies.  Raised to
# 16 (not lowered) before HIP starts.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

METRIC = "grid-point stage updates/s (3D HO 256³, FP64 vs FP32); p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1805_03155_amd/csrc/kernels.hip", "paper_1805_03155_amd/csrc/passes.hpp",
                  "paper_1805_03155_amd/csrc/body_axis_acc.inc", "paper_1805_03155_amd/csrc/body_axis_ba.inc",
                  "paper_1805_03155_amd/csrc/body_x_ab.inc", "paper_1805_03155_amd/csrc/fft_core.hpp"]
KERNEL_NAMES = {"y": "k_axis_acc (y pass)", "z": "k_axis_acc (z pass)",
                "yba": "k_axis_ba (y passes of a stage boundary, fused)",
                "xab": "k_x_ab (fused A+B x pass)", "x": "k_x_acc (x half-stage)"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kind, prec):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it
    was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    if data.get("kernel_source_hash") != kernel_source_hash():
        return None
    ent = data.get("entries", {}).get(f"{prec}:{kind}")
    return None if ent is None else ent.get("hbm_bytes_per_launch")


def run_precision(w, prec, steps, warmup):
    import torch
    from paper_1805_03155_amd import spstd
    code = spstd.FP64 if prec == "fp64" else spstd.FP32
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    p = spstd.plan_from_workload(w, precision=code, nsteps_max=steps + warmup,
                                 flags=spstd.TIMING)
    setup_s = time.perf_counter() - s0   # host arrays in, over PCIe (not in the timed region)
    st = p.info()
    npts = w.npoints
    su_per_step = npts * st.substeps_per_step / 2.0
    p.step(warmup)
    p.pass_times()                       # synchronises; discards warm-up timings
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    times = p.pass_times()
    el = t1 - t0
    info = p.info()
    r0 = time.perf_counter()
    _, st2 = p.run(0)                    # norm check (raises on NaN/Inf), probe series out
    readback_s = time.perf_counter() - r0
    log(f"{prec}: {steps} steps in {el:.3f} s, norm drift {st2.norm / st2.norm0 - 1:.2e}")
    kinds = {k: v for k, v in times.items() if v[0] > 0}
    dom = max(kinds, key=lambda k: kinds[k][1])
    n, ms, by = kinds[dom]
    avg_s = ms / n / 1e3
    achieved = by / avg_s / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(dom, prec),
            "kernel": KERNEL_NAMES[dom], "avg_launch_us": avg_s * 1e6,
            "algorithmic_bytes_per_launch": by}
    per_kernel = {KERNEL_NAMES[k]: {"launches": v[0], "avg_us": v[1] / v[0] * 1e3,
                                    "GBps": v[2] / (v[1] / v[0] / 1e3) / 1e9,
                                    "share_of_pass_time": v[1] / sum(x[1] for x in kinds.values())}
                  for k, v in kinds.items()}
    # graph-replayed steps (the default execution mode) for reference
    # its warm-up covers at least one 16-step chunk, so that the chunk's graph
    # is captured and instantiated before the timed region
    gw = max(warmup, 32)
    q = spstd.plan_from_workload(w, precision=code, nsteps_max=steps + gw)
    q.step(gw)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    q.step(steps)
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    del q
    # the same graph-replayed steps with every step boundary kept (no merged
    # A halves): the rate the stage sequence gives without the merge
    u = spstd.plan_from_workload(w, precision=code, nsteps_max=steps + gw, flags=spstd.NO_MERGE)
    u.step(gw)
    torch.cuda.synchronize()
    u0 = time.perf_counter()
    u.step(steps)
    torch.cuda.synchronize()
    u1 = time.perf_counter()
    del u
    pcie = {"plan_setup_s": setup_s, "readback_s": readback_s,
            "value_including_transfers": su_per_step * steps / (el + setup_s + readback_s)}
    # whole-step byte accounting: the passes' algorithmic bytes over the
    # timed steps; the irreducible bytes of a stage update (read f, V, g and
    # write g once per half-stage: 64 B FP64, 32 B FP32) at the measured
    # rate; and the per-axis 3D FFT schedule model (192 B / 96 B), whose
    # fraction only says how far the engine's schedule is from that one
    rate = su_per_step * steps / el
    step_bytes = sum(v[0] * v[2] for v in kinds.values()) / steps
    model_b = 192.0 if prec == "fp64" else 96.0
    irred_b = 64.0 if prec == "fp64" else 32.0
    step_model = {"engine_bytes_per_stage_update": step_bytes / su_per_step,
                  "engine_GBps_over_step": step_bytes / (el / steps) / 1e9,
                  "engine_frac_over_step": step_bytes / (el / steps) / 1e9 / HBM_PEAK_GBS,
                  "irreducible_bytes_per_stage_update": irred_b,
                  "irreducible_frac": irred_b * rate / (HBM_PEAK_GBS * 1e9),
                  "schedule_model_bytes_per_stage_update": model_b,
                  "schedule_model_ratio_not_bandwidth": model_b * rate / (HBM_PEAK_GBS * 1e9)}
    return {"value": rate, "ms_per_step": el / steps * 1e3, "host_transfers": pcie, "bytes": step_model,
            "roofline": roof, "kernels": per_kernel, "dt": info.dt,
            "graph_mode": {"value": su_per_step * steps / (g1 - g0),
                           "ms_per_step": (g1 - g0) / steps * 1e3,
                           "without_merged_boundaries": {"value": su_per_step * steps / (u1 - u0),
                                                         "ms_per_step": (u1 - u0) / steps * 1e3}},
            "stage_updates_per_step": su_per_step}


def cpu_baseline(w, steps):
    import oracle
    c, d = w.coeffs
    dt = oracle.stable_dt(c, d, w.V, w.n, w.dx)
    nsub = sum(1 for x in c if x != 0.0) + sum(1 for x in d if x != 0.0)
    t0 = time.perf_counter()
    ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, c, d, dt, steps, w.probes)
    el = time.perf_counter() - t0
    su = w.npoints * nsub / 2.0 * steps
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    out = {"value": su / el, "unit": "stage updates/s", "cores": oracle.num_threads(),
           "cpu_model": model, "host_cpus": os.cpu_count(), "kind": "oracle",
           "sample": f"{steps} full time step(s) ({nsub} substeps each) of the "
                     f"{'x'.join(str(k) for k in w.n)} FP64 oracle run, {el:.1f} s wall"}
    return out, (dt, steps, ro, io, so)


def accuracy_vs_oracle(w, ref):
    """Error of each precision against the FP64 oracle: the state and probe
    samples after the CPU baseline's steps of the bench workload (same dt),
    and the levels of the 1D finite-well workload (20000 steps, paper set)
    against the oracle's levels of the same run."""
    import numpy as np
    import oracle
    from oracle import spectrum
    from paper_1805_03155_amd import spstd
    from paper_1805_03155_amd import workloads as W
    dt, steps, ro, io, so = ref
    b = np.concatenate([ro, io])
    fw = W.finite_well_1d(seed=0)
    c, d = fw.coeffs
    fdt = oracle.stable_dt(c, d, fw.V, fw.n, fw.dx)
    _, _, fso, _ = oracle.run(fw.psiR, fw.psiI, fw.V, fw.n, fw.dx, c, d, fdt, fw.steps, fw.probes)
    E_or, _ = spectrum.extract(fso, fdt, 1.0, 4)
    out = {"reference": "FP64 oracle",
           "state": f"{'x'.join(str(k) for k in w.n)} bench workload after {steps} steps",
           "levels": "1D finite well (256 points, 20000 steps, paper set), lowest 4 levels",
           "oracle_levels": [float(e) for e in E_or]}
    for name, code in (("fp64", spstd.FP64), ("fp32", spstd.FP32)):
        p = spstd.plan_from_workload(w, precision=code, dt=dt, nsteps_max=steps)
        ser, _ = p.run(steps)
        r, i, _ = p.get_state()
        del p
        a = np.concatenate([r, i])
        q = spstd.plan_from_workload(fw, precision=code, dt=fdt, nsteps_max=fw.steps)
        fser, _ = q.run(fw.steps)
        del q
        E, _ = spstd.spectrum(fser, fdt, nlevels=4)
        k = min(len(E), len(E_or))
        out[name] = {"psi_rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                     "probe_rel_l2": float(np.linalg.norm(ser - so) / np.linalg.norm(so)),
                     "level_rel_err": [float(abs(E[j] - E_or[j]) / abs(E_or[j])) for j in range(k)]}
        log(f"accuracy {name}: psi rel-L2 {out[name]['psi_rel_l2']:.2e}, "
            f"levels max rel err {max(out[name]['level_rel_err']):.2e}")
    return out


def batching_leg(count, steps, seed=0):
    """The batching workload: `count` seeded 1D/2D instances of uneven sizes
    (1D 2^7..2^14, 2D 32^2..512^2, square or harmonic wells), FP32 fields
    with FP64 probes, paper coefficient set; one batch per shape; the 2D
    shapes of 128^2..512^2 either stepped together as one group (one launch
    per pass) or on their own streams, whichever a 64-step trial of each on
    the loaded workload finds faster; the others by their resident
    kernels."""
    from paper_1805_03155_amd import batching, spstd
    from paper_1805_03155_amd import workloads as W
    inst = W.batch_instances(count=count, seed=seed, steps=steps)
    _, st = batching.run_instances(inst, steps, precision=spstd.FP32, warmup=32)
    # schedules the autotuner chose, counted over the shape groups
    picks = {}
    for sched, wpb in st["schedules"].values():
        k = "resident" if sched == "resident" else f"passes_{wpb}_waves"
        picks[k] = picks.get(k, 0) + 1
    return {"value": st["stage_updates_per_s"], "unit": "stage updates/s", "instances": count,
            "steps": steps, "points": st["points"], "elapsed_s": st["elapsed_s"],
            "shape_groups": len(st["groups"]), "workload_schedule": st["workload_schedule"],
            "trials_us_per_step": st["trials"], "schedules_outside_the_group": picks,
            "mixed_group": st["mixed_group"], "dtype": "f32 fields, f64 probes"}


def pmc_batch(count=512, steps=48, seed=0):
    """Short run of the batching workload for hardware-counter passes: the
    same 512 seeded instances, FP32, the 2D shapes of 128^2..512^2 as one
    group with its built-in schedule, 48 steps (resident launches of whole
    chunks, the group's kernels and the long-row pass kernels)."""
    from paper_1805_03155_amd import batching, spstd
    from paper_1805_03155_amd import workloads as W
    inst = W.batch_instances(count=count, seed=seed, steps=steps)
    _, st = batching.run_instances(inst, steps, precision=spstd.FP32, group=True)
    print(json.dumps({"pmc_batch": True, "instances": count, "steps": steps,
                      "stage_updates": st["stage_updates"]}), flush=True)


def class_step_times(steps=1000, warmup=64, seed=5):
    """Per-step time of serving classes alone: one batch of 1 or 8 seeded
    requests of one shape and precision (the server's flags: 1D classes
    autotuned, 3D classes with the fused x-z planes and, for comparison,
    with the separate passes), `warmup` untimed steps (graph capture), then
    `steps` timed steps on the batch's stream."""
    import torch
    from paper_1805_03155_amd import serve, spstd
    from paper_1805_03155_amd import workloads as W
    out = []
    cases = [((n,), 0) for n in (1024, 16384)]
    cases += [((n, n, n), f) for n in (32, 64, 128) for f in (0, spstd.NO_PLANES)]
    for shape, extra in cases:
        for prec in (spstd.FP64, spstd.FP32):
            for k in (1, 8):
                if len(shape) == 3 and shape[0] == 128 and extra:
                    continue                 # 128^3 has no plane form
                reqs = serve.request_mix(k, 1.0, seed=seed, p1d=1.0 if len(shape) == 1 else 0.0,
                                         sizes_1d=(shape[0],), sizes_3d=((shape[0], 1.0),))
                st = torch.cuda.Stream()
                flags = (spstd.AUTOTUNE if len(shape) == 1 else 0) | extra
                b = spstd.Batch(shape, W.PAPER, capacity=k, nprobes=1, nsteps_max=steps + warmup,
                                precision=prec, stream=st, flags=flags)
                for s, r in enumerate(reqs):
                    w = r.work
                    b.load(s, w.dx, w.V, w.psiR, w.psiI, w.probes[:1], cfl_fraction=w.cfl_fraction,
                           hbar=w.hbar, mass=w.mass)
                b.step(warmup)
                st.synchronize()
                t0 = time.perf_counter()
                b.step(steps)
                st.synchronize()
                us = 1e6 * (time.perf_counter() - t0) / steps
                rec = {"shape": list(shape), "precision": "fp64" if prec == spstd.FP64 else "fp32",
                       "slots": k, "form": ("separate passes" if extra else "planes") if len(shape) == 3
                       else b.schedule()[0], "us_per_step": us}
                log(f"class {rec}")
                out.append(rec)
                del b
    return out


def serving_leg(count, rate, steps, seed=0, budget_gb=64):
    """Poisson arrivals of eigenvalue-solve requests (1D 1024..16384 points
    or 3D 32^3..128^3, 80/20; FP32 or FP64; square or harmonic wells), served
    with continuous batching under an HBM budget."""
    from paper_1805_03155_amd import serve
    reqs = serve.request_mix(count, rate, seed=seed, steps=steps)
    srv = serve.Server(hbm_budget=budget_gb << 30, max_slots=64, max_steps=steps[1], keep_series=False)
    t0 = time.perf_counter()
    srv.run(reqs, progress=lambda t, k, n: log(f"  serving: {k}/{n} finished at {t:.0f} s"))
    el = time.perf_counter() - t0
    out = serve.latency_summary(reqs, el, srv.stage_updates)
    out.update({"rate_per_s": rate, "steps_range": list(steps), "budget_GB": budget_gb,
                "peak_workspace_GB": srv.peak_used / 2 ** 30, "elapsed_s": el})
    return out


def serving_sweep(count, rates, steps, budgets_gb=(64,), small_budget_gb=2, small_rate=30.0, small=True):
    """The serving workload at several offered rates (same seeded request
    mix at each rate), plus (small) one run whose HBM budget forces
    queueing."""
    out = []
    for rate in rates:
        log(f"serving sweep: {count} requests at {rate}/s")
        r = serving_leg(count, rate, steps, budget_gb=budgets_gb[0])
        r["offered_per_s"] = rate
        out.append(r)
        log(f"  p50 {r['p50_s']:.2f} s, p99 {r['p99_s']:.2f} s, {r['completed_per_s']:.2f} done/s")
    if not small:
        return out
    log(f"serving sweep: {count} requests at {small_rate}/s under a {small_budget_gb} GB budget")
    r = serving_leg(count, small_rate, steps, budget_gb=small_budget_gb)
    r["offered_per_s"] = small_rate
    out.append(r)
    return out


def pmc_sample(w, steps):
    """Short run for hardware-counter passes: a plain device copy and an
    in-place add of known sizes (the calibration of FETCH_SIZE /
    WRITE_SIZE), then a few eager steps of the hot path in each precision."""
    import torch
    from paper_1805_03155_amd import spstd
    nbytes = 256 << 20
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    # a second streaming kernel of known bytes: b += a reads 2 and writes 1 array
    for _ in range(3):
        b.add_(a)
    torch.cuda.synchronize()
    del a, b
    for code in (spstd.FP64, spstd.FP32):
        p = spstd.plan_from_workload(w, precision=code, nsteps_max=steps, flags=spstd.EAGER)
        p.step(steps)
        torch.cuda.synchronize()
        del p
    print(json.dumps({"pmc_sample": True, "copy_bytes_each_way": nbytes, "steps": steps}))


def _advance(p, steps, chunk, label):
    """Queue steps in chunks, waiting for each so progress can be printed."""
    import torch
    done = 0
    t0 = time.perf_counter()
    while done < steps:
        k = min(chunk, steps - done)
        p.step(k)
        torch.cuda.synchronize()
        done += k
        log(f"{label}: {done}/{steps} steps, {time.perf_counter() - t0:.1f} s")
    return time.perf_counter() - t0


def precision_study(w, which, steps, nlevels=8):
    """Long runs of the 256^3 oscillator: FP64 and FP32 symplectic runs, or
    the RK4 run at the FP64 run's dt.  Reports rate, norm and energy drift,
    eigenvalues against the oscillator ladder (n + 3/2) hbar omega, and
    FP32 against FP64 (state and eigenvalues)."""
    import numpy as np
    from paper_1805_03155_amd import spstd
    exact = np.arange(nlevels) + 1.5
    out = {"workload": f"{w.n[0]}^3 oscillator, Yoshida-6, dt = 0.5 x limit", "steps": steps}
    runs = [("fp64", spstd.FP64, spstd.SYMPLECTIC), ("fp32", spstd.FP32, spstd.SYMPLECTIC)] \
        if which == "precision" else [("rk4", spstd.FP64, spstd.RK4)]
    dt64 = spstd.plan_from_workload(w, nsteps_max=1).dt
    states = {}
    for name, prec, method in runs:
        p = spstd.plan_from_workload(w, precision=prec, method=method, dt=dt64, nsteps_max=steps)
        st0 = p.info()
        kin0, pot0, nrm0 = p.energy()
        el = _advance(p, steps, 5000, name)
        series, st = p.run(0)
        kin1, pot1, nrm1 = p.energy()
        E, _ = spstd.spectrum(series, st.dt, nlevels=nlevels)
        r, i, _ = p.get_state()
        states[name] = (r, i, E)
        subs = st0.substeps_per_step
        res = {"seconds": el, "ms_per_step": el / steps * 1e3,
               "stage_updates_per_s": w.npoints * subs / 2.0 * steps / el,
               "dt": st.dt, "norm_drift": nrm1 / nrm0 - 1.0,
               "energy_drift": ((kin1 + pot1) / nrm1) / ((kin0 + pot0) / nrm0) - 1.0,
               "energy0": (kin0 + pot0) / nrm0,
               "levels": [float(x) for x in E]}
        k = min(len(E), nlevels)
        res["level_rel_err_vs_ladder"] = [float(abs(E[j] - exact[j]) / exact[j]) for j in range(k)]
        out[name] = res
        log(f"{name}: levels {np.round(E, 7).tolist()}, norm drift {res['norm_drift']:.2e}")
        del p
    if "fp32" in states:
        r64, i64, E64 = states["fp64"]
        r32, i32, E32 = states["fp32"]
        a, b = np.concatenate([r32, i32]), np.concatenate([r64, i64])
        k = min(len(E64), len(E32))
        out["fp32_vs_fp64"] = {
            "psi_rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
            "level_rel_err": [float(abs(E32[j] - E64[j]) / abs(E64[j])) for j in range(k)]}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256, help="grid points per axis")
    ap.add_argument("--cpu-baseline", choices=["on", "off"], default="on")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--batch-steps", type=int, default=5000,
                    help="steps of the 512-instance batching leg (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests per offered rate of the serving leg (0: skip)")
    ap.add_argument("--serve-rate", default="5,30",
                    help="offered rates of the serving leg (requests/s, comma-separated)")
    ap.add_argument("--pmc-sample", action="store_true",
                    help="short run for rocprofv3 counter passes (no timing output)")
    ap.add_argument("--pmc-batch", action="store_true",
                    help="short run of the batching workload for rocprofv3 counter passes")
    ap.add_argument("--study", choices=["precision", "rk4"],
                    help="long-run accuracy study instead of the timing line")
    ap.add_argument("--study-steps", type=int, default=100000)
    ap.add_argument("--serve-sweep", action="store_true",
                    help="serving at offered rates 10..1000/s instead of the timing line")
    ap.add_argument("--serve-rates", default="10,30,100,300,1000",
                    help="offered rates of --serve-sweep (requests/s, comma-separated)")
    ap.add_argument("--class-steps", type=int, default=0,
                    help="per-step time of serving classes alone over this many steps, instead of the timing line")
    ap.add_argument("--no-small-budget", action="store_true",
                    help="--serve-sweep without the small-budget run")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this engine has no multi-GPU path "
              "(one MI355X per run); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1805_03155_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    log(f"building the {args.n}^3 oscillator workload")
    w = W.harmonic_3d(seed=0, n=args.n, half_box=12.0, omega=1.0, steps=100000,
                      coeffs=W.YOSHIDA6, nprobes=3)
    if args.pmc_sample:
        pmc_sample(w, 2)
        return
    if args.pmc_batch:
        pmc_batch()
        return
    if args.study:
        print(json.dumps(precision_study(w, args.study, args.study_steps)), flush=True)
        return
    if args.class_steps > 0:
        print(json.dumps({"class_step_times": class_step_times(args.class_steps)}), flush=True)
        return
    if args.serve_sweep:
        rates = tuple(float(x) for x in args.serve_rates.split(","))
        sweep = serving_sweep(args.serve_requests, rates, (2000, 20000), small=not args.no_small_budget)
        print(json.dumps({"serving_sweep": sweep}), flush=True)
        return
    res = {}
    for prec in ("fp64", "fp32"):
        log(f"{prec}: warmup {args.warmup}, timed {args.steps} steps")
        res[prec] = run_precision(w, prec, args.steps, args.warmup)
    batch = serving = None
    if args.batch_steps > 0:
        log(f"batching leg: 512 instances, {args.batch_steps} steps")
        batch = batching_leg(512, args.batch_steps)
        log(f"batching: {batch['value']:.3e} stage updates/s")
    if args.serve_requests > 0:
        serving = []
        for rate in (float(x) for x in args.serve_rate.split(",")):
            log(f"serving leg: {args.serve_requests} requests at {rate}/s")
            r = serving_leg(args.serve_requests, rate, (2000, 20000))
            log(f"serving: p50 {r['p50_s']:.2f} s, p99 {r['p99_s']:.2f} s, "
                f"{r['completed_per_s']:.2f} completed/s")
            serving.append(r)
    cpu = accuracy = None
    if args.cpu_baseline == "on":
        log("timing the CPU oracle on a bounded sample")
        cpu, ref = cpu_baseline(w, args.cpu_steps)
        accuracy = accuracy_vs_oracle(w, ref)
    r64, r32 = res["fp64"], res["fp32"]
    line = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D harmonic oscillator {args.n}^3 on [-12,12)^3, "
                               "Yoshida-6 8-stage symplectic set, dt = 0.5 x stability limit, "
                               "3 probes",
                   "grid": [args.n] * 3, "stage_updates_per_step": r64["stage_updates_per_step"],
                   "dt": r64["dt"], "execution": "eager launches with per-pass HIP events",
                   "step_boundaries": "A halves of consecutive steps applied as one within 16-step chunks "
                                      "(the set's last stage has no B half)"},
        "roofline": r64["roofline"],
        "cpu_baseline": cpu,
        "kernels": r64["kernels"],
        "bytes": r64["bytes"],
        "graph_mode": r64["graph_mode"],
        "host_transfers": r64["host_transfers"],
        "batching": batch,
        "serving": serving,
        "accuracy": accuracy,
        "fp32": {"value": r32["value"], "ms_per_step": r32["ms_per_step"], "dtype": "f32",
                 "roofline": r32["roofline"], "kernels": r32["kernels"],
                 "graph_mode": r32["graph_mode"], "host_transfers": r32["host_transfers"],
                 "bytes": r32["bytes"],
                 "speedup_vs_fp64": r32["value"] / r64["value"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
