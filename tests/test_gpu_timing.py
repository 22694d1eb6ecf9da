"""Per-pass timing (SPSTD_TIMING plans, spstd_pass_times) on the GPU.

A timing plan brackets each pass launch with HIP events; back-to-back passes
share the event between them.  The launch counts per pass kind follow from
the stage sequence of Eq. (17) (A half y, z, x; B half x, z, y, with the
stage-boundary y passes fused and the two x halves of a stage fused), the
durations are positive and add up to no more than the wall time, and the
state is the one an untimed plan reaches.
"""
import time

import numpy as np
import pytest
import torch

from paper_1805_03155_amd import spstd
from paper_1805_03155_amd import workloads as W

pytestmark = pytest.mark.gpu


def case(n, seed=5, coeffs=W.PAPER):
    rng = np.random.default_rng(seed)
    N = int(np.prod(n))
    return W.Workload(f"t{seed}", tuple(n), (0.2,) * len(n), (0.0,) * len(n), 2.0 * rng.random(N),
                      rng.standard_normal(N), rng.standard_normal(N), np.array([3], np.int64), 0, coeffs)


# passes per step for the three-stage paper set (every c_l and d_l nonzero):
# stage 1 opens with a plain y pass, stages 2 and 3 with the fused boundary
# sweep, every stage has one fused x pass and two z passes, and the step
# ends with the y pass its last B half owes.  Within one call the boundaries
# between steps chain: each of the steps - 1 boundaries runs one fused sweep
# in place of the owed y pass and the next opening y pass (not with
# SPSTD_NO_MERGE)
@pytest.mark.parametrize("n,per_step", [((32, 16, 64), {"y": 2, "z": 6, "xab": 3, "x": 0, "yba": 2}),
                                        ((64, 32), {"y": 2, "z": 0, "xab": 3, "x": 0, "yba": 2}),
                                        ((256,), {"y": 0, "z": 0, "xab": 3, "x": 0, "yba": 0})])
@pytest.mark.parametrize("precision", [spstd.FP64, spstd.FP32])
@pytest.mark.parametrize("chained", [True, False])
def test_pass_counts_durations_and_state(n, per_step, precision, chained):
    steps = 10
    w = case(n)
    extra = 0 if chained else spstd.NO_MERGE
    p = spstd.plan_from_workload(w, precision=precision, nsteps_max=2 * steps + 2, flags=spstd.TIMING | extra)
    # the same pass kernels, replayed from graphs (1D plans would otherwise
    # take the resident kernel), with the same calls
    q = spstd.plan_from_workload(w, precision=precision, nsteps_max=2 * steps + 2,
                                 flags=spstd.NO_RESIDENT | extra)
    p.step(2)
    p.pass_times()                                  # discard the first steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.step(steps)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    t = p.pass_times()
    want = {k: v * steps for k, v in per_step.items()}
    if chained and len(n) >= 2:
        want["y"] -= 2 * (steps - 1)
        want["yba"] += steps - 1
    for kind, count in want.items():
        assert t[kind][0] == count, (kind, t[kind], count)
        if count:
            assert t[kind][1] > 0.0
    assert sum(v[1] for v in t.values()) <= wall_ms
    # nothing left over: a second call reports no launches
    assert all(v[0] == 0 for v in p.pass_times().values())
    q.step(2)
    q.step(steps)
    r, i, _ = p.get_state()
    rq, iq, _ = q.get_state()
    assert np.array_equal(r, rq) and np.array_equal(i, iq)


def test_rk4_pass_counts():
    # four K applications per step, each a y, z and x pass, for psi_R and psi_I
    steps = 5
    w = case((32, 16, 16))
    p = spstd.plan_from_workload(w, method=spstd.RK4, nsteps_max=steps, flags=spstd.TIMING)
    p.step(steps)
    t = p.pass_times()
    assert t["y"][0] == t["z"][0] == t["x"][0] == 8 * steps
    assert t["xab"][0] == t["yba"][0] == 0
    assert all(t[k][1] > 0.0 for k in ("y", "z", "x"))


def test_merged_boundaries_pass_counts():
    # Yoshida-6 ends on an A-only stage: within a chunk of 16 steps the 15
    # boundaries between steps each run one A half (y, z, x) instead of two
    steps = 16
    w = case((32, 16, 16), coeffs=W.YOSHIDA6)
    p = spstd.plan_from_workload(w, nsteps_max=steps, flags=spstd.TIMING)
    p.step(steps)
    t = p.pass_times()
    per_step = {"y": 1, "z": 15, "xab": 7, "x": 1, "yba": 7}
    saved = {"y": 15, "z": 15, "x": 15, "xab": 0, "yba": 0}
    for kind, count in per_step.items():
        assert t[kind][0] == count * steps - saved[kind], (kind, t[kind])

