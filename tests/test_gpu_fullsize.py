"""The bench workload at its full size: the 256^3 oscillator with the
Yoshida-6 set, in the launch configurations bench.py times.

Element by element against the oracle over 2 steps (the oracle needs about
10-20 s per 2 steps at this size); over 40 steps against the oracle's run
stored by tests/golden/make_harmonic256_y6.py (every probe sample, the state
at 4096 seeded points), in graph replay, in the timed eager mode and split
over two calls, which place the merged step boundaries and the 16-step chunk
edges differently; graph replay against eager launches over 32 steps; and
properties that hold at any length (norm and energy) over 200 steps.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1805_03155_amd import spstd
from paper_1805_03155_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.fixture(scope="module")
def bench_case():
    w = W.harmonic_3d(seed=0, n=256, half_box=12.0, omega=1.0, steps=2, coeffs=W.YOSHIDA6, nprobes=3)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dt, 2, w.probes)
    return w, dt, (ro, io, so)


@pytest.mark.parametrize("flags", [0, spstd.TIMING])
def test_two_steps_match_the_oracle(bench_case, flags):
    w, dt, (ro, io, so) = bench_case
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=2, flags=flags)
    ser, _ = p.run(2)
    r, i, _ = p.get_state()
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12
    assert rel(ser, so) <= 1e-12
    q = spstd.plan_from_workload(w, dt=dt, nsteps_max=2, precision=spstd.FP32, flags=flags)
    q.run(2)
    r, i, _ = q.get_state()
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 2e-5


GOLD40 = os.path.join(os.path.dirname(__file__), "golden", "harmonic256_y6.npz")


@pytest.mark.parametrize("mode", ["graph", "timed", "split"])
def test_forty_steps_match_the_stored_oracle_run(mode):
    g = np.load(GOLD40, allow_pickle=False)
    steps = int(g["steps"])
    w = W.harmonic_3d(seed=int(g["seed"]), n=int(g["n"]), half_box=float(g["half_box"]), omega=1.0,
                      steps=steps, coeffs=W.YOSHIDA6, nprobes=3)
    assert np.array_equal(w.probes, g["probes"])
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    assert dt == float(g["dt"])
    flags = spstd.TIMING if mode == "timed" else 0
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=steps, flags=flags)
    if mode == "split":
        p.run(17)
    ser, st = p.run(steps - 17 if mode == "split" else steps)
    r, i, done = p.get_state()
    assert done == steps
    pts = g["points"]
    assert rel(np.concatenate([r[pts], i[pts]]), np.concatenate([g["psiR"], g["psiI"]])) <= 1e-12
    assert rel(ser, g["series"]) <= 1e-12
    assert abs(st.norm / (float(g["norm_final"]) * np.prod(w.dx)) - 1.0) <= 1e-12
    if mode == "graph":
        q = spstd.plan_from_workload(w, dt=dt, nsteps_max=steps, precision=spstd.FP32)
        ser32, _ = q.run(steps)
        r, i, _ = q.get_state()
        assert rel(np.concatenate([r[pts], i[pts]]), np.concatenate([g["psiR"], g["psiI"]])) <= 5e-5
        assert rel(ser32, g["series"]) <= 5e-5


def test_graph_replay_equals_timed_eager_launches(bench_case):
    w, dt, _ = bench_case
    out = []
    for flags in (0, spstd.TIMING):
        p = spstd.plan_from_workload(w, dt=dt, nsteps_max=32, flags=flags)
        ser, _ = p.run(32)
        out.append((p.get_state()[:2], ser))
        del p
    (a, sa), (b, sb) = out
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(sa, sb)


def test_norm_and_energy_hold_over_200_steps(bench_case):
    w, dt, _ = bench_case
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=200)
    k0, v0, n0 = p.energy()
    _, st = p.run(200)
    k1, v1, n1 = p.energy()
    assert abs(st.norm / st.norm0 - 1.0) < 1e-13
    assert abs(n1 / n0 - 1.0) < 1e-13
    assert abs(((k1 + v1) / n1) / ((k0 + v0) / n0) - 1.0) < 1e-12
