"""Full-length runs against the oracle.

The 64^3 oscillator workload runs its whole 10000 steps on the GPU and is
compared with the oracle's full run, stored by
tests/golden/make_harmonic64_fullrun.py (every probe sample, the final state
at 32768 seeded points, the norm, the lowest 8 levels).  Bars: psi and probe
samples <= 1e-12 relative L2, eigenvalues <= 1e-10 relative.

The FP32 form is checked where it counts, on eigenvalues against the FP64
oracle (<= 1e-5 relative): 1D instances of the batching workload in one
batch with the oracle run live, and the whole 512-instance batching
workload (5000 steps, as bench.py runs it) with the 2D instances of
32^2 .. 512^2 stored by tests/golden/make_batch2d_levels.py.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import spectrum
from paper_1805_03155_amd import batching, spstd
from paper_1805_03155_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "harmonic64_fullrun.npz")
GOLD2D = os.path.join(os.path.dirname(__file__), "golden", "batch2d_levels.npz")


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def test_harmonic_64_full_run_against_the_oracle():
    g = np.load(GOLD, allow_pickle=False)
    w = W.harmonic_3d(seed=int(g["seed"]), n=int(g["n"]), steps=int(g["steps"]))
    assert np.array_equal(w.probes, g["probes"])
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    assert dt == float(g["dt"])
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=w.steps)
    ser, st = p.run(w.steps)
    r, i, _ = p.get_state()
    pts = g["points"]
    assert len(pts) >= 32768
    assert rel(np.concatenate([r[pts], i[pts]]), np.concatenate([g["psiR"], g["psiI"]])) <= 1e-12
    assert rel(ser, g["series"]) <= 1e-12
    assert abs(st.norm / (float(g["norm_final"]) * np.prod(w.dx)) - 1.0) <= 1e-12
    E, _ = spstd.spectrum(ser, dt, nlevels=8)
    assert len(E) == len(g["levels"])
    assert np.abs((E - g["levels"]) / g["levels"]).max() <= 1e-10


def test_fp32_batch_eigenvalues_against_the_fp64_oracle():
    inst = [w for w in W.batch_instances(count=64, seed=3, steps=5000) if len(w.n) == 1 and w.n[0] <= 512][:6]
    assert len(inst) >= 4
    steps = 5000
    groups = {}
    for k, w in enumerate(inst):
        groups.setdefault(w.n, []).append(k)
    for shape, ks in groups.items():
        b = spstd.Batch(shape, W.PAPER, capacity=len(ks), nprobes=1, nsteps_max=steps,
                        precision=spstd.FP32, flags=spstd.AUTOTUNE)
        dts = [b.load(s, inst[k].dx, inst[k].V, inst[k].psiR, inst[k].psiI, inst[k].probes[:1])
               for s, k in enumerate(ks)]
        b.step(steps)
        for s, k in enumerate(ks):
            w = inst[k]
            ser, _, _, _ = b.read(s, state=False)
            _, _, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dts[s], steps, w.probes[:1])
            E32, _ = spstd.spectrum(ser, dts[s], nlevels=4)
            E64, _ = spectrum.extract(so, dts[s], 1.0, 4)
            assert len(E64) >= 2 and len(E32) >= 2
            # each of the oracle's two lowest levels, against the nearest FP32 level
            for e in E64[:2]:
                assert np.abs(E32 - e).min() <= 1e-5 * abs(e)


def test_fp32_batching_workload_2d_eigenvalues_against_the_fp64_oracle():
    g = np.load(GOLD2D, allow_pickle=False)
    steps, every = int(g["steps"]), int(g["every"])
    inst = W.batch_instances(count=int(g["count"]), seed=int(g["seed"]), steps=steps)
    res, _ = batching.run_instances(inst, steps, precision=spstd.FP32, group=True)
    shapes = set()
    for k, dt64, ser64, E64 in zip(g["index"], g["dt"], g["series"], g["levels"]):
        w = inst[int(k)]
        ser, dt = res[int(k)]
        shapes.add(w.n)
        assert dt == pytest.approx(float(dt64), rel=1e-13)
        # the FP32 probe series follows the FP64 oracle's to single precision
        scale = np.abs(np.concatenate([w.psiR, w.psiI])).max()
        assert np.abs(ser[::every] - ser64).max() <= 1e-4 * scale, (k, w.n)
        E32, _ = spstd.spectrum(ser, dt, nlevels=4)
        E64 = E64[np.isfinite(E64)]
        assert len(E64) >= 2 and len(E32) == len(E64), (k, w.n, E32, E64)
        assert np.abs((E32 - E64) / E64).max() <= 1e-5, (k, w.n, E32, E64)
    assert {(128, 128), (512, 512)} <= shapes
