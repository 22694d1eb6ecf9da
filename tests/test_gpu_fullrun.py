"""Full-length runs against the oracle.

The 64^3 oscillator workload runs its whole 10000 steps on the GPU and is
compared with the oracle's full run, stored as sampled outputs by
tests/golden/make_harmonic64_fullrun.py (every 50th probe sample, the final
state at 512 seeded points, the final norm, the lowest 8 levels).  Bars:
psi and probe samples <= 1e-12 relative L2, eigenvalues <= 1e-10 relative.

The FP32 form is checked where it counts, on eigenvalues: 1D instances of
the batching workload run FP32 in one batch and their levels are compared
with the FP64 oracle's (<= 1e-5 relative).
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import spectrum
from paper_1805_03155_amd import spstd
from paper_1805_03155_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "harmonic64_fullrun.json")


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def test_harmonic_64_full_run_against_the_oracle():
    g = json.load(open(GOLD))
    w = W.harmonic_3d(seed=g["seed"], n=g["n"], steps=g["steps"])
    assert [int(p) for p in w.probes] == g["probes"]
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    assert dt == g["dt"]
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=w.steps)
    ser, st = p.run(w.steps)
    r, i, _ = p.get_state()
    pts = np.array(g["points"])
    assert rel(np.concatenate([r[pts], i[pts]]), np.concatenate([g["psiR"], g["psiI"]])) <= 1e-12
    assert rel(ser[:: g["sample_every"]], np.array(g["series"])) <= 1e-12
    assert abs(st.norm / (g["norm_final"] * np.prod(w.dx)) - 1.0) <= 1e-12
    E, _ = spstd.spectrum(ser, dt, nlevels=8)
    assert len(E) == len(g["levels"])
    assert np.abs((E - np.array(g["levels"])) / np.array(g["levels"])).max() <= 1e-10


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
