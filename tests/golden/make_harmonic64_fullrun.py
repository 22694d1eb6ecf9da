"""Writes harmonic64_fullrun.json: the oracle's full run of the 64^3
oscillator workload (seed 7, [-8, 8)^3, paper coefficient set, dt = 0.5 x
the stability limit, 10000 steps, 3 probes), kept as sampled outputs:
every 50th probe sample, the final state at 512 seeded grid points, the
final norm and the lowest 8 extracted levels.  Calls only the oracle and the
input generators.  About 8 minutes on 8 cores:

    python tests/golden/make_harmonic64_fullrun.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                                      # noqa: E402
from oracle import spectrum                        # noqa: E402
from paper_1805_03155_amd import workloads as W    # noqa: E402

SEED, N, STEPS, SAMPLE_EVERY, NPOINTS = 7, 64, 10000, 50, 512


def main():
    w = W.harmonic_3d(seed=SEED, n=N, steps=STEPS)
    c, d = w.coeffs
    dt = oracle.stable_dt(c, d, w.V, w.n, w.dx)
    r, i, ser, norm = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, c, d, dt, STEPS, w.probes,
                                 want_norm=True)
    E, A = spectrum.extract(ser, dt, 1.0, 8)
    pts = np.random.default_rng(12345).choice(w.npoints, NPOINTS, replace=False)
    out = {
        "_what": "oracle full run of the 64^3 oscillator (seed 7, paper set, dt = 0.5 x limit, "
                 "10000 steps); written by make_harmonic64_fullrun.py",
        "seed": SEED, "n": N, "steps": STEPS, "dt": dt,
        "probes": [int(p) for p in w.probes],
        "sample_every": SAMPLE_EVERY,
        "series": ser[::SAMPLE_EVERY].tolist(),
        "points": [int(p) for p in pts],
        "psiR": r[pts].tolist(), "psiI": i[pts].tolist(),
        "max_abs_psi": float(np.abs(np.concatenate([r, i])).max()),
        "norm_final": float(norm[-1]), "norm_initial": float(norm[0]),
        "levels": [float(e) for e in E],
    }
    with open(os.path.join(HERE, "harmonic64_fullrun.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
