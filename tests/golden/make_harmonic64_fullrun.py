"""Writes harmonic64_fullrun.npz: the oracle's full run of the 64^3
oscillator workload (seed 7, [-8, 8)^3, paper coefficient set, dt = 0.5 x
the stability limit, 10000 steps, 3 probes), kept as: every probe sample,
the final state at 32768 seeded grid points (one in eight), the norm at
start and end and the lowest 8 extracted levels.  Calls only the oracle and
the input generators.  About 8 minutes on 8 cores:

    python tests/golden/make_harmonic64_fullrun.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                                      # noqa: E402
from oracle import spectrum                        # noqa: E402
from paper_1805_03155_amd import workloads as W    # noqa: E402

SEED, N, STEPS, NPOINTS = 7, 64, 10000, 32768


def main():
    w = W.harmonic_3d(seed=SEED, n=N, steps=STEPS)
    c, d = w.coeffs
    dt = oracle.stable_dt(c, d, w.V, w.n, w.dx)
    r, i, ser, norm = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, c, d, dt, STEPS, w.probes,
                                 want_norm=True)
    E, _ = spectrum.extract(ser, dt, 1.0, 8)
    pts = np.sort(np.random.default_rng(12345).choice(w.npoints, NPOINTS, replace=False))
    np.savez(os.path.join(HERE, "harmonic64_fullrun.npz"),
             seed=SEED, n=N, steps=STEPS, dt=dt, probes=w.probes, series=ser,
             points=pts, psiR=r[pts], psiI=i[pts],
             max_abs_psi=np.abs(np.concatenate([r, i])).max(),
             norm_initial=norm[0], norm_final=norm[-1], levels=E)


if __name__ == "__main__":
    main()
