"""Writes harmonic256_y6.npz: the oracle's run of the bench workload, the
256^3 oscillator on [-12, 12)^3 (seed 0, omega = 1, Yoshida sixth-order
set, dt = 0.5 x the stability limit, 3 probes), for 40 steps, kept as:
every probe sample, the state at 4096 seeded grid points after 40 steps, and
the norm at start and end.  40 steps span two 16-step chunks and a shorter
tail, with the step boundaries inside and between them.  Calls only the
oracle and the input generators.  About 4 minutes on 8 cores:

    python tests/golden/make_harmonic256_y6.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                                      # noqa: E402
from paper_1805_03155_amd import workloads as W    # noqa: E402

SEED, N, HALF_BOX, STEPS, NPOINTS = 0, 256, 12.0, 40, 4096


def main():
    w = W.harmonic_3d(seed=SEED, n=N, half_box=HALF_BOX, omega=1.0, steps=STEPS,
                      coeffs=W.YOSHIDA6, nprobes=3)
    c, d = w.coeffs
    dt = oracle.stable_dt(c, d, w.V, w.n, w.dx)
    r, i, ser, norm = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, c, d, dt, STEPS, w.probes,
                                 want_norm=True)
    pts = np.sort(np.random.default_rng(2024).choice(w.npoints, NPOINTS, replace=False))
    np.savez(os.path.join(HERE, "harmonic256_y6.npz"),
             seed=SEED, n=N, half_box=HALF_BOX, steps=STEPS, dt=dt, probes=w.probes,
             series=ser, points=pts, psiR=r[pts], psiI=i[pts],
             norm_initial=norm[0], norm_final=norm[-1])


if __name__ == "__main__":
    main()
