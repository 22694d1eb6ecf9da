"""Writes batch2d_levels.npz: FP64 oracle runs of ten 2D instances of the
batching workload (512 seeded instances, seed 0, paper coefficient set,
5000 steps, dt = 0.5 x each instance's stability limit): a square and a
harmonic well at each of 32^2, 64^2, 128^2, 256^2 and 512^2.  Kept per
instance: its index in the workload, dt, every 25th probe sample and the
lowest 4 levels extracted from the full series.  Calls only the oracle and
the input generators.  About 10 minutes on 8 cores:

    python tests/golden/make_batch2d_levels.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                                      # noqa: E402
from oracle import spectrum                        # noqa: E402
from paper_1805_03155_amd import workloads as W    # noqa: E402

COUNT, SEED, STEPS, EVERY, NLEVELS = 512, 0, 5000, 25, 4
SHAPES = (32, 64, 128, 256, 512)


def pick(inst):
    """The first square and the first harmonic well of each 2D shape."""
    out = []
    for n in SHAPES:
        for kind in ("square", "harmonic"):
            out.append(next(k for k, w in enumerate(inst)
                            if w.n == (n, n) and w.meta["kind"][0] == kind))
    return out


def main():
    inst = W.batch_instances(count=COUNT, seed=SEED, steps=STEPS)
    idx = pick(inst)
    dts, series, levels = [], [], []
    for k in idx:
        w = inst[k]
        c, d = w.coeffs
        dt = oracle.stable_dt(c, d, w.V, w.n, w.dx)
        _, _, ser, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, c, d, dt, STEPS, w.probes[:1])
        E, _ = spectrum.extract(ser, dt, 1.0, NLEVELS)
        E = np.concatenate([E, np.full(NLEVELS - len(E), np.nan)])
        dts.append(dt)
        series.append(ser[::EVERY])
        levels.append(E)
        print(f"instance {k} {w.n}: dt {dt:.6g}, levels {E}", flush=True)
    np.savez(os.path.join(HERE, "batch2d_levels.npz"),
             count=COUNT, seed=SEED, steps=STEPS, every=EVERY, index=np.array(idx),
             dt=np.array(dts), series=np.array(series), levels=np.array(levels))


if __name__ == "__main__":
    main()
