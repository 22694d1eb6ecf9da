"""The comparison methods of the paper on the GPU versus the oracle: the
three-point finite-difference operator (FDTD column of Tables 1-3) under
the symplectic stages and under RK4, and PSTD (one stage, c = d = 1).
"""
import numpy as np
import pytest

import oracle
from paper_1805_03155_amd import spstd
from paper_1805_03155_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def case(n, seed):
    rng = np.random.default_rng(seed)
    N = int(np.prod(n))
    dx = tuple(0.2 + 0.1 * k for k in range(len(n)))
    return W.Workload(f"fd{seed}", tuple(n), dx, (0.0,) * len(n), 2.0 * rng.random(N),
                      rng.standard_normal(N), rng.standard_normal(N),
                      rng.integers(0, N, 2).astype(np.int64), 0, W.PAPER)


@pytest.mark.parametrize("n", [(64,), (32, 16), (16, 16, 32), (4096,)])
@pytest.mark.parametrize("method", [spstd.SYMPLECTIC, spstd.RK4])
def test_fd3_run_matches_the_oracle(n, method):
    w = case(n, seed=len(n) + 7 * method)
    dt = 0.5 * oracle.xmax(*w.coeffs) / (0.5 * sum(4.0 / h ** 2 for h in w.dx) + w.V.max())
    steps = 100
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=steps, method=method, laplacian=spstd.LAP_FD3)
    ser, _ = p.run(steps)
    r, i, _ = p.get_state()
    ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dt, steps, w.probes,
                               laplacian=oracle.LAP_FD3, method=method)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12
    assert rel(ser, so) <= 1e-12
    q = spstd.plan_from_workload(w, dt=dt, nsteps_max=steps, method=method, laplacian=spstd.LAP_FD3,
                                 precision=spstd.FP32)
    q.run(steps)
    r, i, _ = q.get_state()
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 2e-5


def test_fd3_levels_are_the_difference_operator_spectrum():
    # the FDTD run oscillates at the eigenvalues of the three-point operator
    n, dx = 64, 0.25
    V = W.harmonic_1d_potential(n, 8.0)
    x = W.axis_coords(n, -8.0, 8.0)
    w = W.Workload("fdho", (n,), (dx,), (-8.0,), V, np.exp(-(x - 0.3) ** 2), np.zeros(n),
                   np.array([n // 2 + 3], np.int64), 40000, W.PAPER)
    Kfd = (np.diag(np.full(n, 1.0 / dx ** 2)) - 0.5 / dx ** 2 * (
        np.roll(np.eye(n), 1, 0) + np.roll(np.eye(n), -1, 0))) + np.diag(V)
    lam = np.linalg.eigvalsh(Kfd)
    p = spstd.plan_from_workload(w, nsteps_max=w.steps, laplacian=spstd.LAP_FD3)
    ser, st = p.run(w.steps)
    E, _ = spstd.spectrum(ser, st.dt, nlevels=3)
    assert len(E) == 3
    for k, e in enumerate(E):            # off-centre start: every level
        assert abs(e / lam[k] - 1.0) < 1e-6


def test_fd3_plans_reject_energy():
    w = case((32,), seed=1)
    p = spstd.plan_from_workload(w, nsteps_max=1, laplacian=spstd.LAP_FD3)
    with pytest.raises(spstd.SpstdError) as ei:
        p.energy()
    assert ei.value.code == 1
