"""The no-allocation entry point against the workspace one.

spstd_run_noalloc advances fields the caller holds on the device, with its
working memory in the library's fixed device scratch; its state and probe
series must equal those of spstd_plan + spstd_run on the same inputs, on
two calls in a row (the second on a smaller grid, so that what the first
left in the scratch must not leak into it)."""
import numpy as np
import pytest

from paper_1805_03155_amd import spstd
from paper_1805_03155_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(w, precision, steps, flags=0):
    import torch
    c, d = w.coeffs
    dt = spstd.stable_dt(spstd.make_desc(w.n, w.dx, c, d), w.V)
    # the workspace path (graph replay where it applies)
    p = spstd.plan_from_workload(w, precision=precision, dt=dt, nsteps_max=steps, flags=flags)
    ser, _ = p.run(steps)
    r, i, _ = p.get_state()
    del p
    # the no-allocation path on tensors of the run precision
    tdt = torch.float64 if precision == spstd.FP64 else torch.float32
    dev = torch.device("cuda")
    V = torch.tensor(w.V, dtype=tdt, device=dev)
    pr = torch.tensor(w.psiR, dtype=tdt, device=dev)
    pi = torch.tensor(w.psiI, dtype=tdt, device=dev)
    probes = torch.full((steps + 1, len(w.probes), 2), float("nan"), dtype=torch.float64, device=dev)
    desc = spstd.make_desc(w.n, w.dx, c, d, dt=dt, precision=precision, probes=w.probes, flags=flags)
    spstd.run_noalloc(desc, V, pr, pi, steps, probes)
    torch.cuda.synchronize()
    r2, i2 = pr.double().cpu().numpy(), pi.double().cpu().numpy()
    ser2 = probes.cpu().numpy()
    return (r, i, ser), (r2, i2, ser2)


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("precision", [spstd.FP64, spstd.FP32])
def test_noalloc_equals_the_workspace_entry_point_on_two_calls(precision):
    tol = 1e-12 if precision == spstd.FP64 else 1e-5
    # first call: 3D oscillator with the sixth-order set (merged step boundaries)
    big = W.harmonic_3d(seed=4, n=32, half_box=8.0, steps=40, coeffs=W.YOSHIDA6)
    # second call, smaller: a 1D finite well (the resident kernel path)
    small = W.finite_well_1d(seed=2, n=256, steps=300)
    for w, steps in ((big, 40), (small, 300)):
        (r, i, ser), (r2, i2, ser2) = _case(w, precision, steps)
        assert np.all(np.isfinite(ser2))
        assert _rel(np.concatenate([r2, i2]), np.concatenate([r, i])) <= tol, (w.name, precision)
        assert _rel(ser2, ser) <= tol, (w.name, precision)


def test_noalloc_rejects_an_implicit_dt_and_runs_the_longest_row():
    import torch
    n = (16384,)
    c, d = W.PAPER
    t = torch.zeros(16384, dtype=torch.float64, device="cuda")
    # an implicit dt (V would have to be read on the host) is an argument error
    desc = spstd.make_desc(n, (0.1,), c, d, dt=0.0)
    with pytest.raises(spstd.SpstdError) as ei:
        spstd.run_noalloc(desc, t, t.clone(), t.clone(), 1)
    assert ei.value.code == 1
    # the longest row (16384 points, the largest twiddle table) fits the scratch
    desc = spstd.make_desc(n, (0.1,), c, d, dt=1e-4)
    spstd.run_noalloc(desc, t, t.clone(), t.clone(), 2)
