"""GPU path versus the CPU oracle, element by element, through the C ABI.

FP64 bar: relative L2 of (psi_R, psi_I) <= 1e-12 after the run, eigenvalues
<= 1e-10 relative.  Both sides receive the same seeded arrays and the same
dt (the oracle's).
"""
import numpy as np
import pytest

import oracle
from oracle import modal, spectrum
from paper_1805_03155_amd import spstd
from paper_1805_03155_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def gpu_run(w, dt, steps, precision=spstd.FP64, method=spstd.SYMPLECTIC,
            nyquist=spstd.NYQ_FULL, coeffs=None, flags=0):
    p = spstd.plan_from_workload(w, precision=precision, method=method, dt=dt,
                                 nsteps_max=steps, nyquist=nyquist, coeffs=coeffs, flags=flags)
    series, st = p.run(steps)
    r, i, _ = p.get_state()
    return r, i, series, st


def oracle_run(w, dt, steps, method=oracle.METHOD_SYMPLECTIC, nyquist=oracle.NYQ_FULL,
               coeffs=None):
    c, d = coeffs if coeffs is not None else w.coeffs
    r, i, series, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, c, d, dt, steps, w.probes,
                                 nyquist=nyquist, method=method)
    return r, i, series


def case(n, seed, steps=20, coeffs=W.PAPER, vscale=2.0):
    """Random smooth-ish field and potential on a small grid (ragged aspect)."""
    rng = np.random.default_rng(seed)
    N = int(np.prod(n))
    dx = tuple(0.2 + 0.1 * k for k in range(len(n)))
    V = vscale * rng.random(N)
    psiR = rng.standard_normal(N)
    psiI = rng.standard_normal(N)
    probes = rng.integers(0, N, 3)
    return W.Workload(f"rand_{n}", tuple(n), dx, (0.0,) * len(n), V, psiR, psiI,
                      np.asarray(probes, np.int64), steps, coeffs)


def test_finite_well_1d_full_run():
    w = W.finite_well_1d(seed=0)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    r, i, ser, st = gpu_run(w, dt, w.steps)
    ro, io, sero = oracle_run(w, dt, w.steps)
    assert st.steps_done == w.steps
    e = rel(np.concatenate([r, i]), np.concatenate([ro, io]))
    print("1D psi rel-L2", e)
    assert e <= 1e-12
    assert rel(ser, sero) <= 1e-12
    E, _ = spstd.spectrum(ser, dt, nlevels=4)
    Eo, _ = spectrum.extract(sero, dt, nlevels=4)
    print("1D levels", E, "rel", (E - Eo) / Eo)
    assert len(E) == 4
    assert np.abs((E - Eo) / Eo).max() <= 1e-10


@pytest.mark.parametrize("n", [(16,), (32,), (64,), (128,), (512,), (1024,), (2048,),
                               (4096,), (8192,), (16384,)])
def test_1d_lengths(n):
    w = case(n, seed=n[0], steps=10)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    r, i, ser, _ = gpu_run(w, dt, w.steps)
    ro, io, sero = oracle_run(w, dt, w.steps)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12
    assert rel(ser, sero) <= 1e-12


@pytest.mark.parametrize("n", [(16, 16), (64, 32), (32, 128), (256, 16), (16, 512),
                               (128, 1024), (512, 32), (1024, 16), (32, 64)])
def test_2d_shapes(n):
    w = case(n, seed=sum(n), steps=8)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    r, i, _, _ = gpu_run(w, dt, w.steps)
    ro, io, _ = oracle_run(w, dt, w.steps)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12


@pytest.mark.parametrize("n", [(16, 16, 16), (32, 16, 64), (64, 32, 16), (16, 128, 32),
                               (256, 16, 16), (16, 16, 256)])
def test_3d_shapes(n):
    w = case(n, seed=sum(n), steps=5)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    r, i, _, _ = gpu_run(w, dt, w.steps)
    ro, io, _ = oracle_run(w, dt, w.steps)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12


@pytest.mark.parametrize("name", ["leapfrog", "forest_ruth", "yoshida6"])
def test_other_coefficient_sets(name):
    # Forest-Ruth and Yoshida-6 end on a stage with d = 0 (single-half x pass)
    w = case((32, 16, 16), seed=5, steps=6, coeffs=W.COEFFS[name])
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    r, i, _, _ = gpu_run(w, dt, w.steps)
    ro, io, _ = oracle_run(w, dt, w.steps)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12


def test_zero_nyquist_convention():
    w = case((64, 32), seed=9, steps=10)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    r, i, _, _ = gpu_run(w, dt, w.steps, nyquist=spstd.NYQ_ZERO)
    ro, io, _ = oracle_run(w, dt, w.steps, nyquist=oracle.NYQ_ZERO)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12


def test_rk4_comparison_run():
    w = case((32, 32, 16), seed=3, steps=6)
    dt = 0.5 * 2.8284271247461903 / oracle.rho_bound(w.V, w.n, w.dx)
    r, i, _, _ = gpu_run(w, dt, w.steps, method=spstd.RK4)
    ro, io, _ = oracle_run(w, dt, w.steps, method=oracle.METHOD_RK4)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12


def test_harmonic_64_short_run_and_full_levels():
    w = W.harmonic_3d(seed=7, n=64)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    r, i, ser, _ = gpu_run(w, dt, 100)
    ro, io, sero = oracle_run(w, dt, 100)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12
    assert rel(ser, sero) <= 1e-12
    # full 10000-step run: levels against (n + 3/2) hbar omega (Sec. 3.3)
    _, _, ser, _ = gpu_run(w, dt, w.steps)
    E, _ = spstd.spectrum(ser, dt, nlevels=5)
    print("64^3 levels", E)
    exact = np.arange(5) + 1.5
    # per-level bound of the windowed extraction on this record length
    assert np.abs((E - exact) / exact).max() <= 5e-6


def test_fp32_against_fp64_oracle():
    w = W.finite_well_1d(seed=0)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    r, i, ser, _ = gpu_run(w, dt, w.steps, precision=spstd.FP32)
    ro, io, sero = oracle_run(w, dt, w.steps)
    e = rel(np.concatenate([r, i]), np.concatenate([ro, io]))
    E, _ = spstd.spectrum(ser, dt, nlevels=4)
    Eo, _ = spectrum.extract(sero, dt, nlevels=4)
    print("fp32 psi rel", e, "E rel", (E - Eo) / Eo)
    assert e < 1e-3
    assert np.abs((E - Eo) / Eo).max() <= 1e-5


def test_graph_replay_equals_eager():
    w = case((64, 16, 32), seed=21, steps=40)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    a = gpu_run(w, dt, w.steps)
    b = gpu_run(w, dt, w.steps, flags=spstd.EAGER)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


def test_checkpoint_resume_bitwise_and_deterministic():
    w = case((32, 32, 32), seed=4, steps=40)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    full = gpu_run(w, dt, 40)
    again = gpu_run(w, dt, 40)
    assert np.array_equal(full[0], again[0]) and np.array_equal(full[1], again[1])
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=40)
    p.run(17)
    r, i, s = p.get_state()
    q = spstd.plan_from_workload(w, dt=dt, nsteps_max=40)
    q.set_state(r, i, s)
    ser, _ = q.run(23)
    r2, i2, _ = q.get_state()
    assert np.array_equal(r2, full[0]) and np.array_equal(i2, full[1])
    assert np.array_equal(ser[s:], full[2][s:])


def test_error_paths():
    w = W.finite_well_1d(seed=0)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    with pytest.raises(spstd.SpstdError) as ei:
        spstd.plan_from_workload(w, dt=2.05 * dt)          # beyond the edge
    assert ei.value.code == 2
    p = spstd.plan_from_workload(w, dt=2.05 * dt, flags=spstd.ALLOW_UNSTABLE, nsteps_max=3000)
    with pytest.raises(spstd.SpstdError) as ei:
        p.run(3000)
    assert ei.value.code == 5                               # blew up: non-finite
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=10)
    with pytest.raises(spstd.SpstdError) as ei:
        p.run(11)
    assert ei.value.code == 6


@pytest.mark.parametrize("n", [(64,), (32, 16), (16, 32, 16)])
@pytest.mark.parametrize("flags", [0, spstd.NO_RESIDENT | spstd.EAGER])
def test_degenerate_runs(n, flags):
    # zero steps: the initial sample only and the state untouched
    w = case(n, seed=3)
    N = int(np.prod(n))
    w.probes = np.array([0, N - 1], np.int64)           # first and last grid point
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=5, flags=flags)
    ser, _ = p.run(0)
    assert ser.shape == (1, 2, 2)
    assert np.array_equal(ser[0, :, 0], w.psiR[[0, N - 1]]) and np.array_equal(ser[0, :, 1], w.psiI[[0, N - 1]])
    r, i, step = p.get_state()
    assert step == 0 and np.array_equal(r, w.psiR) and np.array_equal(i, w.psiI)
    # probes at the ends of the grid follow the oracle over a few steps
    ser, _ = p.run(5)
    ro, io, so = oracle_run(w, dt, 5)
    assert rel(ser, so) <= 1e-12
    # no probes: the run still advances the state
    w0 = case(n, seed=3)
    w0.probes = np.zeros(0, np.int64)
    q = spstd.plan_from_workload(w0, dt=dt, nsteps_max=5, flags=flags)
    q.run(5)
    r, i, step = q.get_state()
    assert step == 5
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12
    # the zero state stays exactly zero; a zero potential with psi_I absent
    w0.psiR = np.zeros(N)
    w0.psiI = np.zeros(N)
    z = spstd.plan_from_workload(w0, dt=dt, nsteps_max=5, flags=flags)
    z.run(5)
    r, i, _ = z.get_state()
    assert not r.any() and not i.any()
    wv = case(n, seed=4)
    wv.V = np.zeros(N)
    desc = spstd.make_desc(wv.n, wv.dx, *wv.coeffs, dt=dt, probes=wv.probes, flags=flags)
    pv = spstd.Plan(desc, wv.V, wv.psiR, None, nsteps_max=5)
    pv.run(5)
    r, i, _ = pv.get_state()
    ro, io, _, _ = oracle.run(wv.psiR, np.zeros(N), wv.V, wv.n, wv.dx, *wv.coeffs, dt, 5, wv.probes)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12


@pytest.mark.parametrize("n", [(16, 16), (64, 32), (32, 64), (64, 64)])
@pytest.mark.parametrize("prec", [spstd.FP64, spstd.FP32])
def test_small_2d_plans_resident_vs_passes(n, prec):
    # small periodic 2D plans run the LDS-resident kernel; the pass kernels
    # give the same run, and a resumed run continues bitwise
    steps = 30
    w = case(n, seed=sum(n) + 7, steps=steps)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    a = gpu_run(w, dt, steps, precision=prec)
    b = gpu_run(w, dt, steps, precision=prec, flags=spstd.NO_RESIDENT)
    tol = 1e-13 if prec == spstd.FP64 else 2e-5
    assert rel(np.concatenate(a[:2]), np.concatenate(b[:2])) < tol
    assert rel(a[2], b[2]) < tol
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=steps, precision=prec)
    p.run(11)
    r, i, s = p.get_state()
    q = spstd.plan_from_workload(w, dt=dt, nsteps_max=steps, precision=prec)
    q.set_state(r, i, s)
    ser, _ = q.run(steps - 11)
    r2, i2, _ = q.get_state()
    assert np.array_equal(r2, a[0]) and np.array_equal(i2, a[1])
    assert np.array_equal(ser[s:], a[2][s:])


@pytest.mark.parametrize("name", ["forest_ruth", "yoshida6", "paper", "leapfrog"])
@pytest.mark.parametrize("n", [(32, 16, 64), (64, 32), (256,)])
@pytest.mark.parametrize("prec", [spstd.FP64, spstd.FP32])
def test_merged_step_boundaries(name, n, prec):
    # sets whose last stage has no B half run the A half ending a step and
    # the one opening the next as one (coefficient c_m + c_1); the boundary
    # probe samples are interpolated.  Sets whose last stage has a B half
    # (paper, leapfrog) chain instead: the step's last y pass runs fused with
    # the next step's first, the samples taken around that sweep.  40 steps:
    # two graph chunks of 16 and 8 eager steps; eager launches merge or
    # chain the same boundaries
    steps = 40
    w = case(n, seed=len(n) * 11 + 5, steps=steps, coeffs=W.COEFFS[name])
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    base = spstd.NO_RESIDENT if len(n) == 1 else 0
    g = gpu_run(w, dt, steps, precision=prec, flags=base)
    ea = gpu_run(w, dt, steps, precision=prec, flags=base | spstd.EAGER)
    assert np.array_equal(g[0], ea[0]) and np.array_equal(g[1], ea[1]) and np.array_equal(g[2], ea[2])
    ro, io, so = oracle_run(w, dt, steps)
    tol = 1e-12 if prec == spstd.FP64 else 2e-5
    assert rel(np.concatenate(g[:2]), np.concatenate([ro, io])) <= tol
    assert rel(g[2], so) <= tol
    # split over two calls (other boundaries merged): the same run
    p = spstd.plan_from_workload(w, precision=prec, dt=dt, nsteps_max=steps, flags=base)
    p.run(13)
    ser, _ = p.run(steps - 13)
    r, i, _ = p.get_state()
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= tol
    assert rel(ser, so) <= tol
    # without merging, a split run equals the unsplit one bitwise
    nm = base | spstd.NO_MERGE
    u = gpu_run(w, dt, steps, precision=prec, flags=nm)
    assert rel(np.concatenate(u[:2]), np.concatenate([ro, io])) <= tol
    q = spstd.plan_from_workload(w, precision=prec, dt=dt, nsteps_max=steps, flags=nm)
    q.run(13)
    ser, _ = q.run(steps - 13)
    r, i, _ = q.get_state()
    assert np.array_equal(r, u[0]) and np.array_equal(i, u[1]) and np.array_equal(ser, u[2])
