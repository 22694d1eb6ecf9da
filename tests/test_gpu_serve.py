"""Serving loop and batching form on the GPU: every result is the same
alone (its own plan) and in the mix, and matches the CPU oracle; admission
respects the HBM budget."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from oracle import spectrum
from paper_1805_03155_amd import batching, serve, spstd
from paper_1805_03155_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def alone(r):
    p = spstd.plan_from_workload(r.work, precision=r.precision, dt=r.dt, nsteps_max=r.steps)
    ser, _ = p.run(r.steps)
    E, _ = spstd.spectrum(ser, r.dt, nlevels=r.nlevels)
    return ser, E


def check_alone(reqs):
    for r in reqs:
        assert r.status == "done", r.rid
        ser, E = alone(r)
        fp64 = r.precision == spstd.FP64
        # against the field's scale: a probe can sit where the state is tiny
        scale = np.abs(np.concatenate([r.work.psiR, r.work.psiI])).max()
        assert np.abs(r.series - ser).max() <= (1e-12 if fp64 else 1e-5) * scale, (r.rid, r.key)
        # a run shorter than a level period resolves no level: then neither does
        assert len(E) == len(r.E), (r.rid, r.E, E)
        assert np.allclose(r.E, E, rtol=1e-10 if fp64 else 1e-5), (r.rid, r.E, E)


def _oracle_request(r, coeffs, threads=1):
    oracle.set_threads(threads)
    w = r.work
    c, d = coeffs
    dt = oracle.stable_dt(c, d, w.V, w.n, w.dx, w.hbar, w.mass, fraction=w.cfl_fraction)
    _, _, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, c, d, dt, r.steps,
                             w.probes[:1], hbar=w.hbar, mass=w.mass)
    Eo, _ = spectrum.extract(so, dt, hbar=w.hbar, nlevels=r.nlevels)
    return dt, so, Eo


def check_oracle(reqs, coeffs=W.PAPER):
    """Each served request against the CPU oracle: the time step the server
    chose is 0.5 x_max / rho of the instance (Eq. 24-30 with V), the probe
    series follows Eq. (17)-(18) step by step, and the levels extracted from
    it match the oracle's extraction of the oracle's series.  The oracle
    runs of the requests go side by side on host threads (its calls release
    the interpreter lock), each with its share of the host's cores."""
    # 8 runs at a time on at most 16 host cores
    workers = 8
    threads = max(1, min(16, os.cpu_count() or 8) // workers)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        outs = list(ex.map(lambda r: _oracle_request(r, coeffs, threads), reqs))
    for r, (dt, so, Eo) in zip(reqs, outs):
        w = r.work
        assert r.dt == pytest.approx(dt, rel=1e-13), (r.rid, r.dt, dt)
        fp64 = r.precision == spstd.FP64
        scale = np.abs(np.concatenate([w.psiR, w.psiI])).max()
        assert r.series.shape == so.shape, (r.rid, r.series.shape, so.shape)
        err = np.abs(r.series - so).max() / scale
        assert err <= (1e-12 if fp64 else 1e-4), (r.rid, r.key, err)
        assert len(Eo) == len(r.E), (r.rid, r.E, Eo)
        assert np.allclose(r.E, Eo, rtol=1e-10 if fp64 else 1e-5, atol=0), (r.rid, r.E, Eo)


def test_served_results_equal_alone():
    reqs = serve.request_mix(14, rate=400.0, seed=3, steps=(300, 700),
                             sizes_1d=(1024, 2048, 8192), sizes_3d=((32, 1.0),), p1d=0.7)
    srv = serve.Server(hbm_budget=2 << 30, chunk=128, max_slots=6, max_steps=700)
    srv.run(reqs)
    assert srv.peak_used <= 2 << 30
    check_alone(reqs)
    check_oracle(reqs)
    lat = [r.latency for r in reqs]
    assert all(x > 0 for x in lat)
    # requests overlapped: more than one was admitted before the first finished
    first_done = min(r.done for r in reqs)
    assert sum(1 for r in reqs if r.admitted < first_done) > 1


def test_small_budget_queues_but_completes():
    reqs = serve.request_mix(5, rate=1000.0, seed=5, steps=(200, 300), sizes_1d=(2048,), p1d=1.0,
                             p_fp32=0.0)
    one = spstd.batch_workspace_size(spstd.make_batch_desc((2048,), W.PAPER, 1, 1, 300))
    srv = serve.Server(hbm_budget=one + 4096, chunk=64, max_slots=4, max_steps=300)
    srv.run(reqs)
    assert srv.peak_used <= one + 4096
    starts = sorted(r.admitted for r in reqs)
    dones = sorted(r.done for r in reqs)
    # one slot only: each request starts after the previous one finished
    assert all(s >= d for s, d in zip(starts[1:], dones[:-1]))
    check_alone(reqs)
    check_oracle(reqs)


def test_batching_form_instances_against_oracle():
    inst = W.batch_instances(count=24, seed=11, steps=200, max_1d_log2=11, max_2d_log2=7)
    res, stats = batching.run_instances(inst, 200, precision=spstd.FP64, group=True)
    assert stats["stage_updates_per_s"] > 0
    for i in (0, 5, 11, 17, 23):
        w = inst[i]
        ser, dt = res[i]
        assert dt == pytest.approx(oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx, w.hbar, w.mass,
                                                    fraction=w.cfl_fraction), rel=1e-13)
        _, _, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dt, 200, w.probes)
        scale = np.abs(np.concatenate([w.psiR, w.psiI])).max()
        assert np.abs(ser - so).max() <= 1e-12 * scale
        assert rel(ser, so) <= 1e-11
