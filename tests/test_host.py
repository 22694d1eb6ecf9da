"""Host-side logic on the CPU: the seeded input generators of the batching
and serving workloads, the serving loop's latency summary, and the
descriptor builders of the binding.  No device is touched."""
import numpy as np

from paper_1805_03155_amd import serve, spstd
from paper_1805_03155_amd import workloads as W


def test_request_mix_is_seeded_and_follows_its_recipe():
    a = serve.request_mix(300, rate=20.0, seed=5)
    b = serve.request_mix(300, rate=20.0, seed=5)
    assert [(r.key, r.steps, r.arrival) for r in a] == [(r.key, r.steps, r.arrival) for r in b]
    assert np.array_equal(a[17].work.psiR, b[17].work.psiR)
    arrivals = np.array([r.arrival for r in a])
    assert np.all(np.diff(arrivals) > 0)
    # Poisson arrivals at 20/s: mean gap 0.05 s (300 gaps, a loose bound)
    assert abs(np.diff(arrivals).mean() / 0.05 - 1.0) < 0.2
    shapes = [r.work.n for r in a]
    one_d = [s for s in shapes if len(s) == 1]
    three_d = [s for s in shapes if len(s) == 3]
    assert len(one_d) + len(three_d) == len(shapes)
    assert 0.7 < len(one_d) / len(shapes) < 0.9
    assert {s[0] for s in one_d} <= {1024, 2048, 4096, 8192, 16384}
    assert {s for s in three_d} <= {(32, 32, 32), (64, 64, 64), (128, 128, 128)}
    assert all(2000 <= r.steps <= 20000 for r in a)
    assert {r.precision for r in a} == {spstd.FP32, spstd.FP64}
    for r in a[:40]:
        w = r.work
        N = int(np.prod(w.n))
        assert w.V.shape == w.psiR.shape == w.psiI.shape == (N,)
        assert 0 <= int(w.probes[0]) < N
        assert np.all(np.isfinite(w.V)) and np.abs(w.psiR).max() > 0


def test_batch_instances_follow_their_recipe():
    inst = W.batch_instances(count=64, seed=3, steps=10, max_1d_log2=10, max_2d_log2=7)
    assert len(inst) == 64
    for w in inst:
        N = int(np.prod(w.n))
        assert len(w.n) in (1, 2)
        assert all(n & (n - 1) == 0 for n in w.n)
        if len(w.n) == 2:
            assert w.n[0] == w.n[1] and 32 <= w.n[0] <= 128
        else:
            assert 128 <= w.n[0] <= 1024
        assert w.V.shape == w.psiR.shape == (N,)
        assert np.all(w.psiI == 0.0)
        assert 0 <= int(w.probes[0]) < N
        assert abs(w.dx[0] * w.n[0] - 40.0) < 1e-12
    again = W.batch_instances(count=64, seed=3, steps=10, max_1d_log2=10, max_2d_log2=7)
    assert all(np.array_equal(x.V, y.V) and np.array_equal(x.psiR, y.psiR) for x, y in zip(inst, again))


def test_latency_summary_percentiles():
    class R:
        def __init__(self, lat):
            self.latency = lat
    reqs = [R(float(k)) for k in range(1, 101)] + [R(None)]
    s = serve.latency_summary(reqs, elapsed=50.0, stage_updates=1e9)
    assert s["requests"] == 100
    assert s["p50_s"] == np.percentile(np.arange(1, 101), 50)
    assert s["p99_s"] == np.percentile(np.arange(1, 101), 99)
    assert s["completed_per_s"] == 2.0 and s["stage_updates_per_s"] == 2e7
    empty = serve.latency_summary([R(None)], elapsed=1.0, stage_updates=0.0)
    assert empty["requests"] == 0 and empty["p50_s"] is None


def test_descriptor_builders():
    d = spstd.make_desc((64, 32), (0.1, 0.2), *W.YOSHIDA6, probes=(3, 5), bc=(1, 0),
                        flags=spstd.NO_MERGE | spstd.EAGER)
    assert d.ndim == 2 and tuple(d.n) == (64, 32, 1)
    assert d.m == len(W.YOSHIDA6[0]) and d.nprobes == 2
    assert tuple(d.bc) == (1, 0, 0) and d.flags == spstd.NO_MERGE | spstd.EAGER
    assert [d.c[k] for k in range(d.m)] == list(W.YOSHIDA6[0])
    b = spstd.make_batch_desc((32, 32), W.PAPER, 7, nprobes=1, nsteps_max=100, wpb=4,
                              flags=spstd.AUTOTUNE)
    assert b.capacity == 7 and b.waves_per_block == 4 and b.flags == spstd.AUTOTUNE
    assert tuple(b.n) == (32, 32, 1) and b.nsteps_max == 100
