"""Resident 1D kernel and batches of instances, through the C ABI.

Each instance is checked alone (a single plan) against the same instance
inside a batch, and against the CPU oracle.  The tolerance for "same alone
and in the mix" is rounding-level: within a batch two instances can share a
complex pencil, which changes the rounding but not the arithmetic.
"""
import numpy as np
import pytest

import oracle
from paper_1805_03155_amd import spstd
from paper_1805_03155_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def inst(n, seed, nprobes=1):
    rng = np.random.default_rng(seed)
    N = int(np.prod(n))
    dx = tuple(0.15 + 0.05 * rng.random() for _ in n)
    V = (1.0 + 3.0 * rng.random()) * rng.random(N)
    return W.Workload(f"inst{seed}", tuple(n), dx, (0.0,) * len(n), V, rng.standard_normal(N),
                      rng.standard_normal(N), rng.integers(0, N, nprobes).astype(np.int64), 0, W.PAPER)


def resident_ok(n):
    """Shapes a batch can run with a resident kernel."""
    if len(n) == 1:
        return 16 <= n[0] <= 16384
    if len(n) == 2:
        return n[0] in (16, 32, 64) and n[1] in (16, 32, 64)
    return len(n) == 3 and all(k == 16 for k in n)


def alone(w, dt, steps, precision=spstd.FP64, flags=0):
    p = spstd.plan_from_workload(w, dt=dt, nsteps_max=steps, precision=precision, flags=flags)
    ser, _ = p.run(steps)
    r, i, _ = p.get_state()
    return r, i, ser


@pytest.mark.parametrize("n", [16, 32, 256, 512, 1024, 4096, 8192, 16384])
@pytest.mark.parametrize("prec", [spstd.FP64, spstd.FP32])
def test_resident_kernel_matches_pass_kernels(n, prec):
    w = inst((n,), seed=n)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    a = alone(w, dt, 50, prec)                              # resident (one launch)
    b = alone(w, dt, 50, prec, flags=spstd.NO_RESIDENT)     # pass kernels
    tol = 1e-13 if prec == spstd.FP64 else 2e-5
    assert rel(np.concatenate(a[:2]), np.concatenate(b[:2])) < tol
    assert rel(a[2], b[2]) < tol
    if prec == spstd.FP64:
        ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dt, 50, w.probes)
        assert rel(np.concatenate(a[:2]), np.concatenate([ro, io])) <= 1e-12
        assert rel(a[2], so) <= 1e-12


@pytest.mark.parametrize("shape,cap,slots", [((512,), 5, [0, 1, 3, 4]),          # resident
                                              ((8192,), 3, [0, 2]),              # pass kernels
                                              ((64, 32), 6, [0, 2, 3, 5]),
                                              ((32, 16, 16), 3, [0, 1, 2])])
def test_batch_instances_alone_vs_in_the_mix(shape, cap, slots):
    steps = 40
    b = spstd.Batch(shape, W.PAPER, capacity=cap, nprobes=2, nsteps_max=steps)
    ws = {s: inst(shape, seed=100 + s, nprobes=2) for s in slots}
    dts = {}
    for s, w in ws.items():
        dts[s] = 0.9 * oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
        assert b.load(s, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dts[s]) == dts[s]
    b.step(steps)
    for s, w in ws.items():
        ser, r, i, k = b.read(s)
        assert k == steps
        ra, ia, sa = alone(w, dts[s], steps)
        assert rel(np.concatenate([r, i]), np.concatenate([ra, ia])) < 1e-13
        assert rel(ser, sa) < 1e-13
        ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dts[s], steps, w.probes)
        assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12
        assert rel(ser, so) <= 1e-12
    # free slots stayed empty
    for s in set(range(cap)) - set(slots):
        assert b.slot_info(s)[0] is False


def test_batch_fp32_against_fp64_oracle():
    shape, steps = (256, 64), 60
    b = spstd.Batch(shape, W.PAPER, capacity=2, nprobes=1, nsteps_max=steps, precision=spstd.FP32)
    w = inst(shape, seed=7)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    b.load(1, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dt)
    b.step(steps)
    ser, r, i, _ = b.read(1)
    ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dt, steps, w.probes)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) < 2e-5


def test_batch_release_and_reload_slot():
    shape, steps = (1024,), 30
    b = spstd.Batch(shape, W.PAPER, capacity=2, nprobes=1, nsteps_max=2 * steps,
                    flags=spstd.NO_RESIDENT)
    w0, w1, w2 = inst(shape, 1), inst(shape, 2), inst(shape, 3)
    dt = lambda w: oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    b.load(0, w0.dx, w0.V, w0.psiR, w0.psiI, w0.probes, dt=dt(w0))
    b.load(1, w1.dx, w1.V, w1.psiR, w1.psiI, w1.probes, dt=dt(w1))
    b.step(steps)
    b.release(0)
    b.load(0, w2.dx, w2.V, w2.psiR, w2.psiI, w2.probes, dt=dt(w2))
    b.step(steps)
    ser2, r2, i2, k2 = b.read(0)
    ser1, r1, i1, k1 = b.read(1)
    assert (k2, k1) == (steps, 2 * steps)
    ra, ia, sa = alone(w2, dt(w2), steps)
    assert rel(np.concatenate([r2, i2]), np.concatenate([ra, ia])) < 1e-13
    rb, ib, sb = alone(w1, dt(w1), 2 * steps)
    assert rel(np.concatenate([r1, i1]), np.concatenate([rb, ib])) < 1e-13
    with pytest.raises(spstd.SpstdError) as ei:
        b.step(steps + 1)
    assert ei.value.code == 6
    with pytest.raises(spstd.SpstdError):
        b.load(1, w0.dx, w0.V, w0.psiR, w0.psiI, w0.probes)   # slot busy


@pytest.mark.parametrize("n,prec", [((512,), spstd.FP64), ((8192,), spstd.FP64), ((2048,), spstd.FP32),
                                    ((64, 32), spstd.FP64), ((32, 16, 16), spstd.FP32),
                                    ((64, 64, 64), spstd.FP64)])
def test_autotuned_batch_starts_empty_and_matches_alone(n, prec):
    steps = 40
    b = spstd.Batch(n, W.PAPER, capacity=3, nprobes=2, nsteps_max=steps, precision=prec,
                    flags=spstd.AUTOTUNE)
    sched, wpb, us = b.schedule()
    # resident candidate only where a resident kernel applies; passes always
    # timed at both block sizes (equal where rows longer than 1024 points
    # make the size moot)
    assert (us[0] > 0) == resident_ok(n) and us[1] > 0 and us[2] > 0
    if len(n) == 1 and n[0] > 1024:
        assert us[1] == us[2]
    assert wpb == (4 if us[2] < us[1] else 2)
    assert sched == ("resident" if resident_ok(n) and us[0] <= us[1 if wpb == 2 else 2] else "passes")
    # the same key again: the remembered choice, no new timing
    b2 = spstd.Batch(n, W.PAPER, capacity=3, nprobes=2, nsteps_max=steps, precision=prec,
                     flags=spstd.AUTOTUNE)
    assert b2.schedule() == (sched, wpb, us)
    for s in range(3):
        assert b.slot_info(s)[0] is False
    ws = {s: inst(n, seed=300 + s, nprobes=2) for s in (0, 2)}
    dts = {}
    for s, w in ws.items():
        dts[s] = 0.9 * oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
        b.load(s, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dts[s])
    b.step(steps)
    tol = 1e-13 if prec == spstd.FP64 else 2e-5
    for s, w in ws.items():
        ser, r, i, k = b.read(s)
        assert k == steps
        ra, ia, sa = alone(w, dts[s], steps, prec)
        assert rel(np.concatenate([r, i]), np.concatenate([ra, ia])) < tol
        assert rel(ser, sa) < tol


@pytest.mark.parametrize("wpb", [2, 4])
def test_forced_block_sizes_match_the_oracle(wpb):
    # both block sizes give the oracle's result (the autotuner may pick either)
    n = (32, 16, 64)
    w = inst(n, seed=77)
    dt = oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    b = spstd.Batch(n, W.PAPER, capacity=2, nprobes=1, nsteps_max=20, wpb=wpb)
    assert b.schedule()[1] == wpb
    b.load(1, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dt)
    b.step(20)
    ser, r, i, _ = b.read(1)
    ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dt, 20, w.probes)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12
    assert rel(ser, so) <= 1e-12


@pytest.mark.parametrize("n", [(16, 16), (32, 64), (64, 16), (64, 64)])
@pytest.mark.parametrize("prec", [spstd.FP64, spstd.FP32])
def test_resident_2d_matches_pass_kernels_and_oracle(n, prec):
    # small 2D instances held in one workgroup's LDS against the pass-kernel
    # schedule of the same batch, and (FP64) against the oracle
    steps = 30
    ws = [inst(n, seed=700 + k, nprobes=2) for k in range(3)]
    res = spstd.Batch(n, W.PAPER, capacity=3, nprobes=2, nsteps_max=steps, precision=prec)
    split = spstd.Batch(n, W.PAPER, capacity=3, nprobes=2, nsteps_max=steps, precision=prec)
    pas = spstd.Batch(n, W.PAPER, capacity=3, nprobes=2, nsteps_max=steps, precision=prec,
                      flags=spstd.NO_RESIDENT)
    assert res.schedule()[0] == "resident" and pas.schedule()[0] == "passes"
    dts = []
    for k, w in enumerate(ws):
        dt = 0.9 * oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
        dts.append(dt)
        for b in (res, split, pas):
            b.load(k, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dt)
    res.step(steps)
    split.step(11)
    split.step(steps - 11)
    pas.step(steps)
    tol = 1e-13 if prec == spstd.FP64 else 2e-5
    for k, w in enumerate(ws):
        s1, r1, i1, c1 = res.read(k)
        s2, r2, i2, c2 = pas.read(k)
        s3, r3, i3, c3 = split.read(k)
        assert c1 == c2 == c3 == steps
        # one launch or two: the same arithmetic
        assert np.array_equal(r1, r3) and np.array_equal(i1, i3) and np.array_equal(s1, s3)
        assert rel(np.concatenate([r1, i1]), np.concatenate([r2, i2])) < tol
        assert rel(s1, s2) < tol
        if prec == spstd.FP64:
            ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dts[k], steps, w.probes)
            assert rel(np.concatenate([r1, i1]), np.concatenate([ro, io])) <= 1e-12
            assert rel(s1, so) <= 1e-12


# ------------------------------------------------------------- mixed groups
GROUP_SHAPES = ((128, 128), (256, 256), (512, 512), (128, 256))


def _group_members(prec, steps, count=(3, 2, 1, 2), flags=0):
    """Batches of the group shapes filled with seeded instances."""
    out = []
    for shape, k in zip(GROUP_SHAPES, count):
        b = spstd.Batch(shape, W.PAPER, capacity=k + 1, nprobes=1, nsteps_max=steps, precision=prec,
                        flags=flags)
        ws = [inst(shape, seed=1000 * shape[0] + shape[1] + j) for j in range(k)]
        out.append((b, ws))
    return out


def _load(members):
    dts = []
    for b, ws in members:
        dts.append([b.load(s, w.dx, w.V, w.psiR, w.psiI, w.probes) for s, w in enumerate(ws)])
    return dts


@pytest.mark.parametrize("prec", [spstd.FP64, spstd.FP32])
def test_group_schedules_match_the_oracle(prec):
    # every candidate schedule of a group (mixed-shape kernels under each
    # block size / exchange / pencils-per-lane-group variant, and the
    # members' own kernels) steps each instance as the oracle does; one
    # slot of each member stays free (its zero scales make it a no-op)
    steps = 40
    ncand = 17 if prec == spstd.FP32 else 9
    ref = None
    for choice in range(ncand):
        members = _group_members(prec, steps)
        g = spstd.BatchGroup([b for b, _ in members])
        assert len(g.schedule()[1]) == ncand
        g.set_schedule(choice)
        dts = _load(members)
        g.step(steps)
        got = []
        for (b, ws), dd in zip(members, dts):
            for s, w in enumerate(ws):
                ser, r, i, done = b.read(s)
                assert done == steps
                got.append((w, dd[s], ser, r, i))
        if ref is None:
            ref = []
            for w, dt, _, _, _ in got:
                ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dt, steps, w.probes)
                ref.append((ro, io, so))
        tol = 1e-12 if prec == spstd.FP64 else 2e-5
        for (w, dt, ser, r, i), (ro, io, so) in zip(got, ref):
            assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= tol, (choice, w.n)
            assert rel(ser, so) <= tol, (choice, w.n)
        g.close()


def test_group_autotune_and_alone_versus_mix():
    # FP32 group with the tuner: it times every candidate and keeps the
    # fastest; each instance then equals its own single-shape batch run
    steps = 50
    members = _group_members(spstd.FP32, steps + 2)
    g = spstd.BatchGroup([b for b, _ in members], flags=spstd.AUTOTUNE)
    choice, us = g.schedule()
    assert len(us) == 17 and all(u > 0 for u in us)
    assert us[choice] <= 1.03 * min(us)
    dts = _load(members)
    g.step(steps)
    for (b, ws), dd in zip(members, dts):
        for s, w in enumerate(ws):
            ser, r, i, _ = b.read(s)
            ra, ia, sa = alone(w, dd[s], steps, spstd.FP32)
            assert rel(np.concatenate([r, i]), np.concatenate([ra, ia])) <= 1e-5
            assert rel(ser, sa) <= 1e-5
    g.close()
    # after the group, the members step on their own again
    b, ws = members[0]
    b.step(2)
    assert b.slot_info(0)[1] == steps + 2


def test_group_rejects_unfit_members_and_overflow():
    b1 = spstd.Batch((1024,), W.PAPER, capacity=2, nsteps_max=4)
    b2 = spstd.Batch((128, 128), W.PAPER, capacity=2, nsteps_max=4)
    b3 = spstd.Batch((256, 256), W.PAPER, capacity=2, nsteps_max=4, precision=spstd.FP32)
    for bad in ([b1], [b2, b3], [b2, b2]):
        with pytest.raises(spstd.SpstdError):
            spstd.BatchGroup(bad)
    w = inst((128, 128), seed=3)
    g = spstd.BatchGroup([b2])
    b2.load(0, w.dx, w.V, w.psiR, w.psiI, w.probes)
    g.step(4)
    with pytest.raises(spstd.SpstdError) as ei:
        g.step(1)
    assert ei.value.code == 6


@pytest.mark.parametrize("prec", [spstd.FP64, spstd.FP32])
def test_resident_3d_matches_pass_kernels_and_oracle(prec):
    # small 3D instances stepped by one workgroup each (fields in their own
    # arrays) against the pass-kernel schedule of the same batch, and (FP64)
    # against the oracle; a run split over two calls is the same arithmetic
    n, steps = (16, 16, 16), 30
    ws = [inst(n, seed=900 + k, nprobes=2) for k in range(3)]
    res = spstd.Batch(n, W.PAPER, capacity=3, nprobes=2, nsteps_max=steps, precision=prec)
    split = spstd.Batch(n, W.PAPER, capacity=3, nprobes=2, nsteps_max=steps, precision=prec)
    pas = spstd.Batch(n, W.PAPER, capacity=3, nprobes=2, nsteps_max=steps, precision=prec,
                      flags=spstd.NO_RESIDENT)
    assert res.schedule()[0] == "resident" and pas.schedule()[0] == "passes"
    dts = []
    for k, w in enumerate(ws):
        dt = 0.9 * oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
        dts.append(dt)
        for b in (res, split, pas):
            b.load(k, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dt)
    res.release(1)              # a free slot between active ones
    split.release(1)
    pas.release(1)
    res.step(steps)
    split.step(7)
    split.step(steps - 7)
    pas.step(steps)
    tol = 1e-13 if prec == spstd.FP64 else 2e-5
    for k in (0, 2):
        w = ws[k]
        s1, r1, i1, c1 = res.read(k)
        s2, r2, i2, c2 = pas.read(k)
        s3, r3, i3, c3 = split.read(k)
        assert c1 == c2 == c3 == steps
        assert np.array_equal(r1, r3) and np.array_equal(i1, i3) and np.array_equal(s1, s3)
        assert rel(np.concatenate([r1, i1]), np.concatenate([r2, i2])) < tol
        assert rel(s1, s2) < tol
        if prec == spstd.FP64:
            ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dts[k], steps, w.probes)
            assert rel(np.concatenate([r1, i1]), np.concatenate([ro, io])) <= 1e-12
            assert rel(s1, so) <= 1e-12
    assert res.slot_info(1)[0] is False


@pytest.mark.parametrize("n", [(32, 32, 32), (64, 16, 32), (16, 64, 64), (32, 128, 16), (64, 32, 64),
                               (16, 32, 16)])
@pytest.mark.parametrize("prec", [spstd.FP64, spstd.FP32])
@pytest.mark.parametrize("name", ["paper", "yoshida6"])
def test_fused_planes_match_separate_passes_and_oracle(n, prec, name):
    # 3D batches with x and z of 16 to 64 points run z(A), x(A+B), z(B) of a
    # stage as one launch per x-z plane (square planes transform the x rows
    # and z columns of a half together); the same batch with separate passes
    # (SPSTD_NO_PLANES) and the oracle agree.  Yoshida-6's last stage has no
    # B half (a plane launch with the A part alone).  40 steps: two graph
    # chunks and 8 eager steps; a free slot between active ones stays zero.
    steps = 40
    coeffs = W.COEFFS[name]
    ws = []
    for k in range(3):
        w = inst(n, seed=1300 + k, nprobes=2)
        w.coeffs = coeffs
        ws.append(w)
    fused = spstd.Batch(n, coeffs, capacity=3, nprobes=2, nsteps_max=steps, precision=prec)
    sep = spstd.Batch(n, coeffs, capacity=3, nprobes=2, nsteps_max=steps, precision=prec, flags=spstd.NO_PLANES)
    dts = []
    for k, w in enumerate(ws):
        dt = 0.9 * oracle.stable_dt(*coeffs, w.V, w.n, w.dx)
        dts.append(dt)
        if k == 1:
            continue
        for b in (fused, sep):
            b.load(k, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dt)
    fused.step(steps)
    sep.step(steps)
    tol = 1e-13 if prec == spstd.FP64 else 2e-5
    for k in (0, 2):
        w = ws[k]
        s1, r1, i1, c1 = fused.read(k)
        s2, r2, i2, c2 = sep.read(k)
        assert c1 == c2 == steps
        assert rel(np.concatenate([r1, i1]), np.concatenate([r2, i2])) < tol
        assert rel(s1, s2) < tol
        if prec == spstd.FP64:
            ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *coeffs, dts[k], steps, w.probes)
            assert rel(np.concatenate([r1, i1]), np.concatenate([ro, io])) <= 1e-12
            assert rel(s1, so) <= 1e-12
    assert fused.slot_info(1)[0] is False


@pytest.mark.parametrize("n", [8192, 16384])
@pytest.mark.parametrize("prec", [spstd.FP64, spstd.FP32])
@pytest.mark.parametrize("name", ["paper", "yoshida6"])
def test_fourstep_rows_match_one_workgroup_rows_and_oracle(n, prec, name):
    # 1D batches of 8192- and 16384-point rows run each x pass as four-step
    # launches (128 columns) over many workgroups; the same batch with one
    # workgroup per row pair (SPSTD_NO_FOURSTEP) and the oracle agree.  Five
    # slots (the last pencil holds one row), slot 1 free between active
    # ones; 40 steps (two graph chunks and 8 eager steps); Yoshida-6 runs the
    # single A half of its last stage (merged step boundaries) and the paper
    # set chains its boundaries.
    steps = 40
    coeffs = W.COEFFS[name]
    ws = []
    for k in range(5):
        w = inst((n,), seed=2100 + k, nprobes=2)
        w.coeffs = coeffs
        ws.append(w)
    four = spstd.Batch((n,), coeffs, capacity=5, nprobes=2, nsteps_max=steps, precision=prec,
                       flags=spstd.NO_RESIDENT)
    one = spstd.Batch((n,), coeffs, capacity=5, nprobes=2, nsteps_max=steps, precision=prec,
                      flags=spstd.NO_RESIDENT | spstd.NO_FOURSTEP)
    dts = []
    for k, w in enumerate(ws):
        dt = 0.9 * oracle.stable_dt(*coeffs, w.V, w.n, w.dx)
        dts.append(dt)
        if k == 1:
            continue
        for b in (four, one):
            b.load(k, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dt)
    four.step(steps)
    one.step(steps)
    tol = 1e-13 if prec == spstd.FP64 else 2e-5
    for k in (0, 2, 3, 4):
        w = ws[k]
        s1, r1, i1, c1 = four.read(k)
        s2, r2, i2, c2 = one.read(k)
        assert c1 == c2 == steps
        assert rel(np.concatenate([r1, i1]), np.concatenate([r2, i2])) < tol, k
        assert rel(s1, s2) < tol, k
        if prec == spstd.FP64 or k == 4:
            ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *coeffs, dts[k], steps, w.probes)
            ot = 1e-12 if prec == spstd.FP64 else 2e-5
            assert rel(np.concatenate([r1, i1]), np.concatenate([ro, io])) <= ot, k
            assert rel(s1, so) <= ot, k
    assert four.slot_info(1)[0] is False


@pytest.mark.parametrize("n,flags", [((32, 16, 64), 0), ((32, 16, 64), spstd.NO_PLANES), ((16, 16, 16), 0),
                                     ((32, 32, 32), 0),
                                     ((64, 32), 0), ((64, 32), spstd.NO_RESIDENT), ((1024,), 0),
                                     ((1024,), spstd.NO_RESIDENT), ((16384,), spstd.NO_RESIDENT)])
def test_zero_nyquist_batches_against_oracle(n, flags):
    # the ZERO convention (the Nyquist bin removed) in every batch schedule:
    # fused x-z planes and separate passes (3D), the resident kernels and the
    # pass kernels (16^3, 2D and 1D)
    steps = 20
    w = inst(n, seed=1500 + len(n), nprobes=2)
    b = spstd.Batch(n, W.PAPER, capacity=2, nprobes=2, nsteps_max=steps, nyquist=spstd.NYQ_ZERO, flags=flags)
    dt = 0.9 * oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    b.load(1, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dt)
    b.step(steps)
    ser, r, i, k = b.read(1)
    assert k == steps
    ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dt, steps, w.probes,
                               nyquist=oracle.NYQ_ZERO)
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12
    assert rel(ser, so) <= 1e-12


@pytest.mark.parametrize("n", [(64, 32), (32, 16, 32), (32, 16, 128)])
@pytest.mark.parametrize("prec", [spstd.FP64, spstd.FP32])
def test_chained_boundaries_over_uneven_calls(n, prec):
    # the paper set's step boundaries chain inside every call (graph chunks
    # of 16 and eager remainders); calls of 1, 5, 16, 17 and 3 steps give
    # the oracle's run and its probe series, every sample in place
    sizes = (1, 5, 16, 17, 3)
    steps = sum(sizes)
    w = inst(n, seed=1700 + len(n), nprobes=3)
    b = spstd.Batch(n, W.PAPER, capacity=2, nprobes=3, nsteps_max=steps, precision=prec,
                    flags=spstd.NO_RESIDENT)
    dt = 0.9 * oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx)
    b.load(0, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dt)
    for k in sizes:
        b.step(k)
    ser, r, i, done = b.read(0)
    assert done == steps and ser.shape == (steps + 1, 3, 2)
    ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dt, steps, w.probes)
    tol = 1e-12 if prec == spstd.FP64 else 2e-5
    assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= tol
    assert rel(ser, so) <= tol
    # every sample individually (a sample written in two halves, one half
    # missing, would show as a zero or stale entry)
    scale = np.abs(so).max()
    assert np.abs(ser - so).max() <= (1e-11 if prec == spstd.FP64 else 1e-4) * scale


@pytest.mark.parametrize("choice", ["built-in", "members"])
def test_group_chained_over_uneven_calls(choice):
    # a group steps its members with chained step boundaries inside each
    # call; calls of 1, 5, 16, 17 and 3 steps match the oracle (FP64)
    sizes = (1, 5, 16, 17, 3)
    steps = sum(sizes)
    members = _group_members(spstd.FP64, steps)
    g = spstd.BatchGroup([b for b, _ in members])
    if choice == "members":
        g.set_schedule(len(g.schedule()[1]) - 1)
    dts = _load(members)
    for k in sizes:
        g.step(k)
    for (b, ws), dd in zip(members, dts):
        for s, w in enumerate(ws):
            ser, r, i, done = b.read(s)
            assert done == steps
            ro, io, so, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, *w.coeffs, dd[s], steps, w.probes)
            assert rel(np.concatenate([r, i]), np.concatenate([ro, io])) <= 1e-12, w.n
            assert rel(ser, so) <= 1e-12, w.n
    g.close()


@pytest.mark.parametrize("n,flags", [((64, 32), spstd.NO_RESIDENT), ((32, 16, 32), 0), ((32, 16, 32), spstd.NO_PLANES),
                                     ((16, 16, 16), 0), ((32, 32), 0), ((256, 128), 0)])
@pytest.mark.parametrize("prec", [spstd.FP64, spstd.FP32])
def test_batch_invariance_is_bitwise(n, flags, prec):
    # the 2D and 3D kernels touch one instance's data per pencil and row
    # (pencil pairs never straddle two slots), so an instance run alone in
    # its batch and the same instance among others give identical bits
    steps = 20
    ws = [inst(n, seed=1900 + k, nprobes=2) for k in range(4)]
    dts = [0.9 * oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx) for w in ws]
    mix = spstd.Batch(n, W.PAPER, capacity=4, nprobes=2, nsteps_max=steps, precision=prec, flags=flags)
    one = spstd.Batch(n, W.PAPER, capacity=4, nprobes=2, nsteps_max=steps, precision=prec, flags=flags)
    for k, w in enumerate(ws):
        mix.load(k, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dts[k])
    w = ws[2]
    one.load(2, w.dx, w.V, w.psiR, w.psiI, w.probes, dt=dts[2])
    mix.step(steps)
    one.step(steps)
    a, b = mix.read(2), one.read(2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
