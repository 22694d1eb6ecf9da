"""C ABI checks that need no GPU: the library loads, exports every symbol
include/spstd.h declares, and its host-only entry points (stability edge,
time step, workspace size, spectrum) agree with the oracle."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from oracle import spectrum
from paper_1805_03155_amd import spstd
from paper_1805_03155_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "spstd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spstd_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", spstd.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = spstd.lib()
    for n in names:
        assert hasattr(L, n)
    assert set(spstd.EXPORTS) == set(names)


@pytest.mark.parametrize("name", sorted(W.COEFFS))
def test_xmax_matches_oracle(name):
    c, d = W.COEFFS[name]
    assert spstd.xmax(c, d) == pytest.approx(oracle.xmax(c, d), rel=1e-13)


def test_stable_dt_matches_oracle():
    for w in (W.finite_well_1d(), W.harmonic_3d(n=32, half_box=8.0)):
        desc = spstd.make_desc(w.n, w.dx, *w.coeffs, probes=w.probes)
        assert spstd.stable_dt(desc, w.V) == pytest.approx(
            oracle.stable_dt(*w.coeffs, w.V, w.n, w.dx), rel=1e-13)


def test_stable_dt_of_the_difference_operator():
    # rho of the three-point operator: (hbar/2m*) sum 4/dx^2 + max|V|/hbar
    n, dx = (64, 32), (0.25, 0.4)
    V = np.linspace(0.0, 3.0, 64 * 32)
    desc = spstd.make_desc(n, dx, *W.PAPER, laplacian=spstd.LAP_FD3)
    rho = 0.5 * (4 / 0.25 ** 2 + 4 / 0.4 ** 2) + 3.0
    assert abs(spstd.stable_dt(desc, V) / (0.5 * oracle.xmax(*W.PAPER) / rho) - 1) < 1e-13
    bad = spstd.make_desc(n, dx, *W.PAPER, laplacian=spstd.LAP_FD3, bc=(1, 0))
    with pytest.raises(spstd.SpstdError):
        spstd.workspace_size(bad, 10)


def test_workspace_size_grows_with_probe_capacity_and_precision():
    w = W.harmonic_3d(n=32, half_box=8.0)
    d64 = spstd.make_desc(w.n, w.dx, *w.coeffs, probes=w.probes)
    d32 = spstd.make_desc(w.n, w.dx, *w.coeffs, probes=w.probes, precision=spstd.FP32)
    a, b = spstd.workspace_size(d64, 10), spstd.workspace_size(d64, 10000)
    assert b - a >= 9990 * 3 * 2 * 8 - 256      # 256-byte alignment of the buffer
    assert spstd.workspace_size(d32, 10) < a
    assert a >= 3 * 32 ** 3 * 8
    # twiddle tables are FP64 (16 B per entry) in both precisions
    for prec, esz in ((spstd.FP64, 8), (spstd.FP32, 4)):
        for n in ((16384,), (1024, 512), (64, 32, 1024)):
            d = spstd.make_desc(n, (0.1,) * len(n), *W.PAPER, precision=prec)
            assert spstd.workspace_size(d, 0) >= 3 * int(np.prod(n)) * esz + 16 * sum(n)


@pytest.mark.parametrize("bad", [dict(n=(24,), dx=(0.1,)), dict(n=(16, 2048), dx=(0.1, 0.1)),
                                 dict(n=(32,), dx=(-1.0,)), dict(n=(8,), dx=(0.1,)),
                                 dict(n=(32,), dx=(0.1,), probes=(40,)),
                                 # walled axes transform twice their length
                                 dict(n=(16384,), dx=(0.1,), bc=(1,)),
                                 dict(n=(16, 1024), dx=(0.1, 0.1), bc=(0, 2)),
                                 dict(n=(32,), dx=(0.1,), bc=(3,))])
def test_bad_descriptors_rejected(bad):
    desc = spstd.make_desc(bad["n"], bad["dx"], *W.PAPER, probes=bad.get("probes", ()),
                           bc=bad.get("bc"))
    with pytest.raises(spstd.SpstdError) as ei:
        spstd.workspace_size(desc, 10)
    assert ei.value.code == 1


@pytest.mark.parametrize("wpb,ok", [(0, True), (2, True), (4, True), (3, False), (8, False)])
def test_batch_block_size_is_validated(wpb, ok):
    d = spstd.make_batch_desc((32, 16), W.PAPER, 4, wpb=wpb)
    if ok:
        assert spstd.batch_workspace_size(d) > 4 * 3 * 32 * 16 * 8
    else:
        with pytest.raises(spstd.SpstdError) as ei:
            spstd.batch_workspace_size(d)
        assert ei.value.code == 1


def test_spectrum_matches_oracle_extraction():
    w = W.finite_well_1d(seed=2, steps=8000)
    c, d = w.coeffs
    dt = oracle.stable_dt(c, d, w.V, w.n, w.dx)
    _, _, ser, _ = oracle.run(w.psiR, w.psiI, w.V, w.n, w.dx, c, d, dt, w.steps, w.probes)
    E, A = spstd.spectrum(ser, dt, nlevels=5)
    Eo, Ao = spectrum.extract(ser, dt, nlevels=5)
    assert len(E) == len(Eo) == 5
    assert np.abs((E - Eo) / Eo).max() < 1e-12
    assert np.abs((A - Ao) / Ao).max() < 1e-9


def test_spectrum_of_pure_tones():
    # closed form: e^{-i w t} sampled every dt peaks exactly at w; with
    # several tones each one is biased only by the others' window sidelobes
    # (4-term Blackman-Harris: about 2.5e-5 in amplitude), i.e. a small
    # fraction of a bin 2 pi / (Ns dt)
    dt, ns = 0.01, 6001
    t = np.arange(ns) * dt
    for w0 in (0.7, 4.1, 9.75):
        z = np.exp(-1j * w0 * t)
        ser = np.stack([z.real, z.imag], -1)[:, None, :]
        E, A = spstd.spectrum(ser, dt, nlevels=1)
        assert abs(E[0] - w0) < 1e-10 * w0
        assert A[0] == pytest.approx(1.0, rel=1e-9)
    ws = np.array([1.3, 4.1, 9.75])
    z = sum(a * np.exp(-1j * w * t) for a, w in zip((1.0, 0.5, 0.25), ws))
    ser = np.stack([z.real, z.imag], -1)[:, None, :]
    E, _ = spstd.spectrum(ser, dt, nlevels=3)
    bin_w = 2 * np.pi / (ns * dt)
    assert np.abs(E - ws).max() < 1e-4 * bin_w
    with pytest.raises(spstd.SpstdError):
        spstd.spectrum(ser[:2], dt)
