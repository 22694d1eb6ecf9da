"""SPSTD oracle -- TEST INFRASTRUCTURE, not part of the product.

A plain, slow, double-precision CPU implementation of the symplectic
pseudospectral time-domain scheme of Shen, Sha, Kuang, Hu, Huang and Wu
(arXiv:1805.03155).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the GPU engine (``paper_1805_03155_amd``) and neither imports the other.

The arithmetic lives in ``spstd_oracle.c`` (its own FFT, the K operator, the
stage-by-stage update, RK4 and finite-difference comparison runs, the
stability edge) plus two NumPy modules: ``spectrum.py`` (eigenvalues from a
probe time series) and ``modal.py`` (the exact discrete solution from a dense
eigendecomposition, used to pin the stepper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spstd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

NYQ_FULL = 0
NYQ_ZERO = 1
LAP_SPECTRAL = 0
LAP_FD3 = 1
METHOD_SYMPLECTIC = 0
METHOD_RK4 = 1
BC_PERIODIC = 0
BC_DIRICHLET = 1
BC_NEUMANN = 2


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-std=c99", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i64, i = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        pd, pi64 = P(d), P(i64)
        L.or_dft_naive.argtypes = [i64, pd, pd, pd, pd, i]
        L.or_fft.argtypes = [i64, pd, pd, i]
        L.or_fft.restype = i
        pint = P(i)
        L.or_d2_axis.argtypes = [pi64, pd, i, i, pd, pd]
        L.or_d2_axis.restype = i
        L.or_d2_axis_bc.argtypes = [pi64, pd, i, i, i, pd, pd]
        L.or_d2_axis_bc.restype = i
        L.or_apply_K.argtypes = [pi64, pd, d, d, i, i, pint, pd, pd, pd]
        L.or_apply_K.restype = i
        L.or_mode_matrix.argtypes = [i, pd, pd, d, pd]
        L.or_xmax.argtypes = [i, pd, pd]
        L.or_xmax.restype = d
        L.or_rho_bound.argtypes = [pi64, pd, d, d, pd]
        L.or_rho_bound.restype = d
        L.or_run.argtypes = [pi64, pd, d, d, i, i, pint, i, pd, pd, pd, i, pd, pd, d,
                             i64, i, pi64, pd, pd]
        L.or_run.restype = i
        L.or_num_threads.restype = i
        L.or_set_threads.argtypes = [i]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _grid(n, dx):
    n3 = np.ones(3, dtype=np.int64)
    d3 = np.ones(3, dtype=np.float64)
    n3[: len(n)] = n
    d3[: len(dx)] = dx
    return n3, d3


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    """Threads of the calling host thread's later oracle runs."""
    lib().or_set_threads(int(n))


def dft_naive(x, sign=-1):
    """Discrete Fourier sum sum_j x_j exp(sign 2 pi i j k / n), by definition."""
    x = np.asarray(x, dtype=np.complex128)
    re, im = _f64(x.real), _f64(x.imag)
    ore, oim = np.empty_like(re), np.empty_like(im)
    lib().or_dft_naive(len(x), _dp(re), _dp(im), _dp(ore), _dp(oim), sign)
    return ore + 1j * oim


def fft(x, sign=-1):
    """The oracle's own radix-2 FFT (unnormalised)."""
    x = np.asarray(x, dtype=np.complex128)
    re, im = _f64(x.real).copy(), _f64(x.imag).copy()
    rc = lib().or_fft(len(x), _dp(re), _dp(im), sign)
    if rc:
        raise ValueError("length must be a power of two")
    return re + 1j * im


def _bc3(bc):
    """Boundary code per axis (None: periodic everywhere)."""
    if bc is None:
        return None
    b = np.zeros(3, dtype=np.int32)
    b[: len(bc)] = bc
    return b


def _bcp(b):
    return b.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if b is not None else None


def d2_axis(f, n, dx, axis, nyquist=NYQ_FULL, bc=BC_PERIODIC):
    """Spectral second derivative of a real field along one axis (Eq. 9-10;
    Sec. 2.2 for the walled axes, BC_DIRICHLET / BC_NEUMANN, whose samples
    sit at cell centres (j + 1/2) dx).

    ``f`` is a flat array in row-major [nz][ny][nx] order (x fastest)."""
    n3, d3 = _grid(n, dx)
    f = _f64(f).ravel()
    out = np.empty_like(f)
    rc = lib().or_d2_axis_bc(_ip(n3), _dp(d3), axis, bc, nyquist, _dp(f), _dp(out))
    if rc:
        raise ValueError("bad grid")
    return out


def apply_K(f, V, n, dx, hbar=1.0, mass=1.0, nyquist=NYQ_FULL,
            laplacian=LAP_SPECTRAL, bc=None):
    """K f = -(hbar/2m*) Laplacian f + (V/hbar) f   (Eq. 16)."""
    n3, d3 = _grid(n, dx)
    f = _f64(f).ravel()
    V = None if V is None else _f64(V).ravel()
    out = np.empty_like(f)
    b = _bc3(bc)
    rc = lib().or_apply_K(_ip(n3), _dp(d3), hbar, mass, nyquist, laplacian, _bcp(b),
                          _dp(V), _dp(f), _dp(out))
    if rc:
        raise ValueError("bad grid")
    return out


def energy(psiR, psiI, V, n, dx, hbar=1.0, mass=1.0, nyquist=NYQ_FULL, bc=None):
    """Energy diagnostics of psi = psiR + i psiI as plain sums over the grid
    (Sec. 2.2, Eq. 16, times hbar), each times the cell volume:
    kinetic = sum psi* (-(hbar^2/2m*) Laplacian) psi, potential =
    sum V |psi|^2, norm = sum |psi|^2.  <H> = (kinetic + potential) / norm.
    The Laplacian is the oracle's own K with V = 0."""
    _, d3 = _grid(n, dx)
    cell = float(np.prod(d3[: len(n)]))
    r, i = _f64(psiR).ravel(), _f64(psiI).ravel()
    kr = apply_K(r, None, n, dx, hbar, mass, nyquist, bc=bc)
    ki = apply_K(i, None, n, dx, hbar, mass, nyquist, bc=bc)
    kin = hbar * float(np.dot(r, kr) + np.dot(i, ki)) * cell
    rho = r * r + i * i
    pot = float(np.dot(_f64(V).ravel(), rho)) * cell
    return kin, pot, float(rho.sum()) * cell


def mode_matrix(c, d, x):
    """One step's 2x2 evolution matrix for a mode with omega*dt = x (Eq. 23)."""
    c, d = _f64(c), _f64(d)
    M = np.empty(4)
    lib().or_mode_matrix(len(c), _dp(c), _dp(d), float(x), _dp(M))
    return M.reshape(2, 2)


def xmax(c, d):
    """First x = omega*dt at which |tr M(x)| exceeds 2 (Eq. 24-25)."""
    c, d = _f64(c), _f64(d)
    return lib().or_xmax(len(c), _dp(c), _dp(d))


def rho_bound(V, n, dx, hbar=1.0, mass=1.0):
    """(hbar/2m*) sum_d (pi/dx_d)^2 + max|V|/hbar: a bound of the spectrum of K."""
    n3, d3 = _grid(n, dx)
    V = None if V is None else _f64(V).ravel()
    return lib().or_rho_bound(_ip(n3), _dp(d3), hbar, mass, _dp(V))


def stable_dt(c, d, V, n, dx, hbar=1.0, mass=1.0, fraction=0.5):
    """dt = fraction * x_max / rho  (the per-mode bound of Eq. 24-30 with V)."""
    return fraction * xmax(c, d) / rho_bound(V, n, dx, hbar, mass)


def run(psiR, psiI, V, n, dx, c, d, dt, nsteps, probes=(), hbar=1.0, mass=1.0,
        nyquist=NYQ_FULL, laplacian=LAP_SPECTRAL, method=METHOD_SYMPLECTIC,
        want_norm=False, bc=None):
    """Advance (psiR, psiI) by ``nsteps`` steps.

    Returns (psiR, psiI, probe_series[(nsteps+1), nprobes, 2], norm or None).
    """
    n3, d3 = _grid(n, dx)
    pr, pi_ = _f64(psiR).ravel().copy(), _f64(psiI).ravel().copy()
    V = None if V is None else _f64(V).ravel()
    c, d = _f64(c), _f64(d)
    pidx = np.ascontiguousarray(np.asarray(probes, dtype=np.int64).ravel())
    npr = len(pidx)
    series = np.zeros((nsteps + 1, npr, 2)) if npr else None
    norm = np.zeros(nsteps + 1) if want_norm else None
    b = _bc3(bc)
    rc = lib().or_run(_ip(n3), _dp(d3), hbar, mass, nyquist, laplacian, _bcp(b), method,
                      _dp(V), _dp(pr), _dp(pi_), len(c), _dp(c), _dp(d), float(dt),
                      int(nsteps), npr, _ip(pidx) if npr else None,
                      _dp(series), _dp(norm))
    if rc:
        raise RuntimeError(f"oracle run failed ({rc})")
    return pr, pi_, series, norm
