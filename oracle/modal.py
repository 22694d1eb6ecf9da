"""Exact discrete solution of the scheme by modes -- oracle side (TEST INFRASTRUCTURE).

For a grid operator K with K phi_j = omega_j phi_j (real symmetric), one step
of the partitioned scheme acts on each mode's coefficient pair (a_j, b_j) of
(psi_R, psi_I) by the 2x2 matrix M(omega_j dt) of Eq. (23).  So

    psi^n = sum_j phi_j [M(omega_j dt)^n (a_j, b_j)].

This module builds that closed form with a dense symmetric eigendecomposition
(NumPy's ``eigh`` as a library step), independent of the oracle's FFT
stepper, and is used to pin it.

M(x) is carried as a matrix of polynomials in x (products of the stage
matrices of Eq. 23), so that tr M - 2 and M00 - M11, which vanish at x = 0,
are evaluated without cancellation; the phase theta with cos(theta) = tr M/2
and the power M^n = cos(n theta) I + sin(n theta) N, N = (M - cos(theta) I)
/ sin(theta), then keep full relative accuracy for slow modes.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import polynomial as P


def mode_poly(c, d):
    """Entries of M(x) as polynomial coefficient arrays (lowest degree first)."""
    one, zero = np.array([1.0]), np.array([0.0])
    a, b, e, f = one, zero, zero, one
    for cl, dl in zip(c, d):
        cx = np.array([0.0, cl])
        a, b = P.polyadd(a, P.polymul(cx, e)), P.polyadd(b, P.polymul(cx, f))
        dx = np.array([0.0, -dl])
        e, f = P.polyadd(e, P.polymul(dx, a)), P.polyadd(f, P.polymul(dx, b))
    return a, b, e, f


def trace_minus_two(c, d, x):
    a, b, e, f = mode_poly(c, d)
    t = P.polyadd(a, f)
    t[0] = 0.0                    # tr M(0) = 2 exactly
    return P.polyval(np.asarray(x, dtype=np.float64), t)


def theta(c, d, x):
    """Phase advance per step of a mode with omega*dt = x (stable range)."""
    q = -trace_minus_two(c, d, x) / 4.0          # sin^2(theta/2)
    return 2.0 * np.arcsin(np.sqrt(np.clip(q, 0.0, 1.0)))


def mode_power_apply(c, d, x, n, a0, b0):
    """(a_n, b_n) = M(x)^n (a0, b0), vectorised over modes x."""
    x = np.asarray(x, dtype=np.float64)
    A, B, E, F = mode_poly(c, d)
    m01, m10 = P.polyval(x, B), P.polyval(x, E)
    diff = P.polysub(A, F)
    diff[0] = 0.0
    half = 0.5 * P.polyval(x, diff)              # M00 - cos(theta)
    th = theta(c, d, x)
    s = np.sin(th)
    safe = np.where(s == 0.0, 1.0, s)
    n00, n01, n10 = half / safe, m01 / safe, m10 / safe
    cn, sn = np.cos(n * th), np.sin(n * th)
    a = cn * a0 + sn * (n00 * a0 + n01 * b0)
    b = cn * b0 + sn * (n10 * a0 - n00 * b0)
    zero = s == 0.0                              # x = 0: M is the identity
    a = np.where(zero, a0, a)
    b = np.where(zero, b0, b)
    return a, b


def kinetic_circulant(n, dx, hbar=1.0, mass=1.0, nyquist_zero=False):
    """Dense matrix of -(hbar/2m*) d^2/dx^2 on a periodic grid of n points,
    from the definition t[m] = (1/n) sum_k s_k cos(2 pi k m / n) with
    s_k = (hbar/2m*) K_k^2, K_k = 2 pi k / (n dx) (signed; |K| = pi/dx at
    the Nyquist bin, or 0 there under the ZERO convention)."""
    L = n * dx
    k = np.arange(n)
    ks = np.where(k <= n // 2, k, k - n).astype(np.float64)
    s = hbar / (2.0 * mass) * (2.0 * np.pi * ks / L) ** 2
    if nyquist_zero and n % 2 == 0:
        s[n // 2] = 0.0
    m = np.arange(n)
    t = np.array([np.sum(s * np.cos(2.0 * np.pi * k * mm / n)) / n for mm in m])
    idx = (m[:, None] - m[None, :]) % n
    return t[idx]


def hamiltonian_1d(V, dx, hbar=1.0, mass=1.0, nyquist_zero=False):
    """K = kinetic circulant + diag(V / hbar) on a 1D periodic grid."""
    V = np.asarray(V, dtype=np.float64)
    K = kinetic_circulant(len(V), dx, hbar, mass, nyquist_zero)
    return K + np.diag(V / hbar)


def evolve_1d(psiR, psiI, V, dx, c, d, dt, nsteps, hbar=1.0, mass=1.0,
              nyquist_zero=False):
    """psi after nsteps by the modal closed form (1D)."""
    K = hamiltonian_1d(V, dx, hbar, mass, nyquist_zero)
    w, phi = np.linalg.eigh(K)
    a0, b0 = phi.T @ psiR, phi.T @ psiI
    a, b = mode_power_apply(c, d, w * dt, nsteps, a0, b0)
    return phi @ a, phi @ b, w


def evolve_separable_3d(psiR, psiI, V1, dx, c, d, dt, nsteps, hbar=1.0,
                        mass=1.0, nyquist_zero=False):
    """Closed form for K = K_x + K_y + K_z with V(x,y,z) = V1(x)+V1(y)+V1(z)
    on an n^3 grid (fields row-major [z][y][x]).  Returns (psiR, psiI, omega_1d)."""
    n = len(V1)
    K1 = hamiltonian_1d(V1, dx, hbar, mass, nyquist_zero)
    w, phi = np.linalg.eigh(K1)
    def fwd(f):
        f = f.reshape(n, n, n)
        return np.einsum("zyx,xi,yj,zk->kji", f, phi, phi, phi, optimize=True)
    def inv(g):
        return np.einsum("kji,xi,yj,zk->zyx", g, phi, phi, phi, optimize=True).ravel()
    a0, b0 = fwd(np.asarray(psiR)), fwd(np.asarray(psiI))
    W = w[:, None, None] + w[None, :, None] + w[None, None, :]
    a, b = mode_power_apply(c, d, W * dt, nsteps, a0, b0)
    return inv(a), inv(b), w
