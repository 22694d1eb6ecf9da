"""Eigenvalues from probe time series -- oracle side (TEST INFRASTRUCTURE).

The paper reads eigenfrequencies off the Fourier transform of the wave
function recorded at a point over time (Sec. 3.1, the text before Table 2,
and Tables 2-4).  It states no window, padding or peak rule; the reading used
here (and, in its own independent code, by the engine) is:

1. per probe, the complex series s_n = psi_R - i psi_I (conjugated, so that
   psi ~ exp(-i E t / hbar) gives positive frequencies), n = 0 .. Ns-1;
2. the symmetric 4-term Blackman-Harris window w_n (Harris 1978,
   coefficients 0.35875, 0.48829, 0.14128, 0.01168) over n / (Ns - 1);
3. zero padding to M = 2**ceil(log2(8 Ns)) points and a DFT (NumPy's FFT
   is used as a library step); power summed over probes;
4. candidate bins k in [1, M/2 - 1): a local maximum of the power
   (above bin k-1, not below bin k+1) whose power exceeds 1e-8 of the
   largest (the window's sidelobes lie near 6e-10 in power);
5. each candidate refined on [theta_{k-1}, theta_{k+1}] to the zero of the
   derivative of the windowed DTFT power (bisection on its sign);
6. E = hbar * theta / dt, ascending; the lowest ``nlevels`` are returned.
"""
from __future__ import annotations

import numpy as np

BH4 = (0.35875, 0.48829, 0.14128, 0.01168)
REL_THRESHOLD = 1e-8


def window(ns: int) -> np.ndarray:
    """Symmetric 4-term Blackman-Harris window of length ns."""
    if ns == 1:
        return np.ones(1)
    t = 2.0 * np.pi * np.arange(ns) / (ns - 1)
    a0, a1, a2, a3 = BH4
    return a0 - a1 * np.cos(t) + a2 * np.cos(2 * t) - a3 * np.cos(3 * t)


def _power_and_slope(theta, ws, n):
    """Windowed DTFT power F(theta) = sum_p |sum_n ws_pn e^{-i theta n}|^2
    and dF/dtheta, evaluated directly (no recurrence)."""
    e = np.exp(-1j * theta * n)
    X = ws @ e                      # [P]
    dX = ws @ (-1j * n * e)         # [P]
    F = float(np.sum(np.abs(X) ** 2))
    dF = float(np.sum(2.0 * np.real(np.conj(X) * dX)))
    return F, dF


def extract(series, dt, hbar=1.0, nlevels=4):
    """series: array [Ns, P, 2] of (psi_R, psi_I) samples, one per step.

    Returns (E[nfound], amplitude[nfound]) for the lowest ``nlevels`` peaks."""
    series = np.asarray(series, dtype=np.float64)
    ns, npr = series.shape[0], series.shape[1]
    s = series[:, :, 0] - 1j * series[:, :, 1]          # [Ns, P], conjugated
    w = window(ns)
    ws = (w[:, None] * s).T                              # [P, Ns]
    M = 1 << int(np.ceil(np.log2(8 * ns)))
    spec = np.fft.fft(ws, n=M, axis=1)
    power = np.sum(np.abs(spec) ** 2, axis=0)
    half = M // 2
    pmax = np.max(power[:half])
    thr = REL_THRESHOLD * pmax
    cands = []
    for k in range(1, half - 1):
        pk = power[k]
        if pk <= thr:
            continue
        if not (pk > power[k - 1] and pk >= power[k + 1]):
            continue
        cands.append(k)
    n = np.arange(ns, dtype=np.float64)
    dth = 2.0 * np.pi / M
    thetas, amps = [], []
    for k in cands:
        a, b = (k - 1) * dth, (k + 1) * dth
        _, da = _power_and_slope(a, ws, n)
        _, db = _power_and_slope(b, ws, n)
        if da > 0.0 and db < 0.0:
            for _ in range(200):
                mid = 0.5 * (a + b)
                if mid <= a or mid >= b:
                    break
                _, dm = _power_and_slope(mid, ws, n)
                if dm > 0.0:
                    a = mid
                else:
                    b = mid
            th = 0.5 * (a + b)
        else:
            th = k * dth
        F, _ = _power_and_slope(th, ws, n)
        thetas.append(th)
        amps.append(np.sqrt(F) / np.sum(w))
    order = np.argsort(thetas)
    E = hbar * np.asarray(thetas)[order] / dt
    A = np.asarray(amps)[order]
    return E[:nlevels], A[:nlevels]
