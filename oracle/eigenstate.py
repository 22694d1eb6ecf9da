"""Eigenstates from the time evolution -- oracle side (TEST INFRASTRUCTURE).

The paper shows eigenstates at chosen eigenfrequencies (Sec. 3.1 and 3.2,
Figs. 1, 2 and 4) obtained from the same time-domain run as the spectrum.
It does not state the recipe; the reading used here (and, in its own code,
by the engine) is the windowed Fourier sum of the state over the run,

    phi_E(r) = sum_{m=0}^{M-1} w_m psi(r, t_m) exp(+i E m dt / hbar),

with psi(r, t_m) the state after m + 1 steps counted from the start of the
accumulation and w_m the symmetric 4-term Blackman-Harris window of length
M (the spectrum's window).  A level E_j of the discrete operator, evolving
as exp(-i E_j t / hbar), adds coherently; the others are suppressed by the
window's sidelobes.  The states come from the oracle's own stepper, one
step at a time.
"""
from __future__ import annotations

import numpy as np

from . import run
from .spectrum import window


def reconstruct(psiR, psiI, V, n, dx, c, d, dt, energies, nsteps, hbar=1.0, mass=1.0,
                nyquist=0, bc=None, method=0):
    """Returns one complex array per energy (flat, x fastest) and the final
    state (psiR, psiI)."""
    w = window(nsteps)
    r, i = np.asarray(psiR, np.float64).ravel(), np.asarray(psiI, np.float64).ravel()
    acc = [np.zeros(r.size, np.complex128) for _ in energies]
    for m in range(nsteps):
        r, i, _, _ = run(r, i, V, n, dx, c, d, dt, 1, hbar=hbar, mass=mass, nyquist=nyquist,
                         bc=bc, method=method)
        psi = r + 1j * i
        for k, E in enumerate(energies):
            acc[k] += w[m] * np.exp(1j * E * m * dt / hbar) * psi
    return acc, (r, i)
