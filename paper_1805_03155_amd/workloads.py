"""Seeded synthetic workloads: grids, potentials, initial states, probes.

This module produces inputs only.  It holds none of the method's arithmetic
(no transform, no operator, no time step, no stability bound) and it is the
one module that both the GPU engine's callers and the CPU oracle take their
inputs from.  Random draws use NumPy's PCG64 (``np.random.default_rng``).

Coefficient sets are inputs too: the engine and the oracle both take (c, d)
arrays.  PAPER is the fourth-order set printed in Sec. 2.1 (after Eq. 18)
and again before Table 1, with d_l = c_{m-l+1}.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# --- coefficient sets (c[m], d[m]); stage l applies c_l first, then d_l ---

PAPER_C = (0.26833010, -0.18799162, 0.91966152)
PAPER = (PAPER_C, tuple(reversed(PAPER_C)))

LEAPFROG = ((1.0,), (1.0,))

_FR_T = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
FOREST_RUTH = (
    (_FR_T / 2, (1 - _FR_T) / 2, (1 - _FR_T) / 2, _FR_T / 2),
    (_FR_T, 1 - 2 * _FR_T, _FR_T, 0.0),
)

# Yoshida (1990) sixth-order "solution A": a symmetric composition of seven
# second-order (kick-drift-kick) steps with weights (w3,w2,w1,w0,w1,w2,w3).
_Y_W1, _Y_W2, _Y_W3 = -1.17767998417887, 0.235573213359357, 0.784513610477560
_Y_W0 = 1.0 - 2.0 * (_Y_W1 + _Y_W2 + _Y_W3)
_Y_WS = (_Y_W3, _Y_W2, _Y_W1, _Y_W0, _Y_W1, _Y_W2, _Y_W3)
YOSHIDA6 = (
    tuple([_Y_WS[0] / 2] + [(_Y_WS[i] + _Y_WS[i + 1]) / 2 for i in range(6)]
          + [_Y_WS[6] / 2]),
    tuple(list(_Y_WS) + [0.0]),
)

COEFFS = {"paper": PAPER, "leapfrog": LEAPFROG, "forest_ruth": FOREST_RUTH,
          "yoshida6": YOSHIDA6}


@dataclass
class Workload:
    """One eigenvalue-solve problem on a periodic grid (x fastest)."""
    name: str
    n: tuple            # (nx,) / (nx, ny) / (nx, ny, nz)
    dx: tuple
    origin: tuple
    V: np.ndarray       # flat, row-major [nz][ny][nx]
    psiR: np.ndarray
    psiI: np.ndarray
    probes: np.ndarray  # linear grid indices (int64)
    steps: int
    coeffs: tuple = PAPER
    hbar: float = 1.0
    mass: float = 1.0
    cfl_fraction: float = 0.5
    meta: dict = field(default_factory=dict)
    bc: tuple = None    # boundary per axis (0 periodic, 1 Dirichlet, 2 Neumann); None: periodic

    @property
    def npoints(self) -> int:
        return int(np.prod(self.n))


def axis_coords(n, lo, hi):
    return lo + (hi - lo) * np.arange(n) / n


def snap(x, lo, d):
    """Nearest grid index of coordinate x on the grid lo + j*d."""
    return int(np.floor((x - lo) / d + 0.5))


def gaussians_1d(x, centers, amps, sigma):
    g = np.zeros_like(x)
    for mu, a in zip(centers, amps):
        g += a * np.exp(-((x - mu) ** 2) / (2.0 * sigma ** 2))
    return g


def finite_well_1d(seed=0, n=256, steps=20000, L=40.0, center=20.0,
                   half_width=5.0, V0=10.0, probe_x=21.3, coeffs=PAPER):
    """1D finite quantum well on the periodic grid [0, L): V = 0 strictly
    inside |x - center| < half_width, V0 elsewhere; psi_R = sum of 8 seeded
    Gaussians (sigma 0.5, centers uniform in the well, amplitudes N(0,1)),
    psi_I = 0; one probe snapped to the nearest grid point of probe_x."""
    rng = np.random.default_rng(seed)
    dx = L / n
    x = axis_coords(n, 0.0, L)
    V = np.where(np.abs(x - center) < half_width, 0.0, V0)
    mus = rng.uniform(center - half_width, center + half_width, 8)
    amps = rng.normal(0.0, 1.0, 8)
    psiR = gaussians_1d(x, mus, amps, 0.5)
    return Workload("finite_well_1d", (n,), (dx,), (0.0,), V, psiR,
                    np.zeros(n), np.array([snap(probe_x, 0.0, dx)], np.int64),
                    steps, coeffs, meta=dict(seed=seed, V0=V0, L=L))


def harmonic_3d(seed=0, n=64, half_box=8.0, omega=1.0, steps=10000,
                coeffs=PAPER, nprobes=3, probe_box=2.5):
    """Isotropic harmonic oscillator V = omega^2 r^2 / 2 on [-h, h)^3 with
    n^3 points; psi_R = exp(-|r - c|^2 / 2) with c uniform in [-1, 1]^3,
    psi_I = 0; probes at seeded points in [-probe_box, probe_box]^3 snapped
    to the grid."""
    rng = np.random.default_rng(seed)
    d = 2.0 * half_box / n
    x = axis_coords(n, -half_box, half_box)
    cx, cy, cz = rng.uniform(-1.0, 1.0, 3)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    V = (0.5 * omega ** 2 * (X ** 2 + Y ** 2 + Z ** 2)).ravel()
    psiR = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2) / 2.0).ravel()
    pts = rng.uniform(-probe_box, probe_box, (nprobes, 3))
    probes = []
    for px, py, pz in pts:
        ix, iy, iz = (snap(v, -half_box, d) for v in (px, py, pz))
        probes.append((iz * n + iy) * n + ix)
    return Workload(f"harmonic_3d_{n}", (n, n, n), (d, d, d),
                    (-half_box,) * 3, V, psiR, np.zeros(n ** 3),
                    np.array(probes, np.int64), steps, coeffs,
                    meta=dict(seed=seed, omega=omega, center=(cx, cy, cz),
                              V1=0.5 * omega ** 2 * x ** 2))


def cell_centres(n, L):
    """Sample points (j + 1/2) L / n of an axis between walls at 0 and L."""
    return (np.arange(n) + 0.5) * (L / n)


def walled_box(seed=0, n=(64, 32), L=(8.0, 6.0), bc=(1, 1), V0=0.0, steps=2000,
               coeffs=PAPER, nprobes=2):
    """A box with walls (Dirichlet 1 / Neumann 2 / periodic 0 per axis) on
    cell-centred samples: V = V0 * (seeded smooth bump), psi_R = a seeded
    Gaussian away from the centre, psi_I = 0, probes at seeded points within
    half a unit of the Gaussian's centre (where the state has weight)."""
    rng = np.random.default_rng(seed)
    dim = len(n)
    axes = [cell_centres(m, l) for m, l in zip(n, L)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")[::-1]      # x first
    ctr = [l * rng.uniform(0.3, 0.45) for l in L]
    r2 = sum((g - c) ** 2 for g, c in zip(grids, ctr))
    bump = np.exp(-sum((g - 0.6 * l) ** 2 for g, l in zip(grids, L)) / 2.0)
    V = (V0 * bump).ravel()
    psiR = np.exp(-r2 / 1.0).ravel()
    npts = int(np.prod(n))
    dx = tuple(l / m for m, l in zip(n, L))
    probes = []
    for _ in range(nprobes):
        idx = [min(m - 1, max(0, int((c + rng.uniform(-0.5, 0.5)) / h)))
               for c, m, h in zip(ctr, n, dx)]
        lin = 0
        for k in reversed(range(dim)):
            lin = lin * n[k] + idx[k]
        probes.append(lin)
    probes = np.array(probes, np.int64)
    return Workload(f"walled_{'x'.join(map(str, n))}", tuple(n), dx, (0.0,) * dim, V, psiR,
                    np.zeros(npts), probes, steps, coeffs, bc=tuple(bc),
                    meta=dict(seed=seed, L=L))


def harmonic_1d_potential(n, half_box, omega=1.0):
    x = axis_coords(n, -half_box, half_box)
    return 0.5 * omega ** 2 * x ** 2


def plane_wave_field(n, dx, kvec, phase=0.0):
    """cos(k . r + phase) sampled on the grid (flat, x fastest)."""
    axes = [np.arange(m) * h for m, h in zip(n, dx)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")   # [z][y][x] order
    arg = phase
    for g, k in zip(reversed(grids), kvec):
        arg = arg + k * g
    return np.cos(arg).ravel()


def random_field(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(int(np.prod(n)))


# --- batching form: many independent 1D / 2D instances ---------------------

def batch_instances(count=512, seed=0, steps=5000, box=20.0, max_1d_log2=14,
                    max_2d_log2=9, min_1d_log2=7, min_2d_log2=5, p2d=0.5,
                    coeffs=PAPER):
    """Independent instances on [-box, box)^dim: dim 1 or 2 (2 with
    probability p2d), sizes 2^U{...}, square wells (width U[2,20], depth
    U[1,50]) or harmonic wells (omega U[0.5,2]) with probability 1/2 each;
    psi_R = 8 seeded Gaussians (sigma 0.5) inside the well, psi_I = 0; one
    probe next to the first Gaussian."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        dim = 2 if rng.uniform() < p2d else 1
        if dim == 1:
            n = 1 << int(rng.integers(min_1d_log2, max_1d_log2 + 1))
            shape = (n,)
        else:
            n = 1 << int(rng.integers(min_2d_log2, max_2d_log2 + 1))
            shape = (n, n)
        d = 2.0 * box / n
        x = axis_coords(n, -box, box)
        grids = np.meshgrid(*([x] * dim), indexing="ij")[::-1]  # x first
        if rng.uniform() < 0.5:
            width = rng.uniform(2.0, 20.0)
            depth = rng.uniform(1.0, 50.0)
            inside = np.ones_like(grids[0], dtype=bool)
            for g in grids:
                inside &= np.abs(g) < width / 2
            V = np.where(inside, 0.0, depth)
            spread = width / 2
            kind = ("square", width, depth)
        else:
            om = rng.uniform(0.5, 2.0)
            V = 0.5 * om ** 2 * sum(g ** 2 for g in grids)
            spread = min(box / 2, 2.0 / np.sqrt(om))
            kind = ("harmonic", om)
        psi = np.zeros_like(V, dtype=np.float64)
        centres = []
        for _ in range(8):
            ctr = rng.uniform(-spread, spread, dim) * 0.8
            centres.append(ctr)
            a = rng.normal()
            r2 = sum((g - cc) ** 2 for g, cc in zip(grids, ctr))
            psi += a * np.exp(-r2 / (2 * 0.25))
        # the probe sits half a width from the first Gaussian, where the state has weight
        pc = centres[0] + 0.25
        idx = [min(n - 1, max(0, snap(v, -box, d))) for v in pc]
        lin = idx[0] if dim == 1 else idx[1] * n + idx[0]
        out.append(Workload(f"batch_{i}", shape, (d,) * dim, (-box,) * dim,
                            np.ascontiguousarray(V.ravel(), np.float64),
                            np.ascontiguousarray(psi.ravel(), np.float64),
                            np.zeros(V.size), np.array([lin], np.int64),
                            steps, coeffs, meta=dict(kind=kind, index=i)))
    return out
