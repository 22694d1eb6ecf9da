// Host-side helpers shared by the single-plan and the batch engines.
#pragma once
#include <cmath>
#include <vector>

#include "../../include/spstd.h"
#include "kernels.hpp"

namespace spstd {

static const double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------------------
// Stability edge from the trace polynomial of the per-mode matrix.
// The matrix of one step (Eq. 23) is the time-ordered product of the stage
// shears A(c_l x) = [[1, c_l x], [0, 1]] and B(d_l x) = [[1, 0], [-d_l x, 1]];
// its entries are polynomials in x of degree <= 2m.  tr = 2 + sum_l (-1)^l
// g_l x^(2l) (Eq. 26-28); the edge is the first x > 0 with |tr| > 2.
// ---------------------------------------------------------------------------
struct Poly {
    double a[2 * SPSTD_MAX_STAGES + 2];
    int deg;
};

static inline Poly pmul_x(const Poly& p, double s) {  // s * x * p(x)
    Poly r{};
    r.deg = p.deg + 1;
    for (int i = 0; i <= p.deg; ++i) r.a[i + 1] = s * p.a[i];
    return r;
}
static inline Poly padd(const Poly& p, const Poly& q) {
    Poly r{};
    r.deg = p.deg > q.deg ? p.deg : q.deg;
    for (int i = 0; i <= r.deg; ++i) r.a[i] = (i <= p.deg ? p.a[i] : 0.0) + (i <= q.deg ? q.a[i] : 0.0);
    return r;
}
static inline double peval(const Poly& p, double x) {
    double s = 0.0;
    for (int i = p.deg; i >= 0; --i) s = s * x + p.a[i];
    return s;
}

static inline bool trace_poly(int m, const double* c, const double* d, Poly* tr) {
    Poly m00{}, m01{}, m10{}, m11{};
    m00.a[0] = 1.0; m11.a[0] = 1.0;
    for (int l = 0; l < m; ++l) {
        // rows: A multiplies from the left: row0 += c x * row1
        Poly n00 = padd(m00, pmul_x(m10, c[l]));
        Poly n01 = padd(m01, pmul_x(m11, c[l]));
        // B: row1 -= d x * row0 (new row0)
        Poly n10 = padd(m10, pmul_x(n00, -d[l]));
        Poly n11 = padd(m11, pmul_x(n01, -d[l]));
        m00 = n00; m01 = n01; m10 = n10; m11 = n11;
    }
    *tr = padd(m00, m11);
    return true;
}

static inline bool xmax_symplectic(int m, const double* c, const double* d, double* out) {
    Poly tr;
    trace_poly(m, c, d, &tr);
    auto beyond = [&](double x) { return std::fabs(peval(tr, x)) > 2.0; };
    // scan in steps of 1/256 of a unit, then bisect the bracketing step
    const double h = 1.0 / 256.0;
    double lo = 0.0;
    for (int i = 1; i <= 256 * 1000; ++i) {
        double x = i * h;
        if (beyond(x)) {
            double hi = x;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                (beyond(mid) ? hi : lo) = mid;
            }
            *out = lo;
            return true;
        }
        lo = x;
    }
    return false;
}

// FP64 twiddles w_n^t = exp(-2 pi i t / n), from long-double cos/sin.
static inline std::vector<double> twiddles(int64_t n) {
    std::vector<double> t(2 * n);
    for (int64_t k = 0; k < n; ++k) {
        long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)n;
        t[2 * k] = (double)cosl(ang);
        t[2 * k + 1] = (double)sinl(ang);
    }
    return t;
}

// Transform length of axis a: n, or 2n for a walled axis (its samples and
// their mirror image form one period of length 2L).
static inline int64_t transform_len(const spstd_desc& d, int a) {
    return d.bc[a] == SPSTD_BC_PERIODIC ? d.n[a] : 2 * d.n[a];
}

// kinetic scale of axis a for substep coefficient coef:
// coef (hbar/2m) (2 pi/P)^2 / nt with nt the transform length and P = nt dx
// its period (the bare pass multiplies bin kk by kk^2).
static inline double kin_scale(const spstd_desc& d, int a, double coef) {
    if (a >= d.ndim) return 0.0;
    const double nt = (double)transform_len(d, a);
    const double k1 = 2.0 * kPi / (nt * d.dx[a]);
    return coef * d.hbar / (2.0 * d.mass) * k1 * k1 / nt;
}

// Kinetic scale of axis a under the three-point difference: the stencil
// kernel adds k (2 f[j] - f[j+1] - f[j-1]) with k = coef (hbar/2m*) / dx^2.
static inline double kin_scale_fd(const spstd_desc& d, int a, double coef) {
    if (a >= d.ndim) return 0.0;
    return coef * d.hbar / (2.0 * d.mass) / (d.dx[a] * d.dx[a]);
}

// One row of the scale table for substep coefficients a (A) and b (B).
static inline void scale_row(const spstd_desc& d, double a, double b, double* row) {
    const bool fd = d.laplacian == SPSTD_LAP_FD3;
    for (int ax = 0; ax < 3; ++ax) {
        row[SC_KXA + ax] = fd ? kin_scale_fd(d, ax, a) : kin_scale(d, ax, a);
        row[SC_KXB + ax] = fd ? kin_scale_fd(d, ax, b) : kin_scale(d, ax, b);
    }
    row[SC_PA] = a / d.hbar;
    row[SC_PB] = b / d.hbar;
}

// Geometry of the y (a = 1) or z (a = 2) pass over `ninst` stacked instances.
static inline AxisGeom axis_geom_of(const spstd_desc& d, int a, int64_t ninst) {
    AxisGeom g;
    const int64_t nx = d.n[0], ny = d.n[1], nz = d.n[2];
    g.half_x = nx / 2;
    g.stride_hi = nx * ny * nz;
    if (a == 1) { g.n_in = nz; g.stride_lo = nx * ny; g.stride = nx; }
    else { g.n_in = ny; g.stride_lo = nx; g.stride = nx * ny; }
    g.n_outer = ninst * g.n_in;
    return g;
}


// The same for a bare shape.
static inline AxisGeom axis_geom_of_n(int ndim, const int64_t* n, int a, int64_t ninst) {
    spstd_desc d{};
    d.ndim = ndim;
    for (int k = 0; k < 3; ++k) d.n[k] = n[k];
    return axis_geom_of(d, a, ninst);
}

// Spectral-radius bound of K on a grid with potential V (Eq. 24-30 with V):
// (hbar/2m*) sum_d (pi/dx_d)^2 + max|V|/hbar over the grid's axes.
static inline double rho_bound_of(int ndim, const double* dx, double hbar, double mass, const double* V,
                                  int64_t N, bool fd3 = false) {
    // the three-point difference's symbol 4 sin^2(k dx/2)/dx^2 peaks at 4/dx^2
    double r = 0.0;
    for (int a = 0; a < ndim; ++a) r += fd3 ? 4.0 / (dx[a] * dx[a]) : (kPi / dx[a]) * (kPi / dx[a]);
    r *= hbar / (2.0 * mass);
    double vm = 0.0;
    for (int64_t i = 0; i < N; ++i) vm = std::fmax(vm, std::fabs(V[i]));
    return r + vm / hbar;
}

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace spstd
