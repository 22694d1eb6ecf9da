/*
 * SPSTD oracle -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, double-precision CPU implementation of the symplectic
 * pseudospectral time-domain (SPSTD) scheme for the time-dependent
 * Schroedinger equation (Shen, Sha, Kuang, Hu, Huang, Wu, arXiv:1805.03155).
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no source, header, table or helper with
 * the GPU engine; its inputs are plain arrays produced by the seeded workload
 * generators.
 *
 * Every routine follows one passage of the paper:
 *   or_dft_naive      -- the discrete Fourier sum itself (definition, no FFT)
 *   or_fft            -- iterative radix-2 FFT, twiddles from cos/sin directly
 *   or_d2_axis        -- Sec. 2.1, Eq. (9)-(10): second derivative along one
 *                        axis by forward FT, wavenumber factor, inverse FT
 *   or_d2_axis_bc     -- Sec. 2.2 (last paragraph): the same along an axis
 *                        with Dirichlet or Neumann walls, by the sine or
 *                        cosine basis of the walled axis (plain sums)
 *   or_apply_K        -- Eq. (16): K = -(hbar/2m*) Laplacian + V/hbar
 *   or_mode_matrix    -- Eq. (23): per-mode evolution matrix of one step
 *   or_xmax           -- Eq. (24)-(25): first x with |tr L^d| = 2
 *   or_run            -- Eq. (17)-(18): stage-by-stage symplectic update;
 *                        also the PSTD (Eq. 11-12, one stage), classical RK4
 *                        and second-order finite-difference comparison runs
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *   - per stage l the psi_R update (coefficient c_l, source psi_I) comes
 *     first and the psi_I update (d_l, source the new psi_R) second; this is
 *     the order under which Table 1's ratio 1.503 is reproduced;
 *   - Nyquist convention: FULL uses the direct symbol -k^2 with
 *     |k| = pi/Delta at the Nyquist bin; ZERO is Eq. (10) taken literally
 *     (two first derivatives, real part kept after each inverse transform),
 *     which removes the Nyquist term.
 *
 * Built with -ffp-contract=off so that no fused multiply-add enters.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846264338327950288
#define OR_BC_PERIODIC 0
#define OR_BC_DIRICHLET 1
#define OR_BC_NEUMANN 2

/* ------------------------------------------------------------------ */
/* Discrete Fourier transform by its definition:                       */
/*   out[k] = sum_j in[j] * exp(sign * 2 pi i j k / n)                 */
/* O(n^2); the angle uses (j*k mod n) so that it stays exact.          */
/* ------------------------------------------------------------------ */
void or_dft_naive(int64_t n, const double *re, const double *im,
                  double *ore, double *oim, int sign)
{
    for (int64_t k = 0; k < n; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t jk = (j * k) % n;
            double ang = (double)sign * 2.0 * OR_PI * (double)jk / (double)n;
            double c = cos(ang), s = sin(ang);
            sr += re[j] * c - im[j] * s;
            si += re[j] * s + im[j] * c;
        }
        ore[k] = sr;
        oim[k] = si;
    }
}

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

/* ------------------------------------------------------------------ */
/* In-place iterative radix-2 decimation-in-time FFT (unnormalised).   */
/* sign = -1: forward, sign = +1: inverse.  Returns 0 on success.      */
/* ------------------------------------------------------------------ */
int or_fft(int64_t n, double *re, double *im, int sign)
{
    if (!is_pow2(n)) return -1;
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < n; ++i) {
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t half = len >> 1;
        for (int64_t k = 0; k < half; ++k) {
            /* twiddle exp(sign * 2 pi i k / len), evaluated directly */
            double ang = (double)sign * 2.0 * OR_PI * (double)k / (double)len;
            double wr = cos(ang), wi = sin(ang);
            for (int64_t s = 0; s < n; s += len) {
                int64_t a = s + k, b = s + k + half;
                double tr = re[b] * wr - im[b] * wi;
                double ti = re[b] * wi + im[b] * wr;
                re[b] = re[a] - tr;
                im[b] = im[a] - ti;
                re[a] = re[a] + tr;
                im[a] = im[a] + ti;
            }
        }
    }
    return 0;
}

/* Signed wavenumber K_j = 2 pi j / L of DFT bin j (Eq. 8), with the bin
 * n/2 taken as +pi/Delta. */
static double wavenumber(int64_t j, int64_t n, double L)
{
    int64_t js = (j <= n / 2) ? j : j - n;
    return 2.0 * OR_PI * (double)js / L;
}

/* Second derivative of one real pencil of length n and period L.
 * On input re[] holds the samples; on output re[] holds d^2 f / dx^2.
 * work_im is scratch of length n. */
static void d2_pencil(int64_t n, double L, int nyq_zero,
                      double *re, double *im)
{
    for (int64_t j = 0; j < n; ++j) im[j] = 0.0;
    or_fft(n, re, im, -1);
    if (!nyq_zero) {
        /* direct symbol: multiply by (i K)^2 = -K^2 */
        for (int64_t j = 0; j < n; ++j) {
            double K = wavenumber(j, n, L);
            re[j] *= -K * K;
            im[j] *= -K * K;
        }
        or_fft(n, re, im, +1);
        for (int64_t j = 0; j < n; ++j) re[j] /= (double)n;
    } else {
        /* Eq. (10) literally: d/dx twice, real part after each inverse */
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) {
                for (int64_t j = 0; j < n; ++j) im[j] = 0.0;
                or_fft(n, re, im, -1);
            }
            for (int64_t j = 0; j < n; ++j) {
                double K = wavenumber(j, n, L);
                double r = re[j], i = im[j];
                re[j] = -K * i; /* (i K)(r + i i_) = -K i_ + i K r */
                im[j] = K * r;
            }
            or_fft(n, re, im, +1);
            for (int64_t j = 0; j < n; ++j) re[j] /= (double)n;
        }
    }
}

/* Axis strides of a row-major [nz][ny][nx] field (x fastest). */
static void axis_geometry(const int64_t *n, int axis, int64_t *len,
                          int64_t *stride, int64_t *npencil)
{
    int64_t nx = n[0], ny = n[1], nz = n[2];
    *len = n[axis];
    *stride = (axis == 0) ? 1 : (axis == 1) ? nx : nx * ny;
    *npencil = (nx * ny * nz) / n[axis];
}

/* Base index of pencil p along the axis. */
static int64_t pencil_base(const int64_t *n, int axis, int64_t p)
{
    int64_t nx = n[0], ny = n[1];
    if (axis == 0) return p * nx;                         /* p = z*ny + y */
    if (axis == 1) return (p / nx) * nx * ny + (p % nx);  /* p = z*nx + x */
    return p;                                             /* p = y*nx + x */
}

/* ------------------------------------------------------------------ */
/* Walled axes (Sec. 2.2, last paragraph: sine transform for Dirichlet,  */
/* cosine transform for Neumann walls).  Samples sit at cell centres     */
/* x_j = (j + 1/2) Delta, j = 0..n-1, with walls at x = 0 and x = L =    */
/* n Delta.  Basis vectors                                               */
/*   Dirichlet: b_k(j) = sin(pi k (j + 1/2) / n),  k = 1..n              */
/*   Neumann:   b_k(j) = cos(pi k (j + 1/2) / n),  k = 0..n-1            */
/* are samples of the wall eigenfunctions, each an exact eigenvector of  */
/* d^2/dx^2 with eigenvalue -(pi k / L)^2.  f is expanded by orthogonal  */
/* projection, a_k = sum_j f_j b_k(j) / sum_j b_k(j)^2, and the          */
/* expansion is differentiated term by term.  The Dirichlet k = n vector */
/* alternates in sign (the Nyquist mode of the mirrored grid): under the */
/* ZERO convention its eigenvalue is taken as 0, as for the periodic     */
/* Nyquist bin.                                                          */
/* ------------------------------------------------------------------ */
static int64_t wall_wavenumber_index(int bc, int64_t row)
{
    return bc == OR_BC_DIRICHLET ? row + 1 : row;
}

/* The basis of the last (n, bc) asked for is kept: a run applies the same
 * axis operator at every substep. */
static double *g_basis = NULL;
static int64_t g_basis_n = 0;
static int g_basis_bc = -1;

static double *wall_basis(int64_t n, int bc)
{
    if (g_basis && g_basis_n == n && g_basis_bc == bc) return g_basis;
    free(g_basis);
    g_basis = NULL;
    double *B = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!B) return NULL;
    for (int64_t r = 0; r < n; ++r) {
        int64_t k = wall_wavenumber_index(bc, r);
        for (int64_t j = 0; j < n; ++j) {
            double arg = OR_PI * (double)k * ((double)j + 0.5) / (double)n;
            B[r * n + j] = bc == OR_BC_DIRICHLET ? sin(arg) : cos(arg);
        }
    }
    g_basis = B;
    g_basis_n = n;
    g_basis_bc = bc;
    return B;
}

static void d2_pencil_wall(int64_t n, double L, int bc, int nyq_zero,
                           const double *B, double *f, double *a)
{
    for (int64_t r = 0; r < n; ++r) {
        double num = 0.0, den = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            num += f[j] * B[r * n + j];
            den += B[r * n + j] * B[r * n + j];
        }
        int64_t k = wall_wavenumber_index(bc, r);
        double K = OR_PI * (double)k / L;
        if (nyq_zero && bc == OR_BC_DIRICHLET && k == n) K = 0.0;
        a[r] = -K * K * num / den;
    }
    for (int64_t j = 0; j < n; ++j) f[j] = 0.0;
    for (int64_t r = 0; r < n; ++r)
        for (int64_t j = 0; j < n; ++j) f[j] += a[r] * B[r * n + j];
}

/* ------------------------------------------------------------------ */
/* out = d^2 f / d(axis)^2 (spectral, Eq. 9-10).  n[3] = (nx, ny, nz); */
/* L = n[axis] * dx.  Axes of length 1 give zero.  bc: boundary of the   */
/* axis (OR_BC_PERIODIC, OR_BC_DIRICHLET, OR_BC_NEUMANN).                */
/* ------------------------------------------------------------------ */
int or_d2_axis_bc(const int64_t *n, const double *dx, int axis, int bc,
                  int nyq_zero, const double *f, double *out)
{
    int64_t len, stride, npen;
    axis_geometry(n, axis, &len, &stride, &npen);
    if (len == 1) {
        for (int64_t i = 0; i < n[0] * n[1] * n[2]; ++i) out[i] = 0.0;
        return 0;
    }
    double L = (double)len * dx[axis];
    if (bc != OR_BC_PERIODIC) {
        if (bc != OR_BC_DIRICHLET && bc != OR_BC_NEUMANN) return -1;
        double *B = wall_basis(len, bc);
        if (!B) return -2;
#pragma omp parallel
        {
            double *v = (double *)malloc(sizeof(double) * (size_t)len);
            double *a = (double *)malloc(sizeof(double) * (size_t)len);
#pragma omp for schedule(static)
            for (int64_t p = 0; p < npen; ++p) {
                int64_t b = pencil_base(n, axis, p);
                for (int64_t j = 0; j < len; ++j) v[j] = f[b + j * stride];
                d2_pencil_wall(len, L, bc, nyq_zero, B, v, a);
                for (int64_t j = 0; j < len; ++j) out[b + j * stride] = v[j];
            }
            free(v);
            free(a);
        }
        return 0;
    }
    if (!is_pow2(len)) return -1;
#pragma omp parallel
    {
        double *re = (double *)malloc(sizeof(double) * (size_t)len);
        double *im = (double *)malloc(sizeof(double) * (size_t)len);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < npen; ++p) {
            int64_t b = pencil_base(n, axis, p);
            for (int64_t j = 0; j < len; ++j) re[j] = f[b + j * stride];
            d2_pencil(len, L, nyq_zero, re, im);
            for (int64_t j = 0; j < len; ++j) out[b + j * stride] = re[j];
        }
        free(re);
        free(im);
    }
    return 0;
}

int or_d2_axis(const int64_t *n, const double *dx, int axis, int nyq_zero,
               const double *f, double *out)
{
    return or_d2_axis_bc(n, dx, axis, OR_BC_PERIODIC, nyq_zero, f, out);
}

/* Second-order central difference (f[i+1] - 2 f[i] + f[i-1]) / dx^2 with
 * periodic wrap: the spatial operator of the FDTD comparison method. */
static int fd3_axis(const int64_t *n, const double *dx, int axis,
                    const double *f, double *out)
{
    int64_t len, stride, npen;
    axis_geometry(n, axis, &len, &stride, &npen);
    if (len == 1) {
        for (int64_t i = 0; i < n[0] * n[1] * n[2]; ++i) out[i] = 0.0;
        return 0;
    }
    double inv = 1.0 / (dx[axis] * dx[axis]);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npen; ++p) {
        int64_t b = pencil_base(n, axis, p);
        for (int64_t j = 0; j < len; ++j) {
            int64_t jm = (j + len - 1) % len, jp = (j + 1) % len;
            out[b + j * stride] = (f[b + jp * stride] - 2.0 * f[b + j * stride]
                                   + f[b + jm * stride]) * inv;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* K f = -(hbar / 2 m*) (d2x + d2y + d2z) f + (V / hbar) f   (Eq. 16)  */
/* laplacian: 0 = spectral (Eq. 9-10), 1 = 3-point finite difference. */
/* ------------------------------------------------------------------ */
int or_apply_K(const int64_t *n, const double *dx, double hbar, double mass,
               int nyq_zero, int laplacian, const int *bc, const double *V,
               const double *f, double *out)
{
    int64_t N = n[0] * n[1] * n[2];
    double *tmp = (double *)malloc(sizeof(double) * (size_t)N);
    if (!tmp) return -2;
    for (int64_t i = 0; i < N; ++i) out[i] = 0.0;
    for (int axis = 0; axis < 3; ++axis) {
        int b = bc ? bc[axis] : OR_BC_PERIODIC;
        int rc = laplacian ? (b == OR_BC_PERIODIC ? fd3_axis(n, dx, axis, f, tmp) : -1)
                           : or_d2_axis_bc(n, dx, axis, b, nyq_zero, f, tmp);
        if (rc) { free(tmp); return rc; }
        for (int64_t i = 0; i < N; ++i) out[i] += tmp[i];
    }
    double a = -hbar / (2.0 * mass);
    for (int64_t i = 0; i < N; ++i)
        out[i] = a * out[i] + (V ? V[i] / hbar * f[i] : 0.0);
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Per-mode evolution matrix of one time step (Eq. 23).  For a mode     */
/* with K phi = omega phi and x = omega * dt, stage l acts as           */
/*   A: (r, i) -> (r + c_l x i, i)   then   B: (r, i) -> (r, i - d_l x r)*/
/* M is returned row-major: M = [[M0, M1], [M2, M3]].                  */
/* ------------------------------------------------------------------ */
void or_mode_matrix(int m, const double *c, const double *d, double x,
                    double *M)
{
    double a = 1.0, b = 0.0, e = 0.0, f = 1.0; /* identity [[a,b],[e,f]] */
    for (int l = 0; l < m; ++l) {
        /* left-multiply by A(c_l x) = [[1, c x], [0, 1]] */
        double cx = c[l] * x;
        a = a + cx * e;
        b = b + cx * f;
        /* left-multiply by B(d_l x) = [[1, 0], [-d x, 1]] */
        double dxl = d[l] * x;
        e = e - dxl * a;
        f = f - dxl * b;
    }
    M[0] = a; M[1] = b; M[2] = e; M[3] = f;
}

/* Stability edge (Eq. 24-25): the smallest x > 0 beyond which
 * |tr M(x)| exceeds 2.  Coarse scan, then bisection to full precision. */
double or_xmax(int m, const double *c, const double *d)
{
    double M[4];
    double h = 1e-3, x = 0.0;
    for (;;) {
        double xn = x + h;
        or_mode_matrix(m, c, d, xn, M);
        if (fabs(0.5 * (M[0] + M[3])) > 1.0) break;
        x = xn;
        if (x > 1e3) return INFINITY;
    }
    double lo = x, hi = x + h;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        or_mode_matrix(m, c, d, mid, M);
        if (fabs(0.5 * (M[0] + M[3])) > 1.0) hi = mid; else lo = mid;
    }
    return lo;
}

/* Upper bound of the spectral radius of K on the grid (V >= 0 not assumed):
 * (hbar/2m*) sum_d (pi/dx_d)^2 over axes of length > 1, plus max|V|/hbar. */
double or_rho_bound(const int64_t *n, const double *dx, double hbar,
                    double mass, const double *V)
{
    double r = 0.0;
    for (int a = 0; a < 3; ++a)
        if (n[a] > 1) r += (OR_PI / dx[a]) * (OR_PI / dx[a]);
    r *= hbar / (2.0 * mass);
    double vmax = 0.0;
    int64_t N = n[0] * n[1] * n[2];
    for (int64_t i = 0; i < N && V; ++i)
        if (fabs(V[i]) > vmax) vmax = fabs(V[i]);
    return r + vmax / hbar;
}

static double norm2(int64_t N, const double *r, const double *i)
{
    double s = 0.0;
    for (int64_t k = 0; k < N; ++k) s += r[k] * r[k] + i[k] * i[k];
    return s;
}

static void record(int nprobes, const int64_t *pidx, const double *r,
                   const double *i, double *out)
{
    for (int p = 0; p < nprobes; ++p) {
        out[2 * p] = r[pidx[p]];
        out[2 * p + 1] = i[pidx[p]];
    }
}

/* ------------------------------------------------------------------ */
/* Time stepping.                                                       */
/*   method 0: partitioned symplectic scheme of Eq. (17)-(18) with      */
/*             coefficient arrays c[m], d[m] (PSTD = m 1, c = d = 1);   */
/*   method 1: classical fourth-order Runge-Kutta on                    */
/*             d/dt (psi_R, psi_I) = (K psi_I, -K psi_R).               */
/* laplacian: 0 spectral, 1 second-order finite difference (FDTD).      */
/* probe_out: [(nsteps+1)][nprobes][2] samples (psi_R, psi_I), sample 0 */
/* is the initial state; norm_out: [(nsteps+1)] sums of |psi|^2 (no    */
/* cell volume).  Either may be NULL.  psiR, psiI are advanced in place.*/
/* ------------------------------------------------------------------ */
int or_run(const int64_t *n, const double *dx, double hbar, double mass,
           int nyq_zero, int laplacian, const int *bc, int method, const double *V,
           double *psiR, double *psiI, int m, const double *c,
           const double *d, double dt, int64_t nsteps, int nprobes,
           const int64_t *probe_idx, double *probe_out, double *norm_out)
{
    int64_t N = n[0] * n[1] * n[2];
    double *Kf = (double *)malloc(sizeof(double) * (size_t)N);
    double *k[4][2] = {{0}};
    double *yr = NULL, *yi = NULL;
    if (!Kf) return -2;
    if (method == 1) {
        for (int s = 0; s < 4; ++s)
            for (int q = 0; q < 2; ++q)
                k[s][q] = (double *)malloc(sizeof(double) * (size_t)N);
        yr = (double *)malloc(sizeof(double) * (size_t)N);
        yi = (double *)malloc(sizeof(double) * (size_t)N);
    }
    if (probe_out) record(nprobes, probe_idx, psiR, psiI, probe_out);
    if (norm_out) norm_out[0] = norm2(N, psiR, psiI);
    int rc = 0;
    for (int64_t step = 0; step < nsteps && rc == 0; ++step) {
        if (method == 0) {
            for (int l = 0; l < m && rc == 0; ++l) {
                if (c[l] != 0.0) { /* A: psi_R <- psi_R + c_l dt K psi_I */
                    rc = or_apply_K(n, dx, hbar, mass, nyq_zero, laplacian, bc, V,
                                    psiI, Kf);
                    for (int64_t q = 0; q < N; ++q) psiR[q] += c[l] * dt * Kf[q];
                }
                if (d[l] != 0.0 && rc == 0) { /* B: psi_I <- psi_I - d_l dt K psi_R */
                    rc = or_apply_K(n, dx, hbar, mass, nyq_zero, laplacian, bc, V,
                                    psiR, Kf);
                    for (int64_t q = 0; q < N; ++q) psiI[q] -= d[l] * dt * Kf[q];
                }
            }
        } else {
            static const double a_in[4] = {0.0, 0.5, 0.5, 1.0};
            for (int s = 0; s < 4 && rc == 0; ++s) {
                for (int64_t q = 0; q < N; ++q) {
                    yr[q] = psiR[q] + (s ? a_in[s] * dt * k[s - 1][0][q] : 0.0);
                    yi[q] = psiI[q] + (s ? a_in[s] * dt * k[s - 1][1][q] : 0.0);
                }
                rc = or_apply_K(n, dx, hbar, mass, nyq_zero, laplacian, bc, V, yi,
                                k[s][0]);
                if (rc == 0)
                    rc = or_apply_K(n, dx, hbar, mass, nyq_zero, laplacian, bc, V,
                                    yr, k[s][1]);
                for (int64_t q = 0; q < N; ++q) k[s][1][q] = -k[s][1][q];
            }
            for (int64_t q = 0; q < N; ++q) {
                psiR[q] += dt / 6.0 * (k[0][0][q] + 2.0 * k[1][0][q]
                                       + 2.0 * k[2][0][q] + k[3][0][q]);
                psiI[q] += dt / 6.0 * (k[0][1][q] + 2.0 * k[1][1][q]
                                       + 2.0 * k[2][1][q] + k[3][1][q]);
            }
        }
        if (probe_out)
            record(nprobes, probe_idx, psiR, psiI,
                   probe_out + (step + 1) * 2 * nprobes);
        if (norm_out) norm_out[step + 1] = norm2(N, psiR, psiI);
    }
    free(Kf);
    if (method == 1) {
        for (int s = 0; s < 4; ++s)
            for (int q = 0; q < 2; ++q) free(k[s][q]);
        free(yr);
        free(yi);
    }
    return rc;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the calling host thread's later parallel regions (for several
 * oracle runs side by side on host threads). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
