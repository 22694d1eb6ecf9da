// SPSTD device kernels for gfx950 (MI355X): launchers of the directional
// passes (passes.hpp), the small kernels (probes, norms, energy, walls,
// the difference operator, eigenstate sums) and their launchers.
#include "passes.hpp"

namespace spstd {

bool axis_len_ok(int64_t n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }
bool row_len_ok(int64_t n) { return n >= 16 && n <= 16384 && (n & (n - 1)) == 0; }
// Walled axes whose mirrored line of 2n points is not one the FFT passes
// take (a power of two of at least 32): the direct Fourier sum, n <= 32.
bool wall_dft_len_ok(int64_t n) { return n >= 2 && n <= 32 && n != 16 && n != 32; }

constexpr int kWPB = 4;             // waves per block of the wave-local passes
constexpr int kWPBF64Fused256 = 2;  // ... of the FP64 256-point fused kernels (boundary sweep, x passes)

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_probe(const R* __restrict__ psiR, const R* __restrict__ psiI,
                        const int64_t* __restrict__ idx, int nprobes, int64_t npts, double* __restrict__ out,
                        int64_t* __restrict__ counter, int64_t capacity, int* __restrict__ fault) {
    const int64_t slot = *counter;
    const int t = threadIdx.x;
    if (slot < capacity && t < nprobes) {
        const int64_t i = idx[t];
        // an index outside the grid (device memory not holding what the host
        // wrote) skips the sample and raises the flag the host checks
        if (i >= 0 && i < npts) {
            out[(slot * nprobes + t) * 2 + 0] = (double)psiR[i];
            out[(slot * nprobes + t) * 2 + 1] = (double)psiI[i];
        } else {
            *fault = 1;
        }
    }
    __syncthreads();
    if (t == 0) *counter = slot + 1;
}

template <typename R>
__global__ __launch_bounds__(256) void k_norm_partials(const R* __restrict__ a, const R* __restrict__ b,
                                                       int64_t n, double* __restrict__ partials) {
    __shared__ double red[256];
    double s = 0.0;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double x = (double)a[i], y = (double)b[i];
        s += x * x + y * y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// Energy diagnostics.  Along one axis the kinetic energy of psi = psi_R +
// i psi_I is (hbar^2/2m*) (2 pi/L)^2 / n * sum over lines and bins of
// ks^2 |FFT_axis(psi)(k)|^2 (Parseval with the symbol of Eq. 9-10): each line
// of the field is one complex pencil (psi_R, psi_I), transformed forward
// only.  Blocks walk the lines with a fixed stride and write one FP64
// partial each, so the sum has a fixed order.
// ---------------------------------------------------------------------------
template <int THREADS>
__device__ __forceinline__ void block_sum_store(double s, double* out) {
    __shared__ double wsum[THREADS / 64 > 0 ? THREADS / 64 : 1];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (THREADS + 63) / 64; ++w) t += wsum[w];
        *out = t;
    }
}

// Transform position i = j + T e of an N-point pencil read from memory.  A
// periodic line maps i to itself.  A walled line holds n = N/2 cell-centred
// samples; the transform sees it extended by its mirror image about the wall
// at x = L (position N - 1 - i for i >= n), times msign (-1 for Dirichlet,
// odd about the walls; +1 for Neumann, even).  The extended line has period
// 2L, so the pencil transform of length 2n diagonalises the walled operator.
template <int N, bool WALL>
__device__ __forceinline__ int line_pos(int j, int e) {
    constexpr int T = N / 16;
    return (WALL && e >= 8) ? N - 1 - (j + T * e) : j + T * e;
}

template <typename R, int N, bool ROWS, bool WALL>
__global__ __launch_bounds__((row_map<R, N, kWPB>::THREADS)) void k_energy_axis(
    const R* __restrict__ psiR, const R* __restrict__ psiI, const cpx<double>* __restrict__ tw,
    EnergyGeom g, int nyq_zero, R msign, double* __restrict__ partials) {
    using C = pencil_cfg<N>;
    using M = row_map<R, N, kWPB>;
    using TU = tuning<R>;
    __shared__ R lds[M::LDS_REALS];
    int j, pin;
    if constexpr (C::WAVE) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        // rows: lanes run along the line; columns: neighbouring lanes take
        // neighbouring lines (neighbouring x)
        const int pw = ROWS ? lane / C::T : lane % C::PPW;
        j = ROWS ? lane % C::T : lane / C::PPW;
        pin = wave * C::PPW + pw;
    } else {
        j = threadIdx.x;
        pin = 0;
    }
    double acc = 0.0;
    for (int64_t L0 = (int64_t)blockIdx.x * M::PPB; L0 < g.nlines; L0 += (int64_t)gridDim.x * M::PPB) {
        const int64_t L = L0 + pin;
        const bool valid = L < g.nlines;
        const int64_t base = valid ? (L / g.n_lo) * g.stride_hi + (L % g.n_lo) : 0;
        cpx<R> v[1][16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t q = base + (int64_t)line_pos<N, WALL>(j, e) * g.stride;
            const R sg = (WALL && e >= 8) ? msign : (R)1;
            v[0][e] = valid ? cpx<R>{sg * psiR[q], sg * psiI[q]} : cpx<R>{(R)0, (R)0};
        }
        fft_pencils<R, N, false, C::WAVE, M::SPLIT, TU::PRODUCTS, 1, (ROWS ? 1 : C::PPW)>(v, j, lds + pin * M::SL, M::SL, tw);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int kk = j + C::T * e;
            const int ks = (kk <= N / 2) ? kk : kk - N;
            double s = (double)ks * (double)ks;
            if (nyq_zero && kk == N / 2) s = 0.0;
            const double re = (double)v[0][e].x, im = (double)v[0][e].y;
            acc += s * (re * re + im * im);
        }
    }
    block_sum_store<M::THREADS>(acc, partials + blockIdx.x);
}

// ---------------------------------------------------------------------------
// Pass along a walled axis (Sec. 2.2, last paragraph: sine transform between
// Dirichlet walls, cosine transform between Neumann walls), any axis:
//   dst += k * T_axis src  (+ p * V * src when pcol >= 0)
// on the cell-centred samples of the axis, with T_axis applied as the
// periodic operator of the mirrored line (line_pos): an N = 2n point
// transform whose bins are the wall modes.  Two neighbouring lines (rows, or
// x columns) form one complex pencil; only the n stored samples are updated.
// ROWS: the lines are contiguous (x axis), lanes run along them; otherwise
// neighbouring lanes take neighbouring lines.  Instance of a line: its first
// sample / npts (stacked instances of a batch).
// ---------------------------------------------------------------------------
template <typename R, int N, bool ROWS>
__global__ __launch_bounds__((row_map<R, N, kWPB>::THREADS)) void k_wall_acc(
    const R* __restrict__ src, R* __restrict__ dst, const R* __restrict__ V,
    const cpx<double>* __restrict__ tw, EnergyGeom g, int64_t npts, ScaleRef sc, int kcol, int pcol,
    int nyq_zero, R msign) {
    using C = pencil_cfg<N>;
    using M = row_map<R, N, kWPB>;
    using TU = tuning<R>;
    __shared__ R lds[M::LDS_REALS];
    int j, pin;
    if constexpr (C::WAVE) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int pw = ROWS ? lane / C::T : lane % C::PPW;
        j = ROWS ? lane % C::T : lane / C::PPW;
        pin = wave * C::PPW + pw;
    } else {
        j = threadIdx.x;
        pin = 0;
    }
    const int64_t q = (int64_t)blockIdx.x * M::PPB + pin;     // pencil: lines 2q, 2q + 1
    const bool ok0 = 2 * q < g.nlines, ok1 = 2 * q + 1 < g.nlines;
    const int64_t L0 = ok0 ? 2 * q : 0, L1 = ok1 ? 2 * q + 1 : L0;
    const int64_t b0 = (L0 / g.n_lo) * g.stride_hi + (L0 % g.n_lo);
    const int64_t b1 = (L1 / g.n_lo) * g.stride_hi + (L1 % g.n_lo);
    const int64_t i0 = b0 / npts, i1 = b1 / npts;
    const R k0 = scale_of<R>(sc, i0, kcol), k1 = scale_of<R>(sc, i1, kcol);
    const R p0 = pcol >= 0 ? scale_of<R>(sc, i0, pcol) : (R)0;
    const R p1 = pcol >= 0 ? scale_of<R>(sc, i1, pcol) : (R)0;
    cpx<R> v[1][16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t m = (int64_t)line_pos<N, true>(j, e) * g.stride;
        const R sg = e >= 8 ? msign : (R)1;
        v[0][e] = cpx<R>{ok0 ? sg * src[b0 + m] : (R)0, ok1 ? sg * src[b1 + m] : (R)0};
    }
    R* l0 = lds + pin * M::SL;
    fft_pencils<R, N, false, C::WAVE, M::SPLIT, TU::PRODUCTS, 1, (ROWS ? 1 : C::PPW)>(v, j, l0, M::SL, tw);
    apply_k2<R, N>(v[0], j, nyq_zero);
    fft_pencils<R, N, true, C::WAVE, M::SPLIT, TU::PRODUCTS, 1, (ROWS ? 1 : C::PPW)>(v, j, l0, M::SL, tw);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t m = (int64_t)(j + C::T * e) * g.stride;
        if (ok0) {
            R t = dst[b0 + m] + k0 * v[0][e].x;
            if (pcol >= 0) t += p0 * V[b0 + m] * src[b0 + m];
            dst[b0 + m] = t;
        }
        if (ok1) {
            R t = dst[b1 + m] + k1 * v[0][e].y;
            if (pcol >= 0) t += p1 * V[b1 + m] * src[b1 + m];
            dst[b1 + m] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// Walled axes of few cells whose mirrored line is not a power of two of at
// least 16 points (n <= 32 cells, e.g. the 10-cell wells of Sec. 3.1-3.2):
// the mirrored line of M = 2n points goes through the discrete Fourier sum
// itself, M^2 products per line (a few hundred for these lines, where a
// mixed-radix transform would save nothing measurable), with the same
// mirror, symbol and scales as k_wall_acc.  One 64-lane block per complex
// pencil (two neighbouring lines); lane t owns bin t and sample t.
// Twiddles: the FP64 table w_M^s, s < M, indexed by (s t) mod M.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void wall_dft_load(cpx<R>* u, const R* __restrict__ src, int n, int64_t b0, int64_t b1,
                                              bool ok0, bool ok1, int64_t stride, R msign) {
    const int t = threadIdx.x, M = 2 * n;
    if (t < M) {
        const int p = t < n ? t : M - 1 - t;
        const R sg = t < n ? (R)1 : msign;
        u[t] = cpx<R>{ok0 ? sg * src[b0 + (int64_t)p * stride] : (R)0, ok1 ? sg * src[b1 + (int64_t)p * stride] : (R)0};
    }
}

// out = sum_s in[s] w^(sign s t), w = exp(-2 pi i / M), for lane t < M
template <typename R>
__device__ __forceinline__ cpx<R> wall_dft_sum(const cpx<R>* in, const cpx<double>* __restrict__ tw, int M, int t,
                                               bool inverse) {
    R ar = (R)0, ai = (R)0;
    for (int s = 0; s < M; ++s) {
        const cpx<double> w = tw[(s * t) % M];
        const R wr = (R)w.x, wi = inverse ? -(R)w.y : (R)w.y;
        ar += in[s].x * wr - in[s].y * wi;
        ai += in[s].x * wi + in[s].y * wr;
    }
    return cpx<R>{ar, ai};
}

template <typename R>
__global__ __launch_bounds__(64) void k_wall_dft_acc(const R* __restrict__ src, R* __restrict__ dst,
                                                     const R* __restrict__ V, const cpx<double>* __restrict__ tw,
                                                     int n, EnergyGeom g, int64_t npts, ScaleRef sc, int kcol,
                                                     int pcol, int nyq_zero, R msign) {
    __shared__ cpx<R> u[64], U[64];
    const int t = threadIdx.x, M = 2 * n;
    const int64_t q = blockIdx.x;
    const bool ok0 = 2 * q < g.nlines, ok1 = 2 * q + 1 < g.nlines;
    const int64_t L0 = ok0 ? 2 * q : 0, L1 = ok1 ? 2 * q + 1 : L0;
    const int64_t b0 = (L0 / g.n_lo) * g.stride_hi + (L0 % g.n_lo);
    const int64_t b1 = (L1 / g.n_lo) * g.stride_hi + (L1 % g.n_lo);
    wall_dft_load<R>(u, src, n, b0, b1, ok0, ok1, g.stride, msign);
    __syncthreads();
    if (t < M) {
        const cpx<R> a = wall_dft_sum<R>(u, tw, M, t, false);
        const int ks = t <= M / 2 ? t : t - M;
        const R sym = (nyq_zero && t == M / 2) ? (R)0 : (R)(ks * ks);
        U[t] = cpx<R>{a.x * sym, a.y * sym};
    }
    __syncthreads();
    if (t < n) {
        const cpx<R> r = wall_dft_sum<R>(U, tw, M, t, true);
        const int64_t i0 = b0 / npts, i1 = b1 / npts;
        const int64_t m = (int64_t)t * g.stride;
        if (ok0) {
            R v = dst[b0 + m] + scale_of<R>(sc, i0, kcol) * r.x;
            if (pcol >= 0) v += scale_of<R>(sc, i0, pcol) * V[b0 + m] * src[b0 + m];
            dst[b0 + m] = v;
        }
        if (ok1) {
            R v = dst[b1 + m] + scale_of<R>(sc, i1, kcol) * r.y;
            if (pcol >= 0) v += scale_of<R>(sc, i1, pcol) * V[b1 + m] * src[b1 + m];
            dst[b1 + m] = v;
        }
    }
}

// Energy sums of the same lines: partials[b] = sum over the block's pencils
// of ks^2 |DFT(mirrored psiR + i psiI)(k)|^2 (cf. k_energy_axis).
template <typename R>
__global__ __launch_bounds__(64) void k_wall_dft_energy(const R* __restrict__ psiR, const R* __restrict__ psiI,
                                                        const cpx<double>* __restrict__ tw, int n, EnergyGeom g,
                                                        int nyq_zero, R msign, double* __restrict__ partials) {
    __shared__ cpx<R> u[64];
    const int t = threadIdx.x, M = 2 * n;
    double acc = 0.0;
    for (int64_t L = blockIdx.x; L < g.nlines; L += gridDim.x) {
        const int64_t b = (L / g.n_lo) * g.stride_hi + (L % g.n_lo);
        if (t < M) {
            const int p = t < n ? t : M - 1 - t;
            const R sg = t < n ? (R)1 : msign;
            u[t] = cpx<R>{sg * psiR[b + (int64_t)p * g.stride], sg * psiI[b + (int64_t)p * g.stride]};
        }
        __syncthreads();
        if (t < M) {
            const cpx<R> a = wall_dft_sum<R>(u, tw, M, t, false);
            const int ks = t <= M / 2 ? t : t - M;
            const double sym = (nyq_zero && t == M / 2) ? 0.0 : (double)ks * (double)ks;
            acc += sym * ((double)a.x * (double)a.x + (double)a.y * (double)a.y);
        }
        __syncthreads();
    }
    block_sum_store<64>(acc, partials + blockIdx.x);
}

// ---------------------------------------------------------------------------
// Finite-difference comparison (the FDTD column of Tables 1-3): one substep
// over all axes at once,
//   dst += sum_d k_d (2 f[j] - f[j + e_d] - f[j - e_d]) + p V f,
// periodic wrap, k_d = coef (hbar/2m*) / dx_d^2 from column kcol0 + d.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_fd_acc(const R* __restrict__ src, R* __restrict__ dst,
                                                const R* __restrict__ V, int64_t nx, int64_t ny,
                                                int64_t nz, ScaleRef sc, int kcol0, int pcol) {
    const R kx = scale_of<R>(sc, 0, kcol0), ky = scale_of<R>(sc, 0, kcol0 + 1);
    const R kz = scale_of<R>(sc, 0, kcol0 + 2), pv = scale_of<R>(sc, 0, pcol);
    const int64_t plane = nx * ny, N = plane * nz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % nx, y = (i / nx) % ny, z = i / plane;
        const R f = src[i];
        const R two = f + f;
        R acc = kx * (two - src[x ? i - 1 : i + nx - 1] - src[x + 1 < nx ? i + 1 : i - (nx - 1)]);
        if (ny > 1)
            acc += ky * (two - src[y ? i - nx : i + (ny - 1) * nx] - src[y + 1 < ny ? i + nx : i - (ny - 1) * nx]);
        if (nz > 1)
            acc += kz * (two - src[z ? i - plane : i + (nz - 1) * plane] -
                         src[z + 1 < nz ? i + plane : i - (nz - 1) * plane]);
        dst[i] = dst[i] + acc + pv * V[i] * f;
    }
}

// ---------------------------------------------------------------------------
// Eigenstate accumulation: one windowed Fourier term per step and energy.
// The window weight and the phase factors depend only on the step; the
// block's first threads form them once in FP64 and share them.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_eig_acc(const R* __restrict__ psiR, const R* __restrict__ psiI,
                                                 int64_t npts, EigParams ep) {
    __shared__ double cs[8][2];
    const int64_t m = *ep.count;
    if (m >= ep.M) return;
    if ((int)threadIdx.x < ep.nE) {
        const double t = 2.0 * 3.14159265358979323846 * (double)m / (double)(ep.M - 1);
        const double w = 0.35875 - 0.48829 * cos(t) + 0.14128 * cos(2.0 * t) - 0.01168 * cos(3.0 * t);
        const double ph = ep.E[threadIdx.x] * (double)m * ep.dt_over_hbar;
        cs[threadIdx.x][0] = w * cos(ph);
        cs[threadIdx.x][1] = w * sin(ph);
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = (double)psiR[i], b = (double)psiI[i];
        for (int k = 0; k < ep.nE; ++k) {
            double2* q = reinterpret_cast<double2*>(ep.acc + 2 * ((int64_t)k * npts + i));
            double2 v = *q;
            v.x += cs[k][0] * a - cs[k][1] * b;
            v.y += cs[k][1] * a + cs[k][0] * b;
            *q = v;
        }
    }
}

__global__ void k_count_tick(int64_t* count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *count = *count + 1;
}

// Per-block FP64 partials of sum V (psiR^2 + psiI^2) and of sum psiR^2 + psiI^2.
template <typename R>
__global__ __launch_bounds__(256) void k_energy_pot(const R* __restrict__ a, const R* __restrict__ b,
                                                    const R* __restrict__ V, int64_t n,
                                                    double* __restrict__ pot, double* __restrict__ nrm) {
    double sp = 0.0, sn = 0.0;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double x = (double)a[i], y = (double)b[i];
        const double r2 = x * x + y * y;
        sn += r2;
        sp += (double)V[i] * r2;
    }
    block_sum_store<256>(sp, pot + blockIdx.x);
    __syncthreads();
    block_sum_store<256>(sn, nrm + blockIdx.x);
}

template <typename R>
__global__ void k_axpby(int64_t n, R a, const R* __restrict__ x, R b, R* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

template <typename R>
__global__ void k_xpay(int64_t n, const R* __restrict__ x, R a, const R* __restrict__ y, R* __restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        z[i] = x[i] + a * y[i];
}

template <typename R>
__global__ void k_fill0(int64_t n, R* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (R)0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------


// Waves per block of the hot pass kernels: 4, except 2 for the FP64
// 256-point fused kernels, the boundary sweep and the x passes (256^3 FP64,
// one box: boundary sweep 95.3 us at 4, 91.9 at 2; y/z passes 67.2 at 2,
// 64.5 at 4 once the LDS strides were free of bank conflicts, while with
// conflicting exchanges 2 had been the faster choice there too; 512^2
// FP64 batch: 596 us per step with 4, 692 with 2).
template <typename R, int N>
constexpr int wpb_of() {
    return kWPB;
}
template <typename R, int N>
constexpr int wpb_fused_of() {
    return (sizeof(R) == 8 && N == 256) ? kWPBF64Fused256 : kWPB;
}

// Pass launch with W waves per block; the block size is a runtime choice
// (wpb: 0 for wpb_of, else 2 or 4) made by the batch autotuner.  Rows longer
// than 1024 points run one pencil per block and ignore it.
template <int N, typename F>
static hipError_t with_wpb(int wpb, F&& f) {
    if constexpr (pencil_cfg<N>::WAVE) {
        if (wpb == 2) return f(std::integral_constant<int, 2>{});
        if (wpb == 4) return f(std::integral_constant<int, 4>{});
    }
    return f(std::integral_constant<int, 0>{});
}

template <typename R, int N, int W0>
static hipError_t axis_acc_nw(const R* src, R* dst, const void* tw, const AxisGeom& g, const ScaleRef& sc,
                              int col, int nyq_zero, hipStream_t st) {
    using C = pencil_cfg<N>;
    constexpr int P = tuning<R>::YZ_PPL;
    constexpr int W = W0 ? W0 : wpb_of<R, N>();
    if (g.half_x % P) return hipErrorInvalidValue;
    const int64_t ngroups = g.half_x / P * g.n_outer;
    const int64_t waves = (ngroups + C::PPW - 1) / C::PPW;
    const int64_t blocks = (waves + W - 1) / W;
    hipLaunchKernelGGL((k_axis_acc<R, N, W, P>), dim3((unsigned)blocks), dim3(64 * W), 0, st,
                       src, dst, (const cpx<double>*)tw, g, sc, col, nyq_zero);
    return hipGetLastError();
}

template <typename R, int N>
static hipError_t axis_acc_n(const R* src, R* dst, const void* tw, const AxisGeom& g, const ScaleRef& sc,
                             int col, int nyq_zero, hipStream_t st, int wpb) {
    return with_wpb<N>(wpb, [&](auto w) {
        return axis_acc_nw<R, N, decltype(w)::value>(src, dst, tw, g, sc, col, nyq_zero, st);
    });
}

template <typename R, int N, int W0>
static hipError_t axis_ba_nw(R* psiR, R* psiI, const void* tw, const AxisGeom& g, const ScaleRef& scB,
                             const ScaleRef& scA, int colB, int colA, int nyq_zero, hipStream_t st) {
    using C = pencil_cfg<N>;
    constexpr int P = tuning<R>::BA_PPL;
    constexpr int W = W0 ? W0 : wpb_fused_of<R, N>();
    if (g.half_x % P) return hipErrorInvalidValue;
    const int64_t ngroups = g.half_x / P * g.n_outer;
    const int64_t waves = (ngroups + C::PPW - 1) / C::PPW;
    const int64_t blocks = (waves + W - 1) / W;
    hipLaunchKernelGGL((k_axis_ba<R, N, W, P>), dim3((unsigned)blocks), dim3(64 * W), 0, st, psiR, psiI,
                       (const cpx<double>*)tw, g, scB, scA, colB, colA, nyq_zero);
    return hipGetLastError();
}

template <typename R, int N>
static hipError_t axis_ba_n(R* psiR, R* psiI, const void* tw, const AxisGeom& g, const ScaleRef& scB,
                            const ScaleRef& scA, int colB, int colA, int nyq_zero, hipStream_t st, int wpb) {
    return with_wpb<N>(wpb, [&](auto w) {
        return axis_ba_nw<R, N, decltype(w)::value>(psiR, psiI, tw, g, scB, scA, colB, colA, nyq_zero, st);
    });
}

template <typename R>
hipError_t launch_axis_ba(int64_t n, R* psiR, R* psiI, const void* tw, const AxisGeom& g, const ScaleRef& scB,
                          const ScaleRef& scA, int colB, int colA, int nyq_zero, hipStream_t st, int wpb) {
    switch (n) {
        case 16: return axis_ba_n<R, 16>(psiR, psiI, tw, g, scB, scA, colB, colA, nyq_zero, st, wpb);
        case 32: return axis_ba_n<R, 32>(psiR, psiI, tw, g, scB, scA, colB, colA, nyq_zero, st, wpb);
        case 64: return axis_ba_n<R, 64>(psiR, psiI, tw, g, scB, scA, colB, colA, nyq_zero, st, wpb);
        case 128: return axis_ba_n<R, 128>(psiR, psiI, tw, g, scB, scA, colB, colA, nyq_zero, st, wpb);
        case 256: return axis_ba_n<R, 256>(psiR, psiI, tw, g, scB, scA, colB, colA, nyq_zero, st, wpb);
        case 512: return axis_ba_n<R, 512>(psiR, psiI, tw, g, scB, scA, colB, colA, nyq_zero, st, wpb);
        case 1024: return axis_ba_n<R, 1024>(psiR, psiI, tw, g, scB, scA, colB, colA, nyq_zero, st, wpb);
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_axis_acc(int64_t n, const R* src, R* dst, const void* tw, const AxisGeom& g,
                           const ScaleRef& sc, int col, int nyq_zero, hipStream_t st, int wpb) {
    switch (n) {
        case 16: return axis_acc_n<R, 16>(src, dst, tw, g, sc, col, nyq_zero, st, wpb);
        case 32: return axis_acc_n<R, 32>(src, dst, tw, g, sc, col, nyq_zero, st, wpb);
        case 64: return axis_acc_n<R, 64>(src, dst, tw, g, sc, col, nyq_zero, st, wpb);
        case 128: return axis_acc_n<R, 128>(src, dst, tw, g, sc, col, nyq_zero, st, wpb);
        case 256: return axis_acc_n<R, 256>(src, dst, tw, g, sc, col, nyq_zero, st, wpb);
        case 512: return axis_acc_n<R, 512>(src, dst, tw, g, sc, col, nyq_zero, st, wpb);
        case 1024: return axis_acc_n<R, 1024>(src, dst, tw, g, sc, col, nyq_zero, st, wpb);
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int N, int W0>
static hipError_t x_acc_nw(const R* src, R* dst, const R* V, const void* tw, const RowGeom& g,
                           const ScaleRef& sc, int kcol, int pcol, int nyq_zero, hipStream_t st) {
    constexpr int W = W0 ? W0 : wpb_fused_of<R, N>();
    using M = row_map<R, N, W>;
    const int64_t npen = (g.nrows + 1) / 2;
    const int64_t blocks = (npen + M::PPB - 1) / M::PPB;
    if (g.nrows % (2 * M::PPB) == 0)
        hipLaunchKernelGGL((k_x_acc<R, N, W, true>), dim3((unsigned)blocks), dim3(M::THREADS), 0, st,
                           src, dst, V, (const cpx<double>*)tw, g, sc, kcol, pcol, nyq_zero);
    else
        hipLaunchKernelGGL((k_x_acc<R, N, W, false>), dim3((unsigned)blocks), dim3(M::THREADS), 0, st,
                           src, dst, V, (const cpx<double>*)tw, g, sc, kcol, pcol, nyq_zero);
    return hipGetLastError();
}

template <typename R, int N>
static hipError_t x_acc_n(const R* src, R* dst, const R* V, const void* tw, const RowGeom& g,
                          const ScaleRef& sc, int kcol, int pcol, int nyq_zero, hipStream_t st, int wpb) {
    return with_wpb<N>(wpb, [&](auto w) {
        return x_acc_nw<R, N, decltype(w)::value>(src, dst, V, tw, g, sc, kcol, pcol, nyq_zero, st);
    });
}

template <typename R, int N, int W0>
static hipError_t x_ab_nw(R* psiR, R* psiI, const R* V, const void* tw, const RowGeom& g,
                          const ScaleRef& sc, int nyq_zero, hipStream_t st) {
    constexpr int W = W0 ? W0 : wpb_fused_of<R, N>();
    using M = row_map<R, N, W>;
    const int64_t npen = (g.nrows + 1) / 2;
    const int64_t blocks = (npen + M::PPB - 1) / M::PPB;
    if (g.nrows % (2 * M::PPB) == 0)
        hipLaunchKernelGGL((k_x_ab<R, N, W, true>), dim3((unsigned)blocks), dim3(M::THREADS), 0, st,
                           psiR, psiI, V, (const cpx<double>*)tw, g, sc, nyq_zero);
    else
        hipLaunchKernelGGL((k_x_ab<R, N, W, false>), dim3((unsigned)blocks), dim3(M::THREADS), 0, st,
                           psiR, psiI, V, (const cpx<double>*)tw, g, sc, nyq_zero);
    return hipGetLastError();
}

template <typename R, int N>
static hipError_t x_ab_n(R* psiR, R* psiI, const R* V, const void* tw, const RowGeom& g,
                         const ScaleRef& sc, int nyq_zero, hipStream_t st, int wpb) {
    return with_wpb<N>(wpb, [&](auto w) {
        return x_ab_nw<R, N, decltype(w)::value>(psiR, psiI, V, tw, g, sc, nyq_zero, st);
    });
}

#define SPSTD_ROW_CASES(F, ...)                         \
    switch (nx) {                                       \
        case 16: return F<R, 16>(__VA_ARGS__);          \
        case 32: return F<R, 32>(__VA_ARGS__);          \
        case 64: return F<R, 64>(__VA_ARGS__);          \
        case 128: return F<R, 128>(__VA_ARGS__);        \
        case 256: return F<R, 256>(__VA_ARGS__);        \
        case 512: return F<R, 512>(__VA_ARGS__);        \
        case 1024: return F<R, 1024>(__VA_ARGS__);      \
        case 2048: return F<R, 2048>(__VA_ARGS__);      \
        case 4096: return F<R, 4096>(__VA_ARGS__);      \
        case 8192: return F<R, 8192>(__VA_ARGS__);      \
        case 16384: return F<R, 16384>(__VA_ARGS__);    \
        default: return hipErrorInvalidValue;           \
    }

template <typename R>
hipError_t launch_x_acc(int64_t nx, const R* src, R* dst, const R* V, const void* tw,
                        const RowGeom& g, const ScaleRef& sc, int kcol, int pcol, int nyq_zero,
                        hipStream_t st, int wpb) {
    SPSTD_ROW_CASES(x_acc_n, src, dst, V, tw, g, sc, kcol, pcol, nyq_zero, st, wpb)
}

template <typename R>
hipError_t launch_x_ab(int64_t nx, R* psiR, R* psiI, const R* V, const void* tw,
                       const RowGeom& g, const ScaleRef& sc, int nyq_zero, hipStream_t st, int wpb) {
    SPSTD_ROW_CASES(x_ab_n, psiR, psiI, V, tw, g, sc, nyq_zero, st, wpb)
}

template <typename R>
__global__ void k_probe_batch(const R* __restrict__ psiR, const R* __restrict__ psiI, int64_t npts,
                              const int64_t* __restrict__ idx, int nprobes, const int* __restrict__ active,
                              int ninst, double* __restrict__ probes, int64_t* __restrict__ counter,
                              int64_t capacity, int* __restrict__ fault, int part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst || !active[i]) return;
    const int64_t slot = counter[i];
    if (slot < capacity) {
        double* out = probes + ((int64_t)i * capacity + slot) * nprobes * 2;
        for (int q = 0; q < nprobes; ++q) {
            const int64_t p = idx[(int64_t)i * nprobes + q];
            if (p < 0 || p >= npts) {       // skipped, and flagged for the host
                *fault = 1;
                continue;
            }
            const int64_t k = (int64_t)i * npts + p;
            if (part & PROBE_R) out[2 * q] = (double)psiR[k];
            if (part & PROBE_I) out[2 * q + 1] = (double)psiI[k];
        }
    }
    if (part & PROBE_I) counter[i] = slot + 1;
}

template <typename R>
hipError_t launch_probe_batch(const R* psiR, const R* psiI, int64_t npts, const int64_t* idx, int nprobes,
                              const int* active, int ninst, double* probes, int64_t* counter,
                              int64_t capacity, int* fault, hipStream_t st, int part) {
    if (part < PROBE_R || part > PROBE_FULL) return hipErrorInvalidValue;
    const int blocks = (ninst + 63) / 64;
    hipLaunchKernelGGL((k_probe_batch<R>), dim3(blocks), dim3(64), 0, st, psiR, psiI, npts, idx, nprobes,
                       active, ninst, probes, counter, capacity, fault, part);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_probe(const R* psiR, const R* psiI, const int64_t* idx, int nprobes, int64_t npts,
                        double* out, int64_t* counter, int64_t capacity, int* fault, hipStream_t st) {
    if (nprobes < 0 || nprobes > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_probe<R>), dim3(1), dim3(64), 0, st, psiR, psiI, idx, nprobes, npts, out,
                       counter, capacity, fault);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_norm_partials(const R* psiR, const R* psiI, int64_t n, double* partials,
                                int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((k_norm_partials<R>), dim3(nblocks), dim3(256), 0, st, psiR, psiI, n,
                       partials);
    return hipGetLastError();
}

template <typename R, int N>
static hipError_t energy_axis_n(const R* psiR, const R* psiI, const void* tw, const EnergyGeom& g,
                                int rows, int wall, int nyq_zero, double* partials, int max_blocks,
                                int* nblocks, hipStream_t st) {
    using M = row_map<R, N, kWPB>;
    int64_t b = (g.nlines + M::PPB - 1) / M::PPB;
    if (b > max_blocks) b = max_blocks;
    if (b < 1) b = 1;
    *nblocks = (int)b;
    const R ms = wall == WALL_NEUMANN ? (R)1 : (R)-1;
    const cpx<double>* t = (const cpx<double>*)tw;
#define SPSTD_ENERGY_LAUNCH(ROWS_, WALL_)                                                              \
    hipLaunchKernelGGL((k_energy_axis<R, N, ROWS_, WALL_>), dim3((unsigned)b), dim3(M::THREADS), 0, st, \
                       psiR, psiI, t, g, nyq_zero, ms, partials)
    if (rows) {
        if (wall) SPSTD_ENERGY_LAUNCH(true, true);
        else SPSTD_ENERGY_LAUNCH(true, false);
    } else if constexpr (pencil_cfg<N>::WAVE) {
        if (wall) SPSTD_ENERGY_LAUNCH(false, true);
        else SPSTD_ENERGY_LAUNCH(false, false);
    } else {
        return hipErrorInvalidValue;   // y/z lines are at most 1024 long
    }
#undef SPSTD_ENERGY_LAUNCH
    return hipGetLastError();
}

template <typename R>
hipError_t launch_energy_axis(int64_t n, int rows, int wall, const R* psiR, const R* psiI,
                              const void* tw, const EnergyGeom& g, int nyq_zero, double* partials,
                              int max_blocks, int* nblocks, hipStream_t st) {
    if (wall && wall_dft_len_ok(n)) {
        int64_t b = g.nlines < max_blocks ? g.nlines : max_blocks;
        if (b < 1) b = 1;
        *nblocks = (int)b;
        const R ms = wall == WALL_NEUMANN ? (R)1 : (R)-1;
        hipLaunchKernelGGL((k_wall_dft_energy<R>), dim3((unsigned)b), dim3(64), 0, st, psiR, psiI,
                           (const cpx<double>*)tw, (int)n, g, nyq_zero, ms, partials);
        return hipGetLastError();
    }
    const int64_t nx = wall ? 2 * n : n;
    SPSTD_ROW_CASES(energy_axis_n, psiR, psiI, tw, g, rows, wall, nyq_zero, partials, max_blocks, nblocks, st)
}

template <typename R, int N>
static hipError_t wall_acc_n(const R* src, R* dst, const R* V, const void* tw, const EnergyGeom& g,
                             int64_t npts, const ScaleRef& sc, int kcol, int pcol, int rows, int wall,
                             int nyq_zero, hipStream_t st) {
    using M = row_map<R, N, kWPB>;
    const int64_t npen = (g.nlines + 1) / 2;
    const int64_t b = (npen + M::PPB - 1) / M::PPB;
    const R ms = wall == WALL_NEUMANN ? (R)1 : (R)-1;
    if (rows)
        hipLaunchKernelGGL((k_wall_acc<R, N, true>), dim3((unsigned)b), dim3(M::THREADS), 0, st, src, dst, V,
                           (const cpx<double>*)tw, g, npts, sc, kcol, pcol, nyq_zero, ms);
    else if constexpr (pencil_cfg<N>::WAVE)
        hipLaunchKernelGGL((k_wall_acc<R, N, false>), dim3((unsigned)b), dim3(M::THREADS), 0, st, src, dst, V,
                           (const cpx<double>*)tw, g, npts, sc, kcol, pcol, nyq_zero, ms);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename R>
hipError_t launch_wall_acc(int64_t n, int rows, int wall, const R* src, R* dst, const R* V,
                           const void* tw, const EnergyGeom& g, int64_t npts, const ScaleRef& sc,
                           int kcol, int pcol, int nyq_zero, hipStream_t st) {
    if (wall != WALL_DIRICHLET && wall != WALL_NEUMANN) return hipErrorInvalidValue;
    if (wall_dft_len_ok(n)) {
        const int64_t b = (g.nlines + 1) / 2;
        const R ms = wall == WALL_NEUMANN ? (R)1 : (R)-1;
        hipLaunchKernelGGL((k_wall_dft_acc<R>), dim3((unsigned)b), dim3(64), 0, st, src, dst, V,
                           (const cpx<double>*)tw, (int)n, g, npts, sc, kcol, pcol, nyq_zero, ms);
        return hipGetLastError();
    }
    const int64_t nx = 2 * n;
    switch (nx) {
        case 32: return wall_acc_n<R, 32>(src, dst, V, tw, g, npts, sc, kcol, pcol, rows, wall, nyq_zero, st);
        case 64: return wall_acc_n<R, 64>(src, dst, V, tw, g, npts, sc, kcol, pcol, rows, wall, nyq_zero, st);
        case 128: return wall_acc_n<R, 128>(src, dst, V, tw, g, npts, sc, kcol, pcol, rows, wall, nyq_zero, st);
        case 256: return wall_acc_n<R, 256>(src, dst, V, tw, g, npts, sc, kcol, pcol, rows, wall, nyq_zero, st);
        case 512: return wall_acc_n<R, 512>(src, dst, V, tw, g, npts, sc, kcol, pcol, rows, wall, nyq_zero, st);
        case 1024: return wall_acc_n<R, 1024>(src, dst, V, tw, g, npts, sc, kcol, pcol, rows, wall, nyq_zero, st);
        case 2048: return wall_acc_n<R, 2048>(src, dst, V, tw, g, npts, sc, kcol, pcol, rows, wall, nyq_zero, st);
        case 4096: return wall_acc_n<R, 4096>(src, dst, V, tw, g, npts, sc, kcol, pcol, rows, wall, nyq_zero, st);
        case 8192: return wall_acc_n<R, 8192>(src, dst, V, tw, g, npts, sc, kcol, pcol, rows, wall, nyq_zero, st);
        case 16384: return wall_acc_n<R, 16384>(src, dst, V, tw, g, npts, sc, kcol, pcol, rows, wall, nyq_zero, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_energy_pot(const R* psiR, const R* psiI, const R* V, int64_t n, double* pot,
                             double* nrm, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((k_energy_pot<R>), dim3(nblocks), dim3(256), 0, st, psiR, psiI, V, n, pot, nrm);
    return hipGetLastError();
}

static unsigned ew_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

template <typename R>
hipError_t launch_fd_acc(const R* src, R* dst, const R* V, const int64_t* n, const ScaleRef& sc, int kcol0,
                         int pcol, hipStream_t st) {
    hipLaunchKernelGGL((k_fd_acc<R>), dim3(ew_blocks(n[0] * n[1] * n[2])), dim3(256), 0, st, src, dst, V, n[0],
                       n[1], n[2], sc, kcol0, pcol);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_eig_acc(const R* psiR, const R* psiI, int64_t npts, const EigParams& ep, hipStream_t st) {
    hipLaunchKernelGGL((k_eig_acc<R>), dim3(ew_blocks(npts)), dim3(256), 0, st, psiR, psiI, npts, ep);
    return hipGetLastError();
}

hipError_t launch_count_tick(int64_t* count, hipStream_t st) {
    hipLaunchKernelGGL(k_count_tick, dim3(1), dim3(64), 0, st, count);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_axpby(int64_t n, double a, const R* x, double b, R* y, hipStream_t st) {
    hipLaunchKernelGGL((k_axpby<R>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (R)a, x, (R)b, y);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_xpay(int64_t n, const R* x, double a, const R* y, R* z, hipStream_t st) {
    hipLaunchKernelGGL((k_xpay<R>), dim3(ew_blocks(n)), dim3(256), 0, st, n, x, (R)a, y, z);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fill0(int64_t n, R* y, hipStream_t st) {
    hipLaunchKernelGGL((k_fill0<R>), dim3(ew_blocks(n)), dim3(256), 0, st, n, y);
    return hipGetLastError();
}

#define SPSTD_INSTANTIATE(R)                                                                    \
    template hipError_t launch_axis_acc<R>(int64_t, const R*, R*, const void*, const AxisGeom&, \
                                           const ScaleRef&, int, int, hipStream_t, int);        \
    template hipError_t launch_axis_ba<R>(int64_t, R*, R*, const void*, const AxisGeom&,        \
                                          const ScaleRef&, const ScaleRef&, int, int, int,      \
                                          hipStream_t, int);                                    \
    template hipError_t launch_x_acc<R>(int64_t, const R*, R*, const R*, const void*,           \
                                        const RowGeom&, const ScaleRef&, int, int, int,         \
                                        hipStream_t, int);                                      \
    template hipError_t launch_x_ab<R>(int64_t, R*, R*, const R*, const void*, const RowGeom&,  \
                                       const ScaleRef&, int, hipStream_t, int);                 \
    template hipError_t launch_probe_batch<R>(const R*, const R*, int64_t, const int64_t*, int, \
                                              const int*, int, double*, int64_t*, int64_t,      \
                                              int*, hipStream_t, int);                          \
    template hipError_t launch_probe<R>(const R*, const R*, const int64_t*, int, int64_t,       \
                                        double*, int64_t*, int64_t, int*, hipStream_t);         \
    template hipError_t launch_norm_partials<R>(const R*, const R*, int64_t, double*, int,      \
                                                hipStream_t);                                   \
    template hipError_t launch_axpby<R>(int64_t, double, const R*, double, R*, hipStream_t);    \
    template hipError_t launch_xpay<R>(int64_t, const R*, double, const R*, R*, hipStream_t);   \
    template hipError_t launch_fill0<R>(int64_t, R*, hipStream_t);                             \
    template hipError_t launch_eig_acc<R>(const R*, const R*, int64_t, const EigParams&, hipStream_t); \
    template hipError_t launch_fd_acc<R>(const R*, R*, const R*, const int64_t*, const ScaleRef&, \
                                         int, int, hipStream_t);                                \
    template hipError_t launch_energy_axis<R>(int64_t, int, int, const R*, const R*, const void*, \
                                              const EnergyGeom&, int, double*, int, int*,       \
                                              hipStream_t);                                     \
    template hipError_t launch_wall_acc<R>(int64_t, int, int, const R*, R*, const R*, const void*, \
                                           const EnergyGeom&, int64_t, const ScaleRef&, int, int, \
                                           int, hipStream_t);                                   \
    template hipError_t launch_energy_pot<R>(const R*, const R*, const R*, int64_t, double*,    \
                                             double*, int, hipStream_t);

SPSTD_INSTANTIATE(double)
SPSTD_INSTANTIATE(float)
template hipError_t launch_fill0<int64_t>(int64_t, int64_t*, hipStream_t);
template hipError_t launch_fill0<int>(int64_t, int*, hipStream_t);

}  // namespace spstd
