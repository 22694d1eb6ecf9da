// SPSTD device kernels for gfx950 (MI355X).
//
// The kinetic part of K (Eq. 16) is a sum over axes, so the paper's update
// (Eq. 18) applies one 1D spectral second derivative per axis (as Eq. 11-12
// write it).  Each kernel here is one such directional pass over the whole
// field: it loads pencils along its axis, runs the forward FFT, multiplies by
// the real, even symbol coef*(hbar/2m*)*k^2/N, runs the inverse FFT, and adds
// the result into the destination field.  Because the symbol is real and
// even, the operator maps real fields to real fields, so two real pencils are
// carried as one complex pencil (real and imaginary parts) at no extra cost.
//
// Passes of one stage l (Eq. 17-18, A(c_l) before B(d_l)):
//   y: psi_R += c_l dt T_y psi_I          z: psi_R += c_l dt T_z psi_I
//   x: psi_R += c_l dt (T_x psi_I + V psi_I / hbar), then on the same rows
//      psi_I -= d_l dt (T_x psi_R + V psi_R / hbar)       (fused A and B)
//   y: psi_I -= d_l dt T_y psi_R          z: psi_I -= d_l dt T_z psi_R
#include "fft_core.hpp"
#include "kernels.hpp"

namespace spstd {

bool axis_len_ok(int64_t n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }
bool row_len_ok(int64_t n) { return n >= 16 && n <= 16384 && (n & (n - 1)) == 0; }

// Multiply bins kk = j + T*e by scale * ks^2 (ks the signed bin index);
// under the ZERO convention the Nyquist bin kk = N/2 is removed.
template <typename R, int N>
__device__ __forceinline__ void apply_symbol(cpx<R> (&v)[16], int j, R scale, int nyq_zero) {
    constexpr int T = N / 16;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int kk = j + T * e;
        const int ks = (kk <= N / 2) ? kk : kk - N;
        R s = scale * (R)(ks * ks);
        if (nyq_zero && kk == N / 2) s = (R)0;
        v[e].x *= s;
        v[e].y *= s;
    }
}

// Lanes per pencil T = N/16; pencils per wave for N <= 1024.
template <int N>
struct pencil_cfg {
    static constexpr int T = N / 16;
    static constexpr bool WAVE = T <= 64;
    static constexpr int PPW = WAVE ? 64 / T : 1;
};

// ---------------------------------------------------------------------------
// y / z pass: dst += T_axis src.  Lane l of a wave: pencil p = l % PPW (the
// fast index, so neighbouring lanes read neighbouring x pairs), position
// j = l / PPW.
// ---------------------------------------------------------------------------
template <typename R, int N, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_axis_acc(const R* __restrict__ src, R* __restrict__ dst,
                                                       const cpx<R>* __restrict__ tw, AxisGeom g,
                                                       R scale, int nyq_zero) {
    using C = pencil_cfg<N>;
    static_assert(C::WAVE, "y/z pencils must fit in one wavefront");
    constexpr int LS = lds_size<N>::value;
    __shared__ R lds[N == 16 ? 1 : WPB * C::PPW * 2 * LS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane % C::PPW, j = lane / C::PPW;
    const int64_t npen = g.half_x * g.n_outer;
    const int64_t pencil = ((int64_t)blockIdx.x * WPB + wave) * C::PPW + p;
    const bool valid = pencil < npen;
    const int64_t px = valid ? pencil % g.half_x : 0, outer = valid ? pencil / g.half_x : 0;
    const int64_t base = outer * g.outer_stride + 2 * px;

    cpx<R> v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        v[e] = valid ? *reinterpret_cast<const cpx<R>*>(src + base + (int64_t)(j + C::T * e) * g.stride)
                     : cpx<R>{(R)0, (R)0};
    }
    R* lre = lds + (wave * C::PPW + p) * 2 * LS;
    fft_pencil<R, N, false, true>(v, j, lre, lre + LS, tw);
    apply_symbol<R, N>(v, j, scale, nyq_zero);
    fft_pencil<R, N, true, true>(v, j, lre, lre + LS, tw);
    if (valid) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            cpx<R>* q = reinterpret_cast<cpx<R>*>(dst + base + (int64_t)(j + C::T * e) * g.stride);
            cpx<R> o = *q;
            *q = cpx<R>{o.x + v[e].x, o.y + v[e].y};
        }
    }
}

// ---------------------------------------------------------------------------
// x pass helpers: lane l -> position j = l % T, pencil-in-wave p = l / T
// (neighbouring lanes read neighbouring x), or one pencil per block for
// N > 1024.
// ---------------------------------------------------------------------------
template <int N, int WPB>
struct row_map {
    using C = pencil_cfg<N>;
    static constexpr int PPB = C::WAVE ? WPB * C::PPW : 1;   // pencils per block
    static constexpr int THREADS = C::WAVE ? 64 * WPB : C::T;
    static constexpr int LS = lds_size<N>::value;
    // large pencils exchange re and im in turn to stay within 160 KB of LDS
    static constexpr bool SPLIT = !C::WAVE;
    // a 16-point pencil is one radix-16 pass in registers: no LDS at all
    static constexpr int LDS_REALS = N == 16 ? 1 : PPB * (SPLIT ? 1 : 2) * LS;
};

template <typename R, int N, int WPB>
__device__ __forceinline__ void row_coords(int& j, int& pin_block, int64_t& q) {
    using C = pencil_cfg<N>;
    if constexpr (C::WAVE) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        j = lane % C::T;
        pin_block = wave * C::PPW + lane / C::T;
    } else {
        j = threadIdx.x;
        pin_block = 0;
    }
    q = (int64_t)blockIdx.x * row_map<N, WPB>::PPB + pin_block;
}

template <typename R, int N, int WPB>
__global__ __launch_bounds__((row_map<N, WPB>::THREADS)) void k_x_acc(
    const R* __restrict__ src, R* __restrict__ dst, const R* __restrict__ V,
    const cpx<R>* __restrict__ tw, int64_t nrows, R scale, R vscale, int nyq_zero) {
    using C = pencil_cfg<N>;
    using M = row_map<N, WPB>;
    __shared__ R lds[M::LDS_REALS];
    int j, pb;
    int64_t q;
    row_coords<R, N, WPB>(j, pb, q);
    const int64_t r0 = 2 * q, r1 = 2 * q + 1;
    const bool v0 = r0 < nrows, v1 = r1 < nrows;
    const R* s0 = src + r0 * N;
    const R* s1 = src + r1 * N;
    cpx<R> v[16];
    R f0[16], f1[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int x = j + C::T * e;
        f0[e] = v0 ? s0[x] : (R)0;
        f1[e] = v1 ? s1[x] : (R)0;
        v[e] = cpx<R>{f0[e], f1[e]};
    }
    R* lre = lds + pb * (M::SPLIT ? 1 : 2) * M::LS;
    fft_pencil<R, N, false, C::WAVE, M::SPLIT>(v, j, lre, lre + M::LS, tw);
    apply_symbol<R, N>(v, j, scale, nyq_zero);
    fft_pencil<R, N, true, C::WAVE, M::SPLIT>(v, j, lre, lre + M::LS, tw);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int x = j + C::T * e;
        if (v0) {
            const int64_t a = r0 * N + x;
            dst[a] = dst[a] + v[e].x + vscale * V[a] * f0[e];
        }
        if (v1) {
            const int64_t a = r1 * N + x;
            dst[a] = dst[a] + v[e].y + vscale * V[a] * f1[e];
        }
    }
}

template <typename R, int N, int WPB>
__global__ __launch_bounds__((row_map<N, WPB>::THREADS)) void k_x_ab(
    R* __restrict__ psiR, R* __restrict__ psiI, const R* __restrict__ V,
    const cpx<R>* __restrict__ tw, int64_t nrows, R sa, R va, R sb, R vb, int nyq_zero) {
    using C = pencil_cfg<N>;
    using M = row_map<N, WPB>;
    __shared__ R lds[M::LDS_REALS];
    int j, pb;
    int64_t q;
    row_coords<R, N, WPB>(j, pb, q);
    const int64_t r0 = 2 * q, r1 = 2 * q + 1;
    const bool v0 = r0 < nrows, v1 = r1 < nrows;
    cpx<R> v[16];
    cpx<R> f[16];   // psi_I on entry; later psi_I + vb * V * psi_R(new)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int x = j + C::T * e;
        f[e].x = v0 ? psiI[r0 * N + x] : (R)0;
        f[e].y = v1 ? psiI[r1 * N + x] : (R)0;
        v[e] = f[e];
    }
    R* lre = lds + pb * (M::SPLIT ? 1 : 2) * M::LS;
    // A half: psi_R += T_x^a psi_I + va V psi_I
    fft_pencil<R, N, false, C::WAVE, M::SPLIT>(v, j, lre, lre + M::LS, tw);
    apply_symbol<R, N>(v, j, sa, nyq_zero);
    fft_pencil<R, N, true, C::WAVE, M::SPLIT>(v, j, lre, lre + M::LS, tw);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int x = j + C::T * e;
        cpx<R> vv = {(R)0, (R)0}, g = {(R)0, (R)0};
        if (v0) { vv.x = V[r0 * N + x]; g.x = psiR[r0 * N + x]; }
        if (v1) { vv.y = V[r1 * N + x]; g.y = psiR[r1 * N + x]; }
        g.x = g.x + v[e].x + va * vv.x * f[e].x;
        g.y = g.y + v[e].y + va * vv.y * f[e].y;
        if (v0) psiR[r0 * N + x] = g.x;
        if (v1) psiR[r1 * N + x] = g.y;
        v[e] = g;
        f[e].x = f[e].x + vb * vv.x * g.x;
        f[e].y = f[e].y + vb * vv.y * g.y;
    }
    // B half: psi_I += T_x^b psi_R(new) + vb V psi_R(new)
    fft_pencil<R, N, false, C::WAVE, M::SPLIT>(v, j, lre, lre + M::LS, tw);
    apply_symbol<R, N>(v, j, sb, nyq_zero);
    fft_pencil<R, N, true, C::WAVE, M::SPLIT>(v, j, lre, lre + M::LS, tw);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int x = j + C::T * e;
        if (v0) psiI[r0 * N + x] = f[e].x + v[e].x;
        if (v1) psiI[r1 * N + x] = f[e].y + v[e].y;
    }
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_probe(const R* __restrict__ psiR, const R* __restrict__ psiI,
                        const int64_t* __restrict__ idx, int nprobes, double* __restrict__ out,
                        int64_t* __restrict__ counter, int64_t capacity) {
    const int64_t slot = *counter;
    const int t = threadIdx.x;
    if (slot < capacity && t < nprobes) {
        const int64_t i = idx[t];
        out[(slot * nprobes + t) * 2 + 0] = (double)psiR[i];
        out[(slot * nprobes + t) * 2 + 1] = (double)psiI[i];
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
constexpr int kWPB = 2;   // waves per block of the wave-local passes

template <typename R, int N>
static hipError_t axis_acc_n(const R* src, R* dst, const void* tw, const AxisGeom& g, double scale,
                             int nyq_zero, hipStream_t st) {
    using C = pencil_cfg<N>;
    const int64_t npen = g.half_x * g.n_outer;
    const int64_t waves = (npen + C::PPW - 1) / C::PPW;
    const int64_t blocks = (waves + kWPB - 1) / kWPB;
    hipLaunchKernelGGL((k_axis_acc<R, N, kWPB>), dim3((unsigned)blocks), dim3(64 * kWPB), 0, st,
                       src, dst, (const cpx<R>*)tw, g, (R)scale, nyq_zero);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_axis_acc(int64_t n, const R* src, R* dst, const void* tw, const AxisGeom& g,
                           double scale, int nyq_zero, hipStream_t st) {
    switch (n) {
        case 16: return axis_acc_n<R, 16>(src, dst, tw, g, scale, nyq_zero, st);
        case 32: return axis_acc_n<R, 32>(src, dst, tw, g, scale, nyq_zero, st);
        case 64: return axis_acc_n<R, 64>(src, dst, tw, g, scale, nyq_zero, st);
        case 128: return axis_acc_n<R, 128>(src, dst, tw, g, scale, nyq_zero, st);
        case 256: return axis_acc_n<R, 256>(src, dst, tw, g, scale, nyq_zero, st);
        case 512: return axis_acc_n<R, 512>(src, dst, tw, g, scale, nyq_zero, st);
        case 1024: return axis_acc_n<R, 1024>(src, dst, tw, g, scale, nyq_zero, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int N>
static hipError_t x_acc_n(const R* src, R* dst, const R* V, const void* tw, const RowGeom& g,
                          double scale, double vscale, int nyq_zero, hipStream_t st) {
    using M = row_map<N, kWPB>;
    const int64_t npen = (g.nrows + 1) / 2;
    const int64_t blocks = (npen + M::PPB - 1) / M::PPB;
    hipLaunchKernelGGL((k_x_acc<R, N, kWPB>), dim3((unsigned)blocks), dim3(M::THREADS), 0, st,
                       src, dst, V, (const cpx<R>*)tw, g.nrows, (R)scale, (R)vscale, nyq_zero);
    return hipGetLastError();
}

template <typename R, int N>
static hipError_t x_ab_n(R* psiR, R* psiI, const R* V, const void* tw, const RowGeom& g, double sa,
                         double va, double sb, double vb, int nyq_zero, hipStream_t st) {
    using M = row_map<N, kWPB>;
    const int64_t npen = (g.nrows + 1) / 2;
    const int64_t blocks = (npen + M::PPB - 1) / M::PPB;
    hipLaunchKernelGGL((k_x_ab<R, N, kWPB>), dim3((unsigned)blocks), dim3(M::THREADS), 0, st,
                       psiR, psiI, V, (const cpx<R>*)tw, g.nrows, (R)sa, (R)va, (R)sb, (R)vb,
                       nyq_zero);
    return hipGetLastError();
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
                        const RowGeom& g, double scale, double vscale, int nyq_zero,
                        hipStream_t st) {
    SPSTD_ROW_CASES(x_acc_n, src, dst, V, tw, g, scale, vscale, nyq_zero, st)
}

template <typename R>
hipError_t launch_x_ab(int64_t nx, R* psiR, R* psiI, const R* V, const void* tw,
                       const RowGeom& g, double sa, double va, double sb, double vb,
                       int nyq_zero, hipStream_t st) {
    SPSTD_ROW_CASES(x_ab_n, psiR, psiI, V, tw, g, sa, va, sb, vb, nyq_zero, st)
}

template <typename R>
hipError_t launch_probe(const R* psiR, const R* psiI, const int64_t* idx, int nprobes,
                        double* out, int64_t* counter, int64_t capacity, hipStream_t st) {
    hipLaunchKernelGGL((k_probe<R>), dim3(1), dim3(64), 0, st, psiR, psiI, idx, nprobes, out,
                       counter, capacity);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_norm_partials(const R* psiR, const R* psiI, int64_t n, double* partials,
                                int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((k_norm_partials<R>), dim3(nblocks), dim3(256), 0, st, psiR, psiI, n,
                       partials);
    return hipGetLastError();
}

static unsigned ew_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
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
                                           double, int, hipStream_t);                          \
    template hipError_t launch_x_acc<R>(int64_t, const R*, R*, const R*, const void*,           \
                                        const RowGeom&, double, double, int, hipStream_t);      \
    template hipError_t launch_x_ab<R>(int64_t, R*, R*, const R*, const void*, const RowGeom&,  \
                                       double, double, double, double, int, hipStream_t);       \
    template hipError_t launch_probe<R>(const R*, const R*, const int64_t*, int, double*,       \
                                        int64_t*, int64_t, hipStream_t);                        \
    template hipError_t launch_norm_partials<R>(const R*, const R*, int64_t, double*, int,      \
                                                hipStream_t);                                   \
    template hipError_t launch_axpby<R>(int64_t, double, const R*, double, R*, hipStream_t);    \
    template hipError_t launch_xpay<R>(int64_t, const R*, double, const R*, R*, hipStream_t);   \
    template hipError_t launch_fill0<R>(int64_t, R*, hipStream_t);

SPSTD_INSTANTIATE(double)
SPSTD_INSTANTIATE(float)

}  // namespace spstd
