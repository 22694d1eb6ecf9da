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
#include <type_traits>

#include "fft_core.hpp"
#include "kernels.hpp"

namespace spstd {

bool axis_len_ok(int64_t n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }
bool row_len_ok(int64_t n) { return n >= 16 && n <= 16384 && (n & (n - 1)) == 0; }

// Build-time tuning switches (defaults are the measured choices):
//   TW_PRODUCTS_*  twiddles of a pass from two table reads and FP64 products
//                  instead of one table read per twiddle (FP32 256^3 graph
//                  step 1.58 -> 1.44 ms, FP32 512^2 batch 428 -> 319 us)
//   SPLIT_*        real-then-imaginary LDS exchange (half the LDS per wave);
//                  the fused FP32 x pass takes the joint exchange below
//                  SPLIT_XAB_F32_FROM points per row, the other FP32 passes
//                  gain occupancy from the split one
//   WPB, WPB_F64_256  waves per block of the pass kernels (wpb_of)
//   BA_RELOAD_*    the stage-boundary y sweep re-reads psi_R for its second
//                  epilogue instead of keeping it in registers (measured
//                  slower: 106 -> 121 us FP64, 65 -> 68 us FP32 at 256^3)
//   YZ_PPL_F64, YZ_MIN_WAVES, YZ_NT  y/z pass variants measured slower
//                  (two pencils per FP64 lane group, a forced 4 waves per
//                  SIMD, non-temporal loads and stores)
//   X_RELOAD, X_RELOAD_FROM  x passes re-read their inputs in the epilogue
//                  instead of keeping them in registers through the
//                  transforms, for all lengths or from X_RELOAD_FROM points
//                  (16384: FP32 batch of 33 such rows 196 -> 178 us per
//                  step; 8192 slower, 84 -> 93 us)
//   MIN_WAVES      minimum waves per SIMD requested for the pass kernels (2
//                  keeps the FP64 x passes of 512..2048-point rows out of
//                  accumulation registers, at one wave per SIMD otherwise)
//   YZ_PPL_F32     complex pencils per lane group in FP32 y/z passes
//   EPI_CHUNK      epilogue elements scheduled together (caps the loads in
//                  flight, and with them the registers)
//   YZ_ACC_WAVES_*, YZ_BA_WAVES_F32, X_AB_WAVES_F32  minimum waves per SIMD of
//                  the 256-point passes (yz_acc_waves and its kin).  Taken:
//                  4 for the FP32 y/z pass.  Measured slower: 4 for the FP64
//                  y/z pass (spills; z 70.5 -> 103 us), 3 or 4 for the FP32
//                  boundary sweep (spills), 4 for the FP32 fused x pass
//                  (54.7 -> 55.4 us); fewer FP64 y/z blocks per CU (4 or 2,
//                  by unused dynamic LDS) slower too (z 70.5 -> 75.9, 99 us)
//   BA_PPL_F32, BA_PPL_F32_LONG  complex pencils per lane group in the FP32
//                  stage-boundary sweep up to 256 and from 512 points: one
//                  (142 registers, three waves per SIMD) against two (248,
//                  two waves) at 256: 256^3 sweep 59.1 -> 55.0 us; two at
//                  512 (a 512^2 batch of 49: 316 against 352 us per step).
//                  Reading psi_I together with psi_R at the start instead
//                  of after the first transform pair was slower in both
//                  precisions (FP32 58.9, with psi_R re-read and four waves
//                  62.2; FP64 98.2 -> 124.4 us with psi_R re-read)
//   YZ_EPI_BATCH_* y/z pass epilogues read YZ_CHUNK elements of the
//                  accumulated field before writing any of them (element by
//                  element, each read waits for the previous write: the
//                  compiler cannot prove that the elements of one pencil are
//                  distinct).  FP32 256^3: z 41.8 -> 41.3 us, boundary sweep
//                  59.5 -> 58.1 us; FP64 slower (z 71.0 -> 73.3 us, sweep
//                  98.6 -> 102.4 us); 8 or 16 reads at once slower in both
//   EPI_FENCE      keep epilogue loads from being hoisted into the inverse
//                  transform
//   YZ_ORDER       0: consecutive blocks take neighbouring x column groups of
//                  one (z or y) plane; 1: consecutive blocks take the same
//                  column groups of neighbouring planes (spreads the
//                  concurrently running blocks over more memory channels)
#ifndef SPSTD_TW_PRODUCTS_F64
#define SPSTD_TW_PRODUCTS_F64 1
#endif
#ifndef SPSTD_TW_PRODUCTS_F32
#define SPSTD_TW_PRODUCTS_F32 1
#endif
#ifndef SPSTD_SPLIT_F64
#define SPSTD_SPLIT_F64 1
#endif
#ifndef SPSTD_SPLIT_F32
#define SPSTD_SPLIT_F32 1
#endif
#ifndef SPSTD_SPLIT_XAB_F32
#define SPSTD_SPLIT_XAB_F32 0
#endif
#ifndef SPSTD_X_RELOAD_FROM
#define SPSTD_X_RELOAD_FROM 16384
#endif
#ifndef SPSTD_X_RELOAD
#define SPSTD_X_RELOAD 0
#endif
#ifndef SPSTD_MIN_WAVES
#define SPSTD_MIN_WAVES 2
#endif
#ifndef SPSTD_YZ_PPL_F32
#define SPSTD_YZ_PPL_F32 2
#endif
#ifndef SPSTD_YZ_PPL_F64
#define SPSTD_YZ_PPL_F64 1
#endif
#ifndef SPSTD_YZ_MIN_WAVES
#define SPSTD_YZ_MIN_WAVES 0
#endif
#ifndef SPSTD_YZ_NT
#define SPSTD_YZ_NT 0
#endif
#ifndef SPSTD_BA_RELOAD_F64
#define SPSTD_BA_RELOAD_F64 0
#endif
#ifndef SPSTD_BA_RELOAD_F32
#define SPSTD_BA_RELOAD_F32 0
#endif
#ifndef SPSTD_V_NT_F64
#define SPSTD_V_NT_F64 1
#endif
#ifndef SPSTD_V_NT_F32
#define SPSTD_V_NT_F32 0
#endif
#ifndef SPSTD_WPB
#define SPSTD_WPB 4
#endif
#ifndef SPSTD_WPB_F64_256
#define SPSTD_WPB_F64_256 2
#endif
#ifndef SPSTD_SPLIT_XAB_F32_FROM
#define SPSTD_SPLIT_XAB_F32_FROM 512
#endif
#ifndef SPSTD_EPI_CHUNK
#define SPSTD_EPI_CHUNK 4
#endif
#ifndef SPSTD_YZ_ACC_WAVES_F32
#define SPSTD_YZ_ACC_WAVES_F32 4
#endif
#ifndef SPSTD_YZ_ACC_WAVES_F64
#define SPSTD_YZ_ACC_WAVES_F64 0
#endif
#ifndef SPSTD_YZ_BA_WAVES_F32
#define SPSTD_YZ_BA_WAVES_F32 0
#endif
#ifndef SPSTD_X_AB_WAVES_F32
#define SPSTD_X_AB_WAVES_F32 0
#endif
#ifndef SPSTD_BA_PPL_F32
#define SPSTD_BA_PPL_F32 1
#endif
#ifndef SPSTD_BA_PPL_F32_LONG
#define SPSTD_BA_PPL_F32_LONG 2
#endif
#ifndef SPSTD_YZ_EPI_BATCH_F64
#define SPSTD_YZ_EPI_BATCH_F64 0
#endif
#ifndef SPSTD_YZ_EPI_BATCH_F32
#define SPSTD_YZ_EPI_BATCH_F32 1
#endif
#ifndef SPSTD_YZ_CHUNK
#define SPSTD_YZ_CHUNK 4
#endif
#ifndef SPSTD_EPI_FENCE
#define SPSTD_EPI_FENCE 1
#endif
#ifndef SPSTD_YZ_ORDER
#define SPSTD_YZ_ORDER 1
#endif

#if SPSTD_MIN_WAVES > 0
#define SPSTD_WAVES_ATTR __attribute__((amdgpu_waves_per_eu(SPSTD_MIN_WAVES)))
#else
#define SPSTD_WAVES_ATTR
#endif

template <typename R>
struct tuning;
template <>
struct tuning<double> {
    static constexpr bool PRODUCTS = SPSTD_TW_PRODUCTS_F64;
    static constexpr bool SPLIT = SPSTD_SPLIT_F64;
    static constexpr bool SPLIT_XAB = SPSTD_SPLIT_F64;
    static constexpr int YZ_PPL = SPSTD_YZ_PPL_F64;
    static constexpr bool BA_RELOAD = SPSTD_BA_RELOAD_F64;
    static constexpr bool V_NT = SPSTD_V_NT_F64;
    static constexpr bool EPI_BATCH = SPSTD_YZ_EPI_BATCH_F64;
    static constexpr int BA_PPL = 1;
};
template <>
struct tuning<float> {
    static constexpr bool PRODUCTS = SPSTD_TW_PRODUCTS_F32;
    static constexpr bool SPLIT = SPSTD_SPLIT_F32;
    static constexpr bool SPLIT_XAB = SPSTD_SPLIT_XAB_F32;
    static constexpr int YZ_PPL = SPSTD_YZ_PPL_F32;
    static constexpr bool BA_RELOAD = SPSTD_BA_RELOAD_F32;
    static constexpr bool V_NT = SPSTD_V_NT_F32;
    static constexpr bool EPI_BATCH = SPSTD_YZ_EPI_BATCH_F32;
    static constexpr int BA_PPL = SPSTD_BA_PPL_F32;
};

// Minimum waves per SIMD requested for the 256-point pass kernels (a value
// of 0 leaves the general setting).  A 256^3 FP32 y/z pass is 16 waves per
// CU: at 137 registers three waves per SIMD fit, which leaves a second round
// a third full; capped at 128 registers all 16 run at once (z 41.4 -> 35.6
// us).
template <typename R, int N>
constexpr int yz_acc_waves() {
    const int k = N != 256 ? 0 : sizeof(R) == 4 ? SPSTD_YZ_ACC_WAVES_F32 : SPSTD_YZ_ACC_WAVES_F64;
    return k > 0 ? k : SPSTD_YZ_MIN_WAVES > 0 ? SPSTD_YZ_MIN_WAVES : SPSTD_MIN_WAVES > 0 ? SPSTD_MIN_WAVES : 1;
}
template <typename R, int N>
constexpr int yz_ba_waves() {
    const int k = N != 256 ? 0 : sizeof(R) == 4 ? SPSTD_YZ_BA_WAVES_F32 : 0;
    return k > 0 ? k : SPSTD_YZ_MIN_WAVES > 0 ? SPSTD_YZ_MIN_WAVES : SPSTD_MIN_WAVES > 0 ? SPSTD_MIN_WAVES : 1;
}
template <typename R, int N>
constexpr int x_ab_waves() {
    const int k = N != 256 ? 0 : sizeof(R) == 4 ? SPSTD_X_AB_WAVES_F32 : 0;
    return k > 0 ? k : SPSTD_MIN_WAVES > 0 ? SPSTD_MIN_WAVES : 1;
}

// The potential is read once per x pass.  In FP64 the three fields of a
// 256^3 grid (403 MB) exceed the 256 MB last-level cache, and reading V
// without keeping it there leaves the cache to psi_R and psi_I, which the
// next pass reads (the z pass after the fused x pass: 86 -> 71 us); in FP32
// the fields fit and V is better cached (non-temporal V: x pass 63 -> 80 us).
template <typename R>
__device__ __forceinline__ R load_v(const R* p) {
    if constexpr (tuning<R>::V_NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// x passes re-read their inputs in the epilogue (instead of keeping them in
// registers through the transforms) for every length with X_RELOAD, else
// from X_RELOAD_FROM points: a 16384-point row runs 1024 lanes per block,
// which caps a lane at 128 registers
template <int N>
constexpr bool x_reload() { return SPSTD_X_RELOAD || N >= SPSTD_X_RELOAD_FROM; }

// Compiler-only memory barrier: values loaded before it are not reused
// after it (the epilogues re-read their inputs rather than keep them live
// in registers through the transforms).
__device__ __forceinline__ void reload_fence() { asm volatile("" ::: "memory"); }

// Start of an epilogue: its loads stay below the inverse transform.
__device__ __forceinline__ void epi_begin() {
    if constexpr (SPSTD_EPI_FENCE) asm volatile("" ::: "memory");
}

// Scheduling fence after every EPI_CHUNK-th epilogue element.
__device__ __forceinline__ void epi_fence(int e) {
    if constexpr (SPSTD_EPI_CHUNK < 16) {
        if ((e + 1) % SPSTD_EPI_CHUNK == 0) __builtin_amdgcn_sched_barrier(0);
    }
}

// Multiply bins kk = j + T*e by ks^2 (ks the signed bin index); under the
// ZERO convention the Nyquist bin kk = N/2 is removed.  The instance's
// scale is applied after the inverse transform.
template <typename R, int N>
__device__ __forceinline__ void apply_k2(cpx<R> (&v)[16], int j, int nyq_zero) {
    constexpr int T = N / 16;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int kk = j + T * e;
        const int ks = (kk <= N / 2) ? kk : kk - N;
        R s = (R)(ks * ks);
        if (nyq_zero && kk == N / 2) s = (R)0;
        v[e].x *= s;
        v[e].y *= s;
    }
}

template <typename R>
__device__ __forceinline__ R scale_of(const ScaleRef& sc, int64_t inst, int col) {
    return reinterpret_cast<const R*>(sc.tab)[(inst * sc.m + sc.l) * SC_COLS + col];
}

// Lanes per pencil T = N/16; lane groups per wave for N <= 1024.
template <int N>
struct pencil_cfg {
    static constexpr int T = N / 16;
    static constexpr bool WAVE = T <= 64;
    static constexpr int PPW = WAVE ? 64 / T : 1;
};

// Vector of 2*P reals: P complex pencils of a lane group.
template <typename R, int P>
struct vec_of;
template <>
struct vec_of<double, 1> { using type = double2; };
template <>
struct vec_of<float, 1> { using type = float2; };
template <>
struct vec_of<double, 2> { using type = double4; };
template <>
struct vec_of<float, 2> { using type = float4; };

// Streaming variant: the passes touch each element once, so the loads and
// stores may bypass cache retention (SPSTD_YZ_NT).
template <typename R, int P>
using ext_vec = R __attribute__((ext_vector_type(2 * P)));

template <typename R, int P>
__device__ __forceinline__ void load_group(const R* src, cpx<R> (&v)[P][16], int e) {
    if constexpr (SPSTD_YZ_NT) {
        const ext_vec<R, P> a = __builtin_nontemporal_load(reinterpret_cast<const ext_vec<R, P>*>(src));
#pragma unroll
        for (int q = 0; q < P; ++q) v[q][e] = cpx<R>{a[2 * q], a[2 * q + 1]};
        return;
    }
    using V = typename vec_of<R, P>::type;
    const V a = *reinterpret_cast<const V*>(src);
    if constexpr (P == 1) {
        v[0][e] = cpx<R>{a.x, a.y};
    } else {
        v[0][e] = cpx<R>{a.x, a.y};
        v[1][e] = cpx<R>{a.z, a.w};
    }
}

template <typename R, int P>
__device__ __forceinline__ void add_group(R* dst, const cpx<R> (&v)[P][16], int e) {
    if constexpr (SPSTD_YZ_NT) {
        ext_vec<R, P>* q = reinterpret_cast<ext_vec<R, P>*>(dst);
        ext_vec<R, P> a = __builtin_nontemporal_load(q);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            a[2 * k] += v[k][e].x;
            a[2 * k + 1] += v[k][e].y;
        }
        __builtin_nontemporal_store(a, q);
        return;
    }
    using V = typename vec_of<R, P>::type;
    V* q = reinterpret_cast<V*>(dst);
    V a = *q;
    if constexpr (P == 1) {
        a.x += v[0][e].x; a.y += v[0][e].y;
    } else {
        a.x += v[0][e].x; a.y += v[0][e].y;
        a.z += v[1][e].x; a.w += v[1][e].y;
    }
    *q = a;
}

// a += s * (the P complex values of element e), as one vector of 2P reals
template <typename R, int P>
__device__ __forceinline__ void add_vec(typename vec_of<R, P>::type& a, const cpx<R> (&v)[P][16], int e, R s) {
    if constexpr (P == 1) {
        a.x += s * v[0][e].x; a.y += s * v[0][e].y;
    } else {
        a.x += s * v[0][e].x; a.y += s * v[0][e].y;
        a.z += s * v[1][e].x; a.w += s * v[1][e].y;
    }
}

// ---------------------------------------------------------------------------
// y / z pass: dst += T_axis src.  A lane group carries P complex pencils
// (2P neighbouring x columns, one vector load per element).  Lane l of a
// wave: group g = l % PPW (the fast index, so neighbouring lanes read
// neighbouring columns), position j = l / PPW.
// ---------------------------------------------------------------------------
template <typename R, int N, int WPB, int P>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(yz_acc_waves<R, N>()))) void k_axis_acc(
    const R* __restrict__ src, R* __restrict__ dst, const cpx<double>* __restrict__ tw, AxisGeom g,
    ScaleRef sc, int col, int nyq_zero) {
    using C = pencil_cfg<N>;
    using TU = tuning<R>;
    static_assert(C::WAVE, "y/z pencils must fit in one wavefront");
    constexpr int LS = lds_size<N>::value;
    constexpr int SL = (TU::SPLIT ? 1 : 2) * LS;
    __shared__ R lds[N == 16 ? 1 : WPB * C::PPW * P * SL];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane % C::PPW, j = lane / C::PPW;
    const int64_t groups_x = g.half_x / P;
    const int64_t ngroups = groups_x * g.n_outer;
    constexpr int GPB = WPB * C::PPW;                 // lane groups per block
    int64_t group;
    if (SPSTD_YZ_ORDER == 1 && groups_x % GPB == 0) {
        // block b: plane b mod n_outer, column block b / n_outer
        const int64_t b = blockIdx.x;
        group = ((b % g.n_outer) * (groups_x / GPB) + b / g.n_outer) * GPB + wave * C::PPW + p;
    } else {
        group = ((int64_t)blockIdx.x * WPB + wave) * C::PPW + p;
    }
    const bool valid = group < ngroups;
    const int64_t gx = valid ? group % groups_x : 0, outer = valid ? group / groups_x : 0;
    const int64_t inst = outer / g.n_in;
    const int64_t base = inst * g.stride_hi + (outer - inst * g.n_in) * g.stride_lo + 2 * P * gx;
    const R scale = scale_of<R>(sc, inst, col);
    // a free batch slot has zero scales: a wave with nothing to update leaves
    // (its LDS barriers are wave-local)
    if (__all(!valid || scale == (R)0)) return;

    cpx<R> v[P][16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        if (valid) {
            load_group<R, P>(src + base + (int64_t)(j + C::T * e) * g.stride, v, e);
        } else {
#pragma unroll
            for (int q = 0; q < P; ++q) v[q][e] = cpx<R>{(R)0, (R)0};
        }
    }
    R* l0 = lds + (wave * C::PPW + p) * P * SL;
    fft_pencils<R, N, false, true, TU::SPLIT, TU::PRODUCTS, P, C::PPW>(v, j, l0, SL, tw);
#pragma unroll
    for (int q = 0; q < P; ++q) apply_k2<R, N>(v[q], j, nyq_zero);
    fft_pencils<R, N, true, true, TU::SPLIT, TU::PRODUCTS, P, C::PPW>(v, j, l0, SL, tw);
    epi_begin();
    if (valid) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                v[q][e].x *= scale;
                v[q][e].y *= scale;
            }
        }
        if constexpr (TU::EPI_BATCH && !SPSTD_YZ_NT) {
            using V = typename vec_of<R, P>::type;
            constexpr int CH = SPSTD_YZ_CHUNK;
#pragma unroll
            for (int e0 = 0; e0 < 16; e0 += CH) {
                V a[CH];
#pragma unroll
                for (int k = 0; k < CH; ++k)
                    a[k] = *reinterpret_cast<const V*>(dst + base + (int64_t)(j + C::T * (e0 + k)) * g.stride);
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    add_vec<R, P>(a[k], v, e0 + k, (R)1);
                    *reinterpret_cast<V*>(dst + base + (int64_t)(j + C::T * (e0 + k)) * g.stride) = a[k];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                add_group<R, P>(dst + base + (int64_t)(j + C::T * e) * g.stride, v, e);
                epi_fence(e);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// y pass at a stage boundary: the B half of stage l and the A half of stage
// l + 1 along the same pencils in one sweep,
//   psi_I += sB T_y psi_R,  then  psi_R += sA T_y psi_I(new).
// With the B half ordered x, z, y and the A half y, z, x, the y pencil of
// psi_I holds its x and z contributions of stage l when its y contribution
// is added, so the pencil is complete in registers when the A half of stage
// l + 1 transforms it.  Reads psi_R, psi_I; writes both (32 B per point in
// FP64 against 48 B for the two passes it replaces).
// ---------------------------------------------------------------------------
template <typename R, int N, int WPB, int P>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(yz_ba_waves<R, N>()))) void k_axis_ba(
    R* __restrict__ psiR, R* __restrict__ psiI, const cpx<double>* __restrict__ tw, AxisGeom g,
    ScaleRef scB, ScaleRef scA, int colB, int colA, int nyq_zero) {
    using C = pencil_cfg<N>;
    using TU = tuning<R>;
    using V = typename vec_of<R, P>::type;
    static_assert(C::WAVE, "y/z pencils must fit in one wavefront");
    constexpr int LS = lds_size<N>::value;
    constexpr int SL = (TU::SPLIT ? 1 : 2) * LS;
    __shared__ R lds[N == 16 ? 1 : WPB * C::PPW * P * SL];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane % C::PPW, j = lane / C::PPW;
    const int64_t groups_x = g.half_x / P;
    const int64_t ngroups = groups_x * g.n_outer;
    constexpr int GPB = WPB * C::PPW;
    int64_t group;
    if (SPSTD_YZ_ORDER == 1 && groups_x % GPB == 0) {
        const int64_t b = blockIdx.x;
        group = ((b % g.n_outer) * (groups_x / GPB) + b / g.n_outer) * GPB + wave * C::PPW + p;
    } else {
        group = ((int64_t)blockIdx.x * WPB + wave) * C::PPW + p;
    }
    const bool valid = group < ngroups;
    const int64_t gx = valid ? group % groups_x : 0, outer = valid ? group / groups_x : 0;
    const int64_t inst = outer / g.n_in;
    const int64_t base = inst * g.stride_hi + (outer - inst * g.n_in) * g.stride_lo + 2 * P * gx;
    const R sB = scale_of<R>(scB, inst, colB), sA = scale_of<R>(scA, inst, colA);
    if (__all(!valid || (sB == (R)0 && sA == (R)0))) return;

    constexpr bool RL = TU::BA_RELOAD;
    cpx<R> v[P][16], f[P][RL ? 1 : 16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        if (valid) {
            load_group<R, P>(psiR + base + (int64_t)(j + C::T * e) * g.stride, v, e);
        } else {
#pragma unroll
            for (int q = 0; q < P; ++q) v[q][e] = cpx<R>{(R)0, (R)0};
        }
        if constexpr (!RL) {
#pragma unroll
            for (int q = 0; q < P; ++q) f[q][e] = v[q][e];
        }
    }
    if constexpr (RL) reload_fence();
    R* l0 = lds + (wave * C::PPW + p) * P * SL;
    // B half of stage l: psi_I += sB T psi_R
    fft_pencils<R, N, false, true, TU::SPLIT, TU::PRODUCTS, P, C::PPW>(v, j, l0, SL, tw);
#pragma unroll
    for (int q = 0; q < P; ++q) apply_k2<R, N>(v[q], j, nyq_zero);
    fft_pencils<R, N, true, true, TU::SPLIT, TU::PRODUCTS, P, C::PPW>(v, j, l0, SL, tw);
    epi_begin();
    if constexpr (TU::EPI_BATCH) {
        constexpr int CH = SPSTD_YZ_CHUNK;
#pragma unroll
        for (int e0 = 0; e0 < 16; e0 += CH) {
            V a[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                a[k] = V{};
                if (valid) a[k] = *reinterpret_cast<const V*>(psiI + base + (int64_t)(j + C::T * (e0 + k)) * g.stride);
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                add_vec<R, P>(a[k], v, e0 + k, sB);
                v[0][e0 + k] = cpx<R>{a[k].x, a[k].y};
                if constexpr (P == 2) v[1][e0 + k] = cpx<R>{a[k].z, a[k].w};
                if (valid) *reinterpret_cast<V*>(psiI + base + (int64_t)(j + C::T * (e0 + k)) * g.stride) = a[k];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            V a{};
            V* q = reinterpret_cast<V*>(psiI + base + (int64_t)(j + C::T * e) * g.stride);
            if (valid) a = *q;
            if constexpr (P == 1) {
                a.x += sB * v[0][e].x; a.y += sB * v[0][e].y;
                v[0][e] = cpx<R>{a.x, a.y};
            } else {
                a.x += sB * v[0][e].x; a.y += sB * v[0][e].y;
                a.z += sB * v[1][e].x; a.w += sB * v[1][e].y;
                v[0][e] = cpx<R>{a.x, a.y};
                v[1][e] = cpx<R>{a.z, a.w};
            }
            if (valid) *q = a;
            epi_fence(e);
        }
    }
    // A half of stage l + 1: psi_R += sA T psi_I(new)
    fft_pencils<R, N, false, true, TU::SPLIT, TU::PRODUCTS, P, C::PPW>(v, j, l0, SL, tw);
#pragma unroll
    for (int q = 0; q < P; ++q) apply_k2<R, N>(v[q], j, nyq_zero);
    fft_pencils<R, N, true, true, TU::SPLIT, TU::PRODUCTS, P, C::PPW>(v, j, l0, SL, tw);
    epi_begin();
    if (valid) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            V* q = reinterpret_cast<V*>(psiR + base + (int64_t)(j + C::T * e) * g.stride);
            V a;
            if constexpr (RL) {
                a = *q;   // psi_R as loaded at the start (unchanged in memory)
                if constexpr (P == 1) {
                    a.x += sA * v[0][e].x; a.y += sA * v[0][e].y;
                } else {
                    a.x += sA * v[0][e].x; a.y += sA * v[0][e].y;
                    a.z += sA * v[1][e].x; a.w += sA * v[1][e].y;
                }
            } else if constexpr (P == 1) {
                a.x = f[0][e].x + sA * v[0][e].x; a.y = f[0][e].y + sA * v[0][e].y;
            } else {
                a.x = f[0][e].x + sA * v[0][e].x; a.y = f[0][e].y + sA * v[0][e].y;
                a.z = f[1][e].x + sA * v[1][e].x; a.w = f[1][e].y + sA * v[1][e].y;
            }
            *q = a;
            epi_fence(e);
        }
    }
}

// ---------------------------------------------------------------------------
// x pass helpers: lane l -> position j = l % T, pencil-in-wave p = l / T
// (neighbouring lanes read neighbouring x), or one pencil per block for
// N > 1024.
// ---------------------------------------------------------------------------
template <typename R, int N, int WPB, bool SPLIT_PREF = tuning<R>::SPLIT>
struct row_map {
    using C = pencil_cfg<N>;
    static constexpr int PPB = C::WAVE ? WPB * C::PPW : 1;   // pencils per block
    static constexpr int THREADS = C::WAVE ? 64 * WPB : C::T;
    static constexpr int LS = lds_size<N>::value;
    // large pencils always exchange re and im in turn to stay within LDS
    static constexpr bool SPLIT = C::WAVE ? SPLIT_PREF : true;
    static constexpr int SL = (SPLIT ? 1 : 2) * LS;
    // a 16-point pencil is one radix-16 pass in registers: no LDS at all
    static constexpr int LDS_REALS = N == 16 ? 1 : PPB * SL;
};

// Row pair of this lane: rows 2q and 2q + 1 with q = block_pair0 + pin_block.
// Fields are addressed as (block-uniform pointer) + (32-bit lane offset) +
// (compile-time element offset), so one VGPR holds a lane's address.
template <typename R, int N, int WPB>
struct row_lane {
    int j;            // position in the pencil
    int pin_block;    // pencil index within the block
    int64_t q;        // global pencil (row pair) index
    int64_t row0;     // first row of the block (uniform)
    int off;          // lane offset of row 2q, element j, from row0
};

template <typename R, int N, int WPB>
__device__ __forceinline__ row_lane<R, N, WPB> row_coords() {
    using C = pencil_cfg<N>;
    row_lane<R, N, WPB> L;
    if constexpr (C::WAVE) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        L.j = lane % C::T;
        L.pin_block = wave * C::PPW + lane / C::T;
    } else {
        L.j = threadIdx.x;
        L.pin_block = 0;
    }
    L.q = (int64_t)blockIdx.x * row_map<R, N, WPB>::PPB + L.pin_block;
    L.row0 = (int64_t)blockIdx.x * row_map<R, N, WPB>::PPB * 2;
    L.off = 2 * L.pin_block * N + L.j;
    return L;
}

// FULL: every row pair of every block exists (no per-lane guards, so the
// epilogue's loads can be batched); otherwise rows past nrows are skipped.
template <typename R, int N, int WPB, bool FULL>
__global__ __launch_bounds__((row_map<R, N, WPB>::THREADS)) SPSTD_WAVES_ATTR void k_x_acc(
    const R* __restrict__ src, R* __restrict__ dst, const R* __restrict__ V,
    const cpx<double>* __restrict__ tw, RowGeom rg, ScaleRef sc, int kcol, int pcol, int nyq_zero) {
    using C = pencil_cfg<N>;
    using M = row_map<R, N, WPB>;
    using TU = tuning<R>;
    __shared__ R lds[M::LDS_REALS];
    const row_lane<R, N, WPB> L = row_coords<R, N, WPB>();
    const int j = L.j;
    const int64_t nrows = rg.nrows;
    const bool v0 = FULL || 2 * L.q < nrows, v1 = FULL || 2 * L.q + 1 < nrows;
    const int64_t inst0 = v0 ? (2 * L.q) / rg.rows_per_inst : 0;
    const int64_t inst1 = v1 ? (2 * L.q + 1) / rg.rows_per_inst : inst0;
    {
        // rows of free batch slots (zero scales) need no work; the test is
        // uniform over the wave, or over the workgroup for one-pencil blocks
        const bool idle = scale_of<R>(sc, inst0, kcol) == (R)0 && scale_of<R>(sc, inst1, kcol) == (R)0 &&
                          scale_of<R>(sc, inst0, pcol) == (R)0 && scale_of<R>(sc, inst1, pcol) == (R)0;
        if (__all(idle)) return;
    }
    const int64_t b = L.row0 * N;
    const R* __restrict__ sb = src + b;
    R* __restrict__ db = dst + b;
    const R* __restrict__ Vb = V + b;
    const int o0 = L.off, o1 = L.off + N;
    constexpr bool RL = x_reload<N>();
    cpx<R> v[1][16];
    R f0[RL ? 1 : 16], f1[RL ? 1 : 16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const R a = v0 ? sb[o0 + C::T * e] : (R)0;
        const R c = v1 ? sb[o1 + C::T * e] : (R)0;
        v[0][e] = cpx<R>{a, c};
        if constexpr (!RL) {
            f0[e] = a;
            f1[e] = c;
        }
    }
    if constexpr (RL) reload_fence();
    R* l0 = lds + L.pin_block * M::SL;
    fft_pencils<R, N, false, C::WAVE, M::SPLIT, TU::PRODUCTS, 1, 1>(v, j, l0, M::SL, tw);
    apply_k2<R, N>(v[0], j, nyq_zero);
    fft_pencils<R, N, true, C::WAVE, M::SPLIT, TU::PRODUCTS, 1, 1>(v, j, l0, M::SL, tw);
    epi_begin();
    const R k0 = scale_of<R>(sc, inst0, kcol), p0 = scale_of<R>(sc, inst0, pcol);
    const R k1 = scale_of<R>(sc, inst1, kcol), p1 = scale_of<R>(sc, inst1, pcol);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i0 = o0 + C::T * e, i1 = o1 + C::T * e;
        R a, c;
        if constexpr (RL) {
            a = v0 ? sb[i0] : (R)0;
            c = v1 ? sb[i1] : (R)0;
        } else {
            a = f0[e];
            c = f1[e];
        }
        if (v0) db[i0] = db[i0] + k0 * v[0][e].x + p0 * load_v(Vb + i0) * a;
        if (v1) db[i1] = db[i1] + k1 * v[0][e].y + p1 * load_v(Vb + i1) * c;
        epi_fence(e);
    }
}

template <typename R, int N, int WPB, bool FULL>
__global__ __launch_bounds__((row_map<R, N, WPB>::THREADS)) __attribute__((amdgpu_waves_per_eu(x_ab_waves<R, N>()))) void k_x_ab(
    R* __restrict__ psiR, R* __restrict__ psiI, const R* __restrict__ V,
    const cpx<double>* __restrict__ tw, RowGeom rg, ScaleRef sc, int nyq_zero) {
    using C = pencil_cfg<N>;
    // FP32: the joint exchange up to 256-point rows, the split one beyond
    // (512^2 batch 463 -> 428 us per step; 256^3 x pass 63 -> 75 us split)
    using M = row_map<R, N, WPB, (sizeof(R) == 4 ? (N >= SPSTD_SPLIT_XAB_F32_FROM) : tuning<R>::SPLIT_XAB)>;
    using TU = tuning<R>;
    __shared__ R lds[M::LDS_REALS];
    const row_lane<R, N, WPB> L = row_coords<R, N, WPB>();
    const int j = L.j;
    const int64_t nrows = rg.nrows;
    const bool v0 = FULL || 2 * L.q < nrows, v1 = FULL || 2 * L.q + 1 < nrows;
    const int64_t inst0 = v0 ? (2 * L.q) / rg.rows_per_inst : 0;
    const int64_t inst1 = v1 ? (2 * L.q + 1) / rg.rows_per_inst : inst0;
    {
        const bool idle = scale_of<R>(sc, inst0, SC_KXA) == (R)0 && scale_of<R>(sc, inst1, SC_KXA) == (R)0 &&
                          scale_of<R>(sc, inst0, SC_KXB) == (R)0 && scale_of<R>(sc, inst1, SC_KXB) == (R)0;
        if (__all(idle)) return;
    }
    const int64_t b = L.row0 * N;
    R* __restrict__ Rb = psiR + b;
    R* __restrict__ Ib = psiI + b;
    const R* __restrict__ Vb = V + b;
    const int o0 = L.off, o1 = L.off + N;
    constexpr bool RL = x_reload<N>();
    cpx<R> v[1][16];
    cpx<R> f[RL ? 1 : 16];   // psi_I on entry; later psi_I + vb * V * psi_R(new)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        v[0][e].x = v0 ? Ib[o0 + C::T * e] : (R)0;
        v[0][e].y = v1 ? Ib[o1 + C::T * e] : (R)0;
        if constexpr (!RL) f[e] = v[0][e];
    }
    if constexpr (RL) reload_fence();
    R* l0 = lds + L.pin_block * M::SL;
    // A half: psi_R += T_x^A psi_I + p_A V psi_I
    fft_pencils<R, N, false, C::WAVE, M::SPLIT, TU::PRODUCTS, 1, 1>(v, j, l0, M::SL, tw);
    apply_k2<R, N>(v[0], j, nyq_zero);
    fft_pencils<R, N, true, C::WAVE, M::SPLIT, TU::PRODUCTS, 1, 1>(v, j, l0, M::SL, tw);
    epi_begin();
    const cpx<R> sa = {scale_of<R>(sc, inst0, SC_KXA), scale_of<R>(sc, inst1, SC_KXA)};
    const cpx<R> va = {scale_of<R>(sc, inst0, SC_PA), scale_of<R>(sc, inst1, SC_PA)};
    const cpx<R> sb = {scale_of<R>(sc, inst0, SC_KXB), scale_of<R>(sc, inst1, SC_KXB)};
    const cpx<R> vb = {scale_of<R>(sc, inst0, SC_PB), scale_of<R>(sc, inst1, SC_PB)};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i0 = o0 + C::T * e, i1 = o1 + C::T * e;
        cpx<R> vv = {(R)0, (R)0}, g = {(R)0, (R)0}, fe;
        if constexpr (RL) fe = cpx<R>{v0 ? Ib[i0] : (R)0, v1 ? Ib[i1] : (R)0};
        else fe = f[e];
        if (v0) { vv.x = load_v(Vb + i0); g.x = Rb[i0]; }
        if (v1) { vv.y = load_v(Vb + i1); g.y = Rb[i1]; }
        g.x = g.x + sa.x * v[0][e].x + va.x * vv.x * fe.x;
        g.y = g.y + sa.y * v[0][e].y + va.y * vv.y * fe.y;
        if (v0) Rb[i0] = g.x;
        if (v1) Rb[i1] = g.y;
        v[0][e] = g;
        if constexpr (!RL) {
            f[e].x = fe.x + vb.x * vv.x * g.x;
            f[e].y = fe.y + vb.y * vv.y * g.y;
        }
        epi_fence(e);
    }
    if constexpr (RL) reload_fence();
    // B half: psi_I += T_x^B psi_R(new) + p_B V psi_R(new)
    fft_pencils<R, N, false, C::WAVE, M::SPLIT, TU::PRODUCTS, 1, 1>(v, j, l0, M::SL, tw);
    apply_k2<R, N>(v[0], j, nyq_zero);
    fft_pencils<R, N, true, C::WAVE, M::SPLIT, TU::PRODUCTS, 1, 1>(v, j, l0, M::SL, tw);
    epi_begin();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i0 = o0 + C::T * e, i1 = o1 + C::T * e;
        if constexpr (RL) {
            // psi_R here is the value this lane stored in the A epilogue
            if (v0) Ib[i0] = Ib[i0] + vb.x * load_v(Vb + i0) * Rb[i0] + sb.x * v[0][e].x;
            if (v1) Ib[i1] = Ib[i1] + vb.y * load_v(Vb + i1) * Rb[i1] + sb.y * v[0][e].y;
        } else {
            if (v0) Ib[i0] = f[e].x + sb.x * v[0][e].x;
            if (v1) Ib[i1] = f[e].y + sb.y * v[0][e].y;
        }
        epi_fence(e);
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
__global__ __launch_bounds__((row_map<R, N, SPSTD_WPB>::THREADS)) void k_energy_axis(
    const R* __restrict__ psiR, const R* __restrict__ psiI, const cpx<double>* __restrict__ tw,
    EnergyGeom g, int nyq_zero, R msign, double* __restrict__ partials) {
    using C = pencil_cfg<N>;
    using M = row_map<R, N, SPSTD_WPB>;
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
__global__ __launch_bounds__((row_map<R, N, SPSTD_WPB>::THREADS)) void k_wall_acc(
    const R* __restrict__ src, R* __restrict__ dst, const R* __restrict__ V,
    const cpx<double>* __restrict__ tw, EnergyGeom g, int64_t npts, ScaleRef sc, int kcol, int pcol,
    int nyq_zero, R msign) {
    using C = pencil_cfg<N>;
    using M = row_map<R, N, SPSTD_WPB>;
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
constexpr int kWPB = SPSTD_WPB;   // waves per block of the wave-local passes

// Waves per block of the hot pass kernels (y/z passes, the stage-boundary y
// sweep, x passes): 2 for FP64 256-point pencils, where smaller blocks let
// consecutive passes overlap their tails (graph-replayed 256^3 FP64 step
// 2.72 -> 2.63 ms), SPSTD_WPB elsewhere (512^2 FP64 batch: 596 us per step
// with 4, 692 with 2).
template <typename R, int N>
constexpr int wpb_of() {
    return (sizeof(R) == 8 && N == 256) ? SPSTD_WPB_F64_256 : SPSTD_WPB;
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
    constexpr int P = (sizeof(R) == 4 && N >= 512) ? SPSTD_BA_PPL_F32_LONG : tuning<R>::BA_PPL;
    constexpr int W = W0 ? W0 : wpb_of<R, N>();
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
    constexpr int W = W0 ? W0 : wpb_of<R, N>();
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
    constexpr int W = W0 ? W0 : wpb_of<R, N>();
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
                              int64_t capacity) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst || !active[i]) return;
    const int64_t slot = counter[i];
    if (slot < capacity) {
        double* out = probes + ((int64_t)i * capacity + slot) * nprobes * 2;
        for (int q = 0; q < nprobes; ++q) {
            const int64_t k = (int64_t)i * npts + idx[(int64_t)i * nprobes + q];
            out[2 * q] = (double)psiR[k];
            out[2 * q + 1] = (double)psiI[k];
        }
    }
    counter[i] = slot + 1;
}

template <typename R>
hipError_t launch_probe_batch(const R* psiR, const R* psiI, int64_t npts, const int64_t* idx, int nprobes,
                              const int* active, int ninst, double* probes, int64_t* counter,
                              int64_t capacity, hipStream_t st) {
    const int blocks = (ninst + 63) / 64;
    hipLaunchKernelGGL((k_probe_batch<R>), dim3(blocks), dim3(64), 0, st, psiR, psiI, npts, idx, nprobes,
                       active, ninst, probes, counter, capacity);
    return hipGetLastError();
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
                                              hipStream_t);                                     \
    template hipError_t launch_probe<R>(const R*, const R*, const int64_t*, int, double*,       \
                                        int64_t*, int64_t, hipStream_t);                        \
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

}  // namespace spstd
