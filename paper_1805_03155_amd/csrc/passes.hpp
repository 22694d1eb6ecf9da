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
#pragma once
#include <type_traits>

#include "fft_core.hpp"
#include "kernels.hpp"

namespace spstd {


// Tuning of the pass kernels (each choice measured on MI355X, 256^3 and the
// batching workload; the alternatives named here were measured slower and
// are not built):
//   - twiddles of a pass from two FP64 table reads and FP64 products instead
//     of one read per twiddle (FP32 256^3 graph step 1.58 -> 1.44 ms, FP32
//     512^2 batch 428 -> 319 us);
//   - the real-then-imaginary (split) LDS exchange, half the LDS per wave;
//     the fused FP32 x pass takes the joint exchange below 512 points per row;
//   - x passes keep their inputs in registers through the transforms, except
//     16384-point rows, whose 1024 lanes per block cap a lane at 128
//     registers (FP32 batch of 33 such rows 196 -> 178 us per step re-reading;
//     at 8192 re-reading is slower, 84 -> 93 us);
//   - at least two waves per SIMD (otherwise the FP64 x passes of 512..2048
//     point rows fall to one); four for the 256-point FP32 y/z pass (z 41.4 ->
//     35.6 us); more for the FP64 y/z pass or the FP32 boundary sweep spill;
//   - two complex pencils per lane group in FP32 y/z passes, one in FP64
//     (two: 256 registers); the FP32 boundary sweep one up to 256 points
//     (142 registers, three waves per SIMD: 59.1 -> 55.0 us) and two from 512;
//     the boundary sweep keeps psi_R in registers (re-reading it: 106 -> 121
//     us FP64, 65 -> 68 us FP32);
//   - non-temporal reads of V in FP64 x passes (the next z pass 86 -> 71 us),
//     cached in FP32; plain (temporal) y/z loads and stores (non-temporal
//     ones: 79 -> 106 us);
//   - epilogues scheduled four elements at a time; FP32 y/z epilogues read
//     four elements before writing them (z 41.8 -> 41.3 us), FP64 ones element
//     by element (73.3 against 71.0 us);
//   - consecutive y/z blocks take the same column group of neighbouring
//     planes (y 80 -> 77 us), which spreads the running blocks over memory
//     channels.
constexpr int kMinWaves = 2;          // minimum waves per SIMD of the pass kernels
constexpr int kWavesF32Axis256 = 4;   // ... of the 256-point FP32 y/z pass
constexpr int kXReloadFrom = 16384;   // x passes re-read their inputs from this row length
constexpr int kSplitXabF32From = 512; // the fused FP32 x pass splits its exchange from here
constexpr int kEpiChunk = 4;          // epilogue elements scheduled together
constexpr int kYzChunk = 4;           // FP32 y/z epilogue reads batched before the writes

#define SPSTD_WAVES_ATTR __attribute__((amdgpu_waves_per_eu(kMinWaves)))

template <typename R>
struct tuning;
template <>
struct tuning<double> {
    static constexpr bool PRODUCTS = true;
    static constexpr bool SPLIT = true;
    static constexpr bool SPLIT_XAB = true;
    static constexpr int YZ_PPL = 1;
    static constexpr bool V_NT = true;
    static constexpr bool EPI_BATCH = false;
    static constexpr int BA_PPL = 1;
};
template <>
struct tuning<float> {
    static constexpr bool PRODUCTS = true;
    static constexpr bool SPLIT = true;
    static constexpr bool SPLIT_XAB = false;
    static constexpr int YZ_PPL = 2;
    static constexpr bool V_NT = false;
    static constexpr bool EPI_BATCH = true;
    // two pencils per lane group in the boundary sweep too (256^3: 53.7 ->
    // 51.2 us once the LDS strides were free of bank conflicts; slower
    // before, 53.8 -> 56.9 us, when its exchanges conflicted four ways)
    static constexpr int BA_PPL = 2;
};

// Minimum waves per SIMD requested for the 256-point pass kernels (a value
// of 0 leaves the general setting).  A 256^3 FP32 y/z pass is 16 waves per
// CU: at 137 registers three waves per SIMD fit, which leaves a second round
// a third full; capped at 128 registers all 16 run at once (z 41.4 -> 35.6
// us).
template <typename R, int N>
constexpr int yz_acc_waves() {
    return (N == 256 && sizeof(R) == 4) ? kWavesF32Axis256 : kMinWaves;
}
template <typename R, int N>
constexpr int yz_ba_waves() {
    return kMinWaves;
}
template <typename R, int N>
constexpr int x_ab_waves() {
    return kMinWaves;
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
constexpr bool x_reload() { return N >= kXReloadFrom; }

// Compiler-only memory barrier: values loaded before it are not reused
// after it (the epilogues re-read their inputs rather than keep them live
// in registers through the transforms).
__device__ __forceinline__ void reload_fence() { asm volatile("" ::: "memory"); }

// Start of an epilogue: its loads stay below the inverse transform.
__device__ __forceinline__ void epi_begin() {
    asm volatile("" ::: "memory");
}

// Scheduling fence after every EPI_CHUNK-th epilogue element.
__device__ __forceinline__ void epi_fence(int e) {
    if ((e + 1) % kEpiChunk == 0) __builtin_amdgcn_sched_barrier(0);
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

template <typename R, int P>
__device__ __forceinline__ void load_group(const R* src, cpx<R> (&v)[P][16], int e) {
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
// LDS of a y/z pass block: per lane group P pencils of SL reals.
// LDS pencil strides.  The LDS serves 128 bytes per cycle (32 FP32 or 16
// FP64 lanes over 32 four-byte banks); the pencils whose lanes share a
// cycle must start on different banks, or each exchange takes two to four
// times its cycles.  A pencil's region is therefore made an odd multiple of
// the words one pencil contributes to a cycle: 32/PPW words where the
// pencil index is fastest over the lanes (y and z passes), T words per
// FP32 lane and 2T per FP64 lane where the position is (x passes).  A
// stride that is a multiple of 32 words put all four pencils of a
// 256-point FP64 y/z wave on one bank (z pass 69.8 -> 67.4 us, boundary
// sweep 96.7 -> 91.9 us once padded).
constexpr int odd_multiple_at_least(int base, int words_per_elem, int unit_words) {
    if (unit_words <= 0 || unit_words >= 32) return base;
    int s = base;
    while ((s * words_per_elem) % unit_words != 0 || ((s * words_per_elem) / unit_words) % 2 == 0) ++s;
    return s;
}

// Elements between the lane groups of a y/z wave (pencil index fastest):
// P pencils of sl elements each per lane group.
template <typename R, int N, int P>
constexpr int yz_pencil_stride(int sl) {
    constexpr int ppw = pencil_cfg<N>::PPW;
    constexpr int ew = (int)(sizeof(R) / 4);
    constexpr int unit = ppw < 2 ? 0 : 32 / ppw;   // words of one pencil in an LDS cycle
    // (an odd multiple is reachable only if P words per element divide it)
    if (unit == 0 || unit % (P * ew) != 0) return sl;
    // the lane-group stride P * sl must be an odd multiple of unit words
    int s = sl;
    while (((P * s * ew) % unit) != 0 || (((P * s * ew) / unit) % 2) == 0) ++s;
    return s;
}

template <typename R, int N, int WPB, int P>
struct yz_lds {
    static constexpr int SL = yz_pencil_stride<R, N, P>((tuning<R>::SPLIT ? 1 : 2) * lds_size<N>::value);
    static constexpr int REALS = N == 16 ? 1 : WPB * pencil_cfg<N>::PPW * P * SL;
};

// The pass of block blk of the launch's grid with the block's LDS.  The
// body text (body_*.inc) is expanded both in the single-shape kernel
// (blk = blockIdx.x) and in this device function, which the mixed-shape
// kernels call with a tile's block: the kernel then compiles as one
// function (an inlined separate body costs the FP64 256-point y/z pass 22
// registers, its boundary sweep and fused x pass spills).
template <typename R, int N, int WPB, int P>
__device__ __forceinline__ void axis_acc_body(int64_t blk, R* __restrict__ lds, const R* __restrict__ src,
                                              R* __restrict__ dst, const cpx<double>* __restrict__ tw,
                                              const AxisGeom& g, const ScaleRef& sc, int col, int nyq_zero) {
#include "body_axis_acc.inc"
}

template <typename R, int N, int WPB, int P>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(yz_acc_waves<R, N>()))) void k_axis_acc(
    const R* __restrict__ src, R* __restrict__ dst, const cpx<double>* __restrict__ tw, AxisGeom g,
    ScaleRef sc, int col, int nyq_zero) {
    __shared__ R lds_block[yz_lds<R, N, WPB, P>::REALS];
    R* const lds = lds_block;
    const int64_t blk = blockIdx.x;
#include "body_axis_acc.inc"
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
__device__ __forceinline__ void axis_ba_body(int64_t blk, R* __restrict__ lds, R* __restrict__ psiR,
                                             R* __restrict__ psiI, const cpx<double>* __restrict__ tw,
                                             const AxisGeom& g, const ScaleRef& scB, const ScaleRef& scA,
                                             int colB, int colA, int nyq_zero) {
#include "body_axis_ba.inc"
}

template <typename R, int N, int WPB, int P>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(yz_ba_waves<R, N>()))) void k_axis_ba(
    R* __restrict__ psiR, R* __restrict__ psiI, const cpx<double>* __restrict__ tw, AxisGeom g,
    ScaleRef scB, ScaleRef scA, int colB, int colA, int nyq_zero) {
    __shared__ R lds_block[yz_lds<R, N, WPB, P>::REALS];
    R* const lds = lds_block;
    const int64_t blk = blockIdx.x;
#include "body_axis_ba.inc"
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
    static constexpr int SL =
        odd_multiple_at_least((SPLIT ? 1 : 2) * LS, (int)(sizeof(R) / 4), C::T * (int)(sizeof(R) / 4));
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
__device__ __forceinline__ row_lane<R, N, WPB> row_coords(int64_t blk) {
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
    L.q = blk * row_map<R, N, WPB>::PPB + L.pin_block;
    L.row0 = blk * row_map<R, N, WPB>::PPB * 2;
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
    const row_lane<R, N, WPB> L = row_coords<R, N, WPB>(blockIdx.x);
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

// LDS exchange of the fused x pass: JOINT (real and imaginary parts
// together) for rows shorter than 512 points, else split (in turn).  The
// built-in choice: FP32 joint up to 256-point rows (512^2 batch 463 -> 428
// us per step; 256^3 x pass 63 -> 75 us split), FP64 split.
template <typename R, int N, int WPB, bool JOINT>
using x_ab_map = row_map<R, N, WPB, (JOINT ? (N >= kSplitXabF32From) : true)>;
template <typename R>
constexpr bool x_ab_joint() { return sizeof(R) == 4 ? true : !tuning<R>::SPLIT_XAB; }

template <typename R, int N, int WPB, bool FULL, bool JOINT>
__device__ __forceinline__ void x_ab_body(int64_t blk, R* __restrict__ lds, R* __restrict__ psiR,
                                          R* __restrict__ psiI, const R* __restrict__ V,
                                          const cpx<double>* __restrict__ tw, const RowGeom& rg,
                                          const ScaleRef& sc, int nyq_zero) {
#include "body_x_ab.inc"
}

template <typename R, int N, int WPB, bool FULL>
__global__ __launch_bounds__((row_map<R, N, WPB>::THREADS)) __attribute__((amdgpu_waves_per_eu(x_ab_waves<R, N>()))) void k_x_ab(
    R* __restrict__ psiR, R* __restrict__ psiI, const R* __restrict__ V,
    const cpx<double>* __restrict__ tw, RowGeom rg, ScaleRef sc, int nyq_zero) {
    constexpr bool JOINT = x_ab_joint<R>();
    __shared__ R lds_block[x_ab_map<R, N, WPB, JOINT>::LDS_REALS];
    R* const lds = lds_block;
    const int64_t blk = blockIdx.x;
#include "body_x_ab.inc"
}

}  // namespace spstd
