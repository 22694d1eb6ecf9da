// x passes of long 1D rows (8192 and 16384 points) spread over many
// workgroups: the four-step factorisation of the transform.
//
// The pass computes g += s T f + p V f with T f = F^-1 (ks^2 F f) along the
// row (Eq. (9)-(10), Eq. (18)); s and p are the instance's scales of the
// half (the kinetic scale carries 1/N).  Two real rows travel as one
// complex pencil (row 2q in the real part, 2q + 1 in the imaginary part),
// as in the one-workgroup row kernels.  With N = N1 N2 (N1 = 128 columns,
// N2 = N / 128 rows; n = n1 + N1 n2, k = k2 + N2 k1) the forward transform
// is
//   X[k2 + N2 k1] = sum_n1 w_N1^(n1 k1) w_N^(n1 k2) sum_n2 w_N2^(n2 k2) x[n1 + N1 n2],
// so one pass of the row is three launches over a scratch copy S of the
// pencil (layout S[k2][n1]):
//   columns: for each n1 the N2-point transform over n2, times w_N^(n1 k2);
//   rows:    for each k2 the N1-point transform over n1 (giving k1), times
//            ks^2 with ks the signed index of k = k2 + N2 k1, and the
//            N1-point inverse back to n1, in place;
//   columns: times w_N^-(n1 k2), the N2-point inverse over k2 (giving n2),
//            and the update of g at n = n1 + N1 n2.
// A fused A+B x pass runs the B half's first column launch inside the A
// half's last (psi_R(new) of a column is in registers there), so it is
// five launches; likewise a B half followed by the next stage's A half
// transforms psi_I(new) for it, which then starts at its row launch.  Each
// launch has N / 16 lanes of work per pencil (eight or sixteen workgroups
// of four waves) where the one-workgroup kernels have one workgroup per
// pencil: the row's latency is spread over the chip.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "passes.hpp"

namespace spstd {

bool fourstep_ok(int64_t n) { return n == 8192 || n == 16384; }

namespace {

constexpr int kFsWaves = 4;   // waves per workgroup

template <int N>
struct fs_shape {
    static constexpr int N1 = 128;
    static constexpr int N2 = N / N1;
    // columns (N2-point transforms): pencil index fastest over the lanes
    static constexpr int T2 = N2 / 16, PPW2 = 64 / T2;
    static constexpr int COLS_PER_BLOCK = kFsWaves * PPW2;
    static constexpr int COL_BLOCKS = N1 / COLS_PER_BLOCK;
    // rows (N1-point transforms): position fastest over the lanes
    static constexpr int T1 = N1 / 16, PPW1 = 64 / T1;
    static constexpr int ROWS_PER_BLOCK = kFsWaves * PPW1;
    static constexpr int ROW_BLOCKS = N2 / ROWS_PER_BLOCK;
    static_assert(COL_BLOCKS >= 1 && ROW_BLOCKS >= 1, "whole workgroups per pencil");
};

template <typename R, int NL>
struct fs_lds {
    static constexpr int LS = lds_size<NL>::value;
    static constexpr int ew = (int)(sizeof(R) / 4);
    // columns: the stride between lane groups avoids bank conflicts as in
    // the y/z passes; rows: as in the x passes
    static constexpr int SL_COL = yz_pencil_stride<R, NL, 1>((tuning<R>::SPLIT ? 1 : 2) * LS);
    static constexpr int SL_ROW =
        odd_multiple_at_least((tuning<R>::SPLIT ? 1 : 2) * LS, ew, (NL / 16) * ew);
};

// The pencil's instances and whether the pass leaves it unchanged (both
// rows with zero kinetic scales in the columns it applies; free slots).
struct FsPencil {
    int64_t inst0, inst1;
    bool v0, v1;
};

template <typename R>
__device__ __forceinline__ FsPencil fs_pencil(int64_t q, const RowGeom& rg) {
    FsPencil P;
    P.v0 = 2 * q < rg.nrows;
    P.v1 = 2 * q + 1 < rg.nrows;
    P.inst0 = P.v0 ? (2 * q) / rg.rows_per_inst : 0;
    P.inst1 = P.v1 ? (2 * q + 1) / rg.rows_per_inst : P.inst0;
    return P;
}

template <typename R>
__device__ __forceinline__ bool fs_idle(const FsPencil& P, const ScaleRef& sc, int ca, int cb) {
    bool idle = scale_of<R>(sc, P.inst0, ca) == (R)0 && scale_of<R>(sc, P.inst1, ca) == (R)0;
    if (cb >= 0) idle = idle && scale_of<R>(sc, P.inst0, cb) == (R)0 && scale_of<R>(sc, P.inst1, cb) == (R)0;
    return idle;
}

// v[e] (bin k2 = j + T2 e of column n1) times w_N^(+-n1 k2), the factor
// formed in FP64 from the row's table and rounded once.
template <typename R, int N, bool CONJ>
__device__ __forceinline__ void fs_twiddle(cpx<R> (&v)[16], int n1, int j, const cpx<double>* __restrict__ twN) {
    using S = fs_shape<N>;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int k2 = j + S::T2 * e;
        const cpx<double> w = twN[n1 * k2];   // n1 k2 < N1 N2 = N
        const cpx<R> wr = {(R)w.x, (R)w.y};
        v[e] = CONJ ? cmulc(v[e], wr) : cmul(v[e], wr);
    }
}

// Column launch, forward: S[k2][n1] = w_N^(n1 k2) sum_n2 w_N2^(n2 k2) f[n1 + N1 n2].
template <typename R, int N>
__global__ __launch_bounds__(64 * kFsWaves) void k_fs_cols_fwd(const R* __restrict__ f, cpx<R>* __restrict__ S,
                                                                const cpx<double>* __restrict__ twN,
                                                                const cpx<double>* __restrict__ tw2, RowGeom rg,
                                                                ScaleRef sc, int ca, int cb) {
    using SH = fs_shape<N>;
    using LD = fs_lds<R, SH::N2>;
    __shared__ R lds[kFsWaves * SH::PPW2 * LD::SL_COL];
    const int64_t q = blockIdx.x / SH::COL_BLOCKS;
    const int cblk = blockIdx.x % SH::COL_BLOCKS;
    const FsPencil P = fs_pencil<R>(q, rg);
    if (fs_idle<R>(P, sc, ca, cb)) return;   // uniform over the workgroup
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane % SH::PPW2, j = lane / SH::PPW2;
    const int n1 = (cblk * kFsWaves + wave) * SH::PPW2 + p;
    const R* f0 = f + (2 * q) * (int64_t)N;
    const R* f1 = f0 + N;
    cpx<R> v[1][16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int n = n1 + SH::N1 * (j + SH::T2 * e);
        v[0][e] = cpx<R>{P.v0 ? f0[n] : (R)0, P.v1 ? f1[n] : (R)0};
    }
    R* l0 = lds + (wave * SH::PPW2 + p) * LD::SL_COL;
    fft_pencils<R, SH::N2, false, true, tuning<R>::SPLIT, tuning<R>::PRODUCTS, 1, SH::PPW2>(v, j, l0, LD::SL_COL,
                                                                                          tw2);
    fs_twiddle<R, N, false>(v[0], n1, j, twN);
    cpx<R>* Sq = S + q * (int64_t)N;
#pragma unroll
    for (int e = 0; e < 16; ++e) Sq[(j + SH::T2 * e) * SH::N1 + n1] = v[0][e];
}

// Row launch: for each k2, S[k2][.] <- F_N1^-1 (ks^2 F_N1 S[k2][.]), ks the
// signed index of k = k2 + N2 k1 (zero at the Nyquist bin under ZERO).
template <typename R, int N>
__global__ __launch_bounds__(64 * kFsWaves) void k_fs_rows(cpx<R>* __restrict__ S,
                                                            const cpx<double>* __restrict__ tw1, RowGeom rg,
                                                            ScaleRef sc, int ca, int cb, int nyq_zero) {
    using SH = fs_shape<N>;
    using LD = fs_lds<R, SH::N1>;
    __shared__ R lds[kFsWaves * SH::PPW1 * LD::SL_ROW];
    const int64_t q = blockIdx.x / SH::ROW_BLOCKS;
    const int rblk = blockIdx.x % SH::ROW_BLOCKS;
    const FsPencil P = fs_pencil<R>(q, rg);
    if (fs_idle<R>(P, sc, ca, cb)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane % SH::T1, p = lane / SH::T1;
    const int k2 = (rblk * kFsWaves + wave) * SH::PPW1 + p;
    cpx<R>* row = S + q * (int64_t)N + (int64_t)k2 * SH::N1;
    cpx<R> v[1][16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[0][e] = row[j + SH::T1 * e];
    R* l0 = lds + (wave * SH::PPW1 + p) * LD::SL_ROW;
    fft_pencils<R, SH::N1, false, true, tuning<R>::SPLIT, tuning<R>::PRODUCTS, 1, 1>(v, j, l0, LD::SL_ROW, tw1);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int k = k2 + SH::N2 * (j + SH::T1 * e);
        const int ks = (k <= N / 2) ? k : k - N;
        R s = (R)(ks * ks);
        if (nyq_zero && k == N / 2) s = (R)0;
        v[0][e].x *= s;
        v[0][e].y *= s;
    }
    fft_pencils<R, SH::N1, true, true, tuning<R>::SPLIT, tuning<R>::PRODUCTS, 1, 1>(v, j, l0, LD::SL_ROW, tw1);
#pragma unroll
    for (int e = 0; e < 16; ++e) row[j + SH::T1 * e] = v[0][e];
}

// Column launch, inverse and update: T f at n = n1 + N1 n2 is the N2-point
// inverse over k2 of w_N^-(n1 k2) S[k2][n1]; g += s T f + p V f.  NEXT: the
// column of g (new) is then transformed forward into S for the next half.
template <typename R, int N, bool NEXT>
__global__ __launch_bounds__(64 * kFsWaves) void k_fs_cols_inv(cpx<R>* __restrict__ S, const R* __restrict__ f,
                                                                const R* __restrict__ V, R* __restrict__ g,
                                                                const cpx<double>* __restrict__ twN,
                                                                const cpx<double>* __restrict__ tw2, RowGeom rg,
                                                                ScaleRef sc, int kcol, int pcol, int ca, int cb) {
    using SH = fs_shape<N>;
    using LD = fs_lds<R, SH::N2>;
    __shared__ R lds[kFsWaves * SH::PPW2 * LD::SL_COL];
    const int64_t q = blockIdx.x / SH::COL_BLOCKS;
    const int cblk = blockIdx.x % SH::COL_BLOCKS;
    const FsPencil P = fs_pencil<R>(q, rg);
    if (fs_idle<R>(P, sc, ca, cb)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane % SH::PPW2, j = lane / SH::PPW2;
    const int n1 = (cblk * kFsWaves + wave) * SH::PPW2 + p;
    cpx<R>* Sq = S + q * (int64_t)N;
    cpx<R> v[1][16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[0][e] = Sq[(j + SH::T2 * e) * SH::N1 + n1];
    fs_twiddle<R, N, true>(v[0], n1, j, twN);
    R* l0 = lds + (wave * SH::PPW2 + p) * LD::SL_COL;
    fft_pencils<R, SH::N2, true, true, tuning<R>::SPLIT, tuning<R>::PRODUCTS, 1, SH::PPW2>(v, j, l0, LD::SL_COL,
                                                                                         tw2);
    const cpx<R> s = {scale_of<R>(sc, P.inst0, kcol), scale_of<R>(sc, P.inst1, kcol)};
    const cpx<R> pv = {scale_of<R>(sc, P.inst0, pcol), scale_of<R>(sc, P.inst1, pcol)};
    const int64_t b0 = (2 * q) * (int64_t)N, b1 = b0 + N;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int n = n1 + SH::N1 * (j + SH::T2 * e);
        cpx<R> gg = {(R)0, (R)0};
        if (P.v0) {
            gg.x = g[b0 + n] + s.x * v[0][e].x + pv.x * load_v(V + b0 + n) * f[b0 + n];
            g[b0 + n] = gg.x;
        }
        if (P.v1) {
            gg.y = g[b1 + n] + s.y * v[0][e].y + pv.y * load_v(V + b1 + n) * f[b1 + n];
            g[b1 + n] = gg.y;
        }
        if constexpr (NEXT) v[0][e] = gg;
    }
    if constexpr (NEXT) {
        // the lane group's reads of its LDS slices above are complete
        fft_pencils<R, SH::N2, false, true, tuning<R>::SPLIT, tuning<R>::PRODUCTS, 1, SH::PPW2>(v, j, l0,
                                                                                              LD::SL_COL, tw2);
        fs_twiddle<R, N, false>(v[0], n1, j, twN);
#pragma unroll
        for (int e = 0; e < 16; ++e) Sq[(j + SH::T2 * e) * SH::N1 + n1] = v[0][e];
    }
}

// s_ready: S already holds the column transforms of psi_I (left by the
// previous pass with fuse_next), so an A half skips its first launch;
// fuse_next: the B half's last launch also transforms psi_I(new) into S for
// the next pass's A half.
template <typename R, int N>
hipError_t fs_pass(R* psiR, R* psiI, const R* V, const cpx<double>* twN, const cpx<double>* tw1,
                   const cpx<double>* tw2, cpx<R>* S, const RowGeom& rg, const ScaleRef& sc, int a, int b,
                   int nyq_zero, bool s_ready, bool fuse_next, hipStream_t st) {
    using SH = fs_shape<N>;
    const int64_t pencils = (rg.nrows + 1) / 2;
    const dim3 cgrid((unsigned)(pencils * SH::COL_BLOCKS)), rgrid((unsigned)(pencils * SH::ROW_BLOCKS));
    const dim3 blk(64 * kFsWaves);
    // the columns whose zero scales mark a pencil that this pass leaves alone
    const int ca = a ? SC_KXA : SC_KXB, cb = (a && b) ? SC_KXB : -1;
    // A half: psi_R += T psi_I + p_A V psi_I;  B half: psi_I += T psi_R + p_B V psi_R
    const R* f = a ? psiI : psiR;
    if (!(a && s_ready))
        hipLaunchKernelGGL((k_fs_cols_fwd<R, N>), cgrid, blk, 0, st, f, S, twN, tw2, rg, sc, ca, cb);
    hipLaunchKernelGGL((k_fs_rows<R, N>), rgrid, blk, 0, st, S, tw1, rg, sc, ca, cb, nyq_zero);
    if (a) {
        // with a B half to follow, this launch also transforms psi_R(new)
        if (b)
            hipLaunchKernelGGL((k_fs_cols_inv<R, N, true>), cgrid, blk, 0, st, S, psiI, V, psiR, twN, tw2, rg,
                               sc, (int)SC_KXA, (int)SC_PA, ca, cb);
        else
            hipLaunchKernelGGL((k_fs_cols_inv<R, N, false>), cgrid, blk, 0, st, S, psiI, V, psiR, twN, tw2, rg,
                               sc, (int)SC_KXA, (int)SC_PA, ca, cb);
        if (!b) return hipGetLastError();
        hipLaunchKernelGGL((k_fs_rows<R, N>), rgrid, blk, 0, st, S, tw1, rg, sc, ca, cb, nyq_zero);
    }
    if (fuse_next)
        hipLaunchKernelGGL((k_fs_cols_inv<R, N, true>), cgrid, blk, 0, st, S, psiR, V, psiI, twN, tw2, rg, sc,
                           (int)SC_KXB, (int)SC_PB, ca, cb);
    else
        hipLaunchKernelGGL((k_fs_cols_inv<R, N, false>), cgrid, blk, 0, st, S, psiR, V, psiI, twN, tw2, rg, sc,
                           (int)SC_KXB, (int)SC_PB, ca, cb);
    return hipGetLastError();
}

}  // namespace

size_t fourstep_scratch_bytes(int64_t n, int64_t nrows, size_t esz) {
    if (!fourstep_ok(n)) return 0;
    return (size_t)((nrows + 1) / 2) * (size_t)n * 2 * esz;
}

template <typename R>
hipError_t launch_x_fourstep(int64_t n, R* psiR, R* psiI, const R* V, const void* twN, const void* tw1,
                             const void* tw2, void* scratch, const RowGeom& rg, const ScaleRef& sc, int a, int b,
                             int nyq_zero, int s_ready, int fuse_next, hipStream_t st) {
    if (!fourstep_ok(n) || rg.nrows < 1 || rg.rows_per_inst != 1 || !scratch) return hipErrorInvalidValue;
    if (!a && !b) return hipSuccess;
    if (fuse_next && !b) return hipErrorInvalidValue;   // only a B half leaves psi_I(new) in registers
    const auto* tN = (const cpx<double>*)twN;
    const auto* t1 = (const cpx<double>*)tw1;
    const auto* t2 = (const cpx<double>*)tw2;
    auto* S = (cpx<R>*)scratch;
    if (n == 8192)
        return fs_pass<R, 8192>(psiR, psiI, V, tN, t1, t2, S, rg, sc, a, b, nyq_zero, s_ready, fuse_next, st);
    return fs_pass<R, 16384>(psiR, psiI, V, tN, t1, t2, S, rg, sc, a, b, nyq_zero, s_ready, fuse_next, st);
}

template hipError_t launch_x_fourstep<double>(int64_t, double*, double*, const double*, const void*, const void*,
                                              const void*, void*, const RowGeom&, const ScaleRef&, int, int, int,
                                              int, int, hipStream_t);
template hipError_t launch_x_fourstep<float>(int64_t, float*, float*, const float*, const void*, const void*,
                                             const void*, void*, const RowGeom&, const ScaleRef&, int, int, int,
                                             int, int, hipStream_t);

}  // namespace spstd
