// Mixed-shape groups of 2D instances: one launch per pass for stacks of
// different shapes.
//
// The batching form advances many independent instances of uneven grid
// sizes.  Instances of one shape sit in one single-shape batch (a member);
// the kernels here run a pass of the stage sequence (Eq. 17-18 with the
// directional passes of passes.hpp) over every member in one persistent
// launch: the grid strides over a table of tiles (member, block of that
// member's own grid), and each tile runs the same pass body as the
// single-shape kernels on that member's fields, with the member's twiddles,
// scales and geometry.  A member's shape selects the body (row and column
// lengths 128, 256 or 512); the switch is uniform over a block.
#include "passes.hpp"

namespace spstd {

bool mix_len_ok(int64_t n) { return n == 128 || n == 256 || n == 512; }

template <typename R, int W, bool J>
constexpr int mix_x_lds() {
    constexpr int a = x_ab_map<R, 128, W, J>::LDS_REALS, b = x_ab_map<R, 256, W, J>::LDS_REALS,
                  c = x_ab_map<R, 512, W, J>::LDS_REALS;
    return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

template <typename R, int W, int P>
constexpr int mix_y_lds() {
    constexpr int a = yz_lds<R, 128, W, P>::REALS, b = yz_lds<R, 256, W, P>::REALS,
                  c = yz_lds<R, 512, W, P>::REALS;
    return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

template <typename R, int W, bool J>
__global__ __launch_bounds__(64 * W) SPSTD_WAVES_ATTR void k_mix_x_ab(const MixMember<R>* __restrict__ mem,
                                                                      const MixTile* __restrict__ tiles,
                                                                      int ntiles, int m, int l, int nyq_zero) {
    __shared__ R lds[mix_x_lds<R, W, J>()];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const MixTile T = tiles[t];
        const MixMember<R>& M = mem[T.member];
        const ScaleRef sc{M.scales, m, l};
        const cpx<double>* tw = (const cpx<double>*)M.twx;
        switch (M.nx) {
            case 128: x_ab_body<R, 128, W, true, J>(T.blk, lds, M.psiR, M.psiI, M.V, tw, M.rg, sc, nyq_zero); break;
            case 256: x_ab_body<R, 256, W, true, J>(T.blk, lds, M.psiR, M.psiI, M.V, tw, M.rg, sc, nyq_zero); break;
            case 512: x_ab_body<R, 512, W, true, J>(T.blk, lds, M.psiR, M.psiI, M.V, tw, M.rg, sc, nyq_zero); break;
            default: break;
        }
    }
}

template <typename R, int W, int P>
__global__ __launch_bounds__(64 * W) SPSTD_WAVES_ATTR void k_mix_axis_acc(const MixMember<R>* __restrict__ mem,
                                                                          const MixTile* __restrict__ tiles,
                                                                          int ntiles, int m, int l, int b_half,
                                                                          int nyq_zero) {
    __shared__ R lds[mix_y_lds<R, W, P>()];
    const int col = b_half ? SC_KYB : SC_KYA;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const MixTile T = tiles[t];
        const MixMember<R>& M = mem[T.member];
        const ScaleRef sc{M.scales, m, l};
        const cpx<double>* tw = (const cpx<double>*)M.twy;
        const R* src = b_half ? M.psiR : M.psiI;
        R* dst = b_half ? M.psiI : M.psiR;
        switch (M.ny) {
            case 128: axis_acc_body<R, 128, W, P>(T.blk, lds, src, dst, tw, M.gy, sc, col, nyq_zero); break;
            case 256: axis_acc_body<R, 256, W, P>(T.blk, lds, src, dst, tw, M.gy, sc, col, nyq_zero); break;
            case 512: axis_acc_body<R, 512, W, P>(T.blk, lds, src, dst, tw, M.gy, sc, col, nyq_zero); break;
            default: break;
        }
    }
}

template <typename R, int W, int P>
__global__ __launch_bounds__(64 * W) SPSTD_WAVES_ATTR void k_mix_axis_ba(const MixMember<R>* __restrict__ mem,
                                                                         const MixTile* __restrict__ tiles,
                                                                         int ntiles, int m, int lB, int lA,
                                                                         int nyq_zero) {
    __shared__ R lds[mix_y_lds<R, W, P>()];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const MixTile T = tiles[t];
        const MixMember<R>& M = mem[T.member];
        const ScaleRef scB{M.scales, m, lB}, scA{M.scales, m, lA};
        const cpx<double>* tw = (const cpx<double>*)M.twy;
        switch (M.ny) {
            case 128:
                axis_ba_body<R, 128, W, P>(T.blk, lds, M.psiR, M.psiI, tw, M.gy, scB, scA, SC_KYB, SC_KYA, nyq_zero);
                break;
            case 256:
                axis_ba_body<R, 256, W, P>(T.blk, lds, M.psiR, M.psiI, tw, M.gy, scB, scA, SC_KYB, SC_KYA, nyq_zero);
                break;
            case 512:
                axis_ba_body<R, 512, W, P>(T.blk, lds, M.psiR, M.psiI, tw, M.gy, scB, scA, SC_KYB, SC_KYA, nyq_zero);
                break;
            default: break;
        }
    }
}

// Tile-per-block forms of the three kernels (grid = number of tiles): the
// same pass bodies, expanded inline for each length.  Expanded this way
// the compiler keeps each length's registers close to its single-shape
// kernel's (FP32 boundary sweep: 168 registers, three waves per SIMD,
// against 256 for the persistent form, whose bodies are device functions
// inside the tile loop).  The persistent forms serve the one-block-per-CU
// schedules.
template <typename R, int P>
constexpr int mix_tile_y_waves() {
    return (sizeof(R) == 4 && P == 1) ? 3 : kMinWaves;
}

#define SPSTD_MIX_TILE_HEAD                                                 \
    const MixTile T = tiles[blockIdx.x];                                    \
    const int mb = __builtin_amdgcn_readfirstlane(T.member);                \
    const int64_t blk = __builtin_amdgcn_readfirstlane(T.blk);              \
    const MixMember<R> M = mem[mb];                                         \
    R* const lds = lds_block;

template <typename R, int W, bool J>
__global__ __launch_bounds__(64 * W) SPSTD_WAVES_ATTR void k_mix_x_ab_tile(const MixMember<R>* __restrict__ mem,
                                                                           const MixTile* __restrict__ tiles,
                                                                           int m, int l, int nyq_zero) {
    __shared__ R lds_block[mix_x_lds<R, W, J>()];
    SPSTD_MIX_TILE_HEAD
    const ScaleRef sc{M.scales, m, l};
    const cpx<double>* __restrict__ tw = (const cpx<double>*)M.twx;
    const RowGeom rg = M.rg;
    R* __restrict__ psiR = M.psiR;
    R* __restrict__ psiI = M.psiI;
    const R* __restrict__ V = M.V;
    constexpr bool FULL = true, JOINT = J;
    constexpr int WPB = W;
    if (M.nx == 128) {
        constexpr int N = 128;
#include "body_x_ab.inc"
    } else if (M.nx == 256) {
        constexpr int N = 256;
#include "body_x_ab.inc"
    } else if (M.nx == 512) {
        constexpr int N = 512;
#include "body_x_ab.inc"
    }
}

template <typename R, int W, int P>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(mix_tile_y_waves<R, P>()))) void
k_mix_axis_acc_tile(const MixMember<R>* __restrict__ mem, const MixTile* __restrict__ tiles, int m, int l,
                    int b_half, int nyq_zero) {
    __shared__ R lds_block[mix_y_lds<R, W, P>()];
    SPSTD_MIX_TILE_HEAD
    const int col = b_half ? SC_KYB : SC_KYA;
    const ScaleRef sc{M.scales, m, l};
    const cpx<double>* __restrict__ tw = (const cpx<double>*)M.twy;
    const AxisGeom g = M.gy;
    const R* __restrict__ src = b_half ? M.psiR : M.psiI;
    R* __restrict__ dst = b_half ? M.psiI : M.psiR;
    constexpr int WPB = W;
    if (M.ny == 128) {
        constexpr int N = 128;
#include "body_axis_acc.inc"
    } else if (M.ny == 256) {
        constexpr int N = 256;
#include "body_axis_acc.inc"
    } else if (M.ny == 512) {
        constexpr int N = 512;
#include "body_axis_acc.inc"
    }
}

template <typename R, int W, int P>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(mix_tile_y_waves<R, P>()))) void
k_mix_axis_ba_tile(const MixMember<R>* __restrict__ mem, const MixTile* __restrict__ tiles, int m, int lB, int lA,
                   int nyq_zero) {
    __shared__ R lds_block[mix_y_lds<R, W, P>()];
    SPSTD_MIX_TILE_HEAD
    const ScaleRef scB{M.scales, m, lB}, scA{M.scales, m, lA};
    const int colB = SC_KYB, colA = SC_KYA;
    const cpx<double>* __restrict__ tw = (const cpx<double>*)M.twy;
    const AxisGeom g = M.gy;
    R* __restrict__ psiR = M.psiR;
    R* __restrict__ psiI = M.psiI;
    constexpr int WPB = W;
    if (M.ny == 128) {
        constexpr int N = 128;
#include "body_axis_ba.inc"
    } else if (M.ny == 256) {
        constexpr int N = 256;
#include "body_axis_ba.inc"
    } else if (M.ny == 512) {
        constexpr int N = 512;
#include "body_axis_ba.inc"
    }
}
#undef SPSTD_MIX_TILE_HEAD

template <typename R>
__global__ void k_mix_probe(const MixMember<R>* __restrict__ mem, const MixTile* __restrict__ slots, int nslots,
                            int nprobes, int part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nslots) return;
    const MixTile ms = slots[i];
    const MixMember<R>& M = mem[ms.member];
    const int s = ms.blk;
    if (!M.active[s]) return;
    const int64_t slot = M.counter[s];
    if (slot < M.samples) {
        double* out = M.probes + ((int64_t)s * M.samples + slot) * nprobes * 2;
        for (int q = 0; q < nprobes; ++q) {
            const int64_t p = M.pidx[(int64_t)s * nprobes + q];
            if (p < 0 || p >= M.npts) {     // skipped, and flagged for the host
                *M.fault = 1;
                continue;
            }
            const int64_t k = (int64_t)s * M.npts + p;
            if (part & PROBE_R) out[2 * q] = (double)M.psiR[k];
            if (part & PROBE_I) out[2 * q + 1] = (double)M.psiI[k];
        }
    }
    if (part & PROBE_I) M.counter[s] = slot + 1;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int64_t mix_blocks(int kind, int nx, int ny, int64_t capacity, int precision_bytes, const MixVariant& v) {
    (void)precision_bytes;
    const int64_t W = v.wpb;
    if (kind == 0) {
        const int64_t ppb = W * (1024 / nx);           // row pairs per block
        const int64_t npen = capacity * ny / 2;
        return (npen + ppb - 1) / ppb;
    }
    const int64_t ppw = 1024 / ny;                     // lane groups per wave
    const int64_t ngroups = (int64_t)(nx / 2 / v.y_ppl) * capacity;
    const int64_t waves = (ngroups + ppw - 1) / ppw;
    return (waves + W - 1) / W;
}

// Calls f with the variant's compile-time parameters.
template <typename F>
static hipError_t with_variant_x(const MixVariant& v, F&& f) {
    if (v.wpb == 2 && !v.x_joint) return f(std::integral_constant<int, 2>{}, std::false_type{});
    if (v.wpb == 2 && v.x_joint) return f(std::integral_constant<int, 2>{}, std::true_type{});
    if (v.wpb == 4 && !v.x_joint) return f(std::integral_constant<int, 4>{}, std::false_type{});
    if (v.wpb == 4 && v.x_joint) return f(std::integral_constant<int, 4>{}, std::true_type{});
    return hipErrorInvalidValue;
}

template <typename F>
static hipError_t with_variant_y(const MixVariant& v, F&& f) {
    if (v.wpb == 2 && v.y_ppl == 1) return f(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{});
    if (v.wpb == 2 && v.y_ppl == 2) return f(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{});
    if (v.wpb == 4 && v.y_ppl == 1) return f(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{});
    if (v.wpb == 4 && v.y_ppl == 2) return f(std::integral_constant<int, 4>{}, std::integral_constant<int, 2>{});
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_mix_x_ab(const MixMember<R>* mem, const MixTile* tiles, int ntiles, int grid, int m, int l,
                           int nyq_zero, const MixVariant& v, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    return with_variant_x(v, [&](auto w, auto j) {
        constexpr int W = decltype(w)::value;
        constexpr bool J = decltype(j)::value;
        if (grid >= ntiles)
            hipLaunchKernelGGL((k_mix_x_ab_tile<R, W, J>), dim3((unsigned)ntiles), dim3(64 * W), 0, st, mem, tiles,
                               m, l, nyq_zero);
        else
            hipLaunchKernelGGL((k_mix_x_ab<R, W, J>), dim3((unsigned)grid), dim3(64 * W), 0, st, mem, tiles, ntiles,
                               m, l, nyq_zero);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t launch_mix_axis_acc(const MixMember<R>* mem, const MixTile* tiles, int ntiles, int grid, int m,
                               int l, int b_half, int nyq_zero, const MixVariant& v, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    return with_variant_y(v, [&](auto w, auto p) {
        constexpr int W = decltype(w)::value;
        constexpr int P = decltype(p)::value;
        if (grid >= ntiles)
            hipLaunchKernelGGL((k_mix_axis_acc_tile<R, W, P>), dim3((unsigned)ntiles), dim3(64 * W), 0, st, mem,
                               tiles, m, l, b_half, nyq_zero);
        else
            hipLaunchKernelGGL((k_mix_axis_acc<R, W, P>), dim3((unsigned)grid), dim3(64 * W), 0, st, mem, tiles,
                               ntiles, m, l, b_half, nyq_zero);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t launch_mix_axis_ba(const MixMember<R>* mem, const MixTile* tiles, int ntiles, int grid, int m,
                              int lB, int lA, int nyq_zero, const MixVariant& v, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    return with_variant_y(v, [&](auto w, auto p) {
        constexpr int W = decltype(w)::value;
        constexpr int P = decltype(p)::value;
        if (grid >= ntiles)
            hipLaunchKernelGGL((k_mix_axis_ba_tile<R, W, P>), dim3((unsigned)ntiles), dim3(64 * W), 0, st, mem,
                               tiles, m, lB, lA, nyq_zero);
        else
            hipLaunchKernelGGL((k_mix_axis_ba<R, W, P>), dim3((unsigned)grid), dim3(64 * W), 0, st, mem, tiles,
                               ntiles, m, lB, lA, nyq_zero);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t launch_mix_probe(const MixMember<R>* mem, const MixTile* slots, int nslots, int nprobes,
                            hipStream_t st, int part) {
    if (part < PROBE_R || part > PROBE_FULL) return hipErrorInvalidValue;
    if (nslots <= 0 || nprobes <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_mix_probe<R>), dim3((unsigned)((nslots + 63) / 64)), dim3(64), 0, st, mem, slots, nslots,
                       nprobes, part);
    return hipGetLastError();
}

#define SPSTD_INST_MIX(R)                                                                                   \
    template hipError_t launch_mix_x_ab<R>(const MixMember<R>*, const MixTile*, int, int, int, int, int,   \
                                           const MixVariant&, hipStream_t);                                \
    template hipError_t launch_mix_axis_acc<R>(const MixMember<R>*, const MixTile*, int, int, int, int,    \
                                               int, int, const MixVariant&, hipStream_t);                  \
    template hipError_t launch_mix_axis_ba<R>(const MixMember<R>*, const MixTile*, int, int, int, int,     \
                                              int, int, const MixVariant&, hipStream_t);                   \
    template hipError_t launch_mix_probe<R>(const MixMember<R>*, const MixTile*, int, int, hipStream_t, int);
SPSTD_INST_MIX(double)
SPSTD_INST_MIX(float)
#undef SPSTD_INST_MIX

}  // namespace spstd
