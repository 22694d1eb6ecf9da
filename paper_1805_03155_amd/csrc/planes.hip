// Fused z and x passes of a stage on x-z planes (3D batches with small x
// and z extents).
//
// In the stage sequence of Eq. (17)-(18) the A half ends with its z and x
// terms and the B half starts with its x and z terms; the y terms of both
// halves come from the y sweeps before and after (the boundary sweep).  On
// a plane of fixed y, z pencils and x rows both lie inside the plane, so
// one workgroup holding the plane's psi_R and psi_I in LDS applies, in
// order,
//   z(A): psi_R += kz_A T_z psi_I
//   x(A): psi_R += kx_A T_x psi_I + p_A V psi_I
//   x(B): psi_I += kx_B T_x psi_R + p_B V psi_R      (psi_R now complete)
//   z(B): psi_I += kz_B T_z psi_R
// (the A or the B part alone where the stage has one half), with workgroup
// barriers between the phases, and writes the plane back: one launch and
// one read and write of the fields (plus V) in place of the three passes
// z(A), x(A+B), z(B).  A lane group of N/16 lanes holds two pencils half
// the plane apart (rows q and q + NZ/2 along x; columns q and q + NX/2
// along z) as one complex pencil, the pencil index fastest over the lanes,
// so the transform's last pass runs on lane swaps (16-, 32- and 64-point
// pencils).  The plane's LDS rows are NX + 1 elements apart: the lanes of a
// phase then read different banks along either axis (with neighbouring rows
// paired and rows NX apart, the x phases read one bank sixteen ways).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "passes.hpp"

namespace spstd {

bool plane_ok(int64_t nx, int64_t nz) {
    auto ok = [](int64_t n) { return n == 16 || n == 32 || n == 64; };
    return ok(nx) && ok(nz);
}

template <int NX, int NZ>
struct plane_cfg {
    static constexpr int NPL = NX * NZ;                        // points of a plane
    // square planes transform their x rows and z columns in one phase
    static constexpr bool BOTH = NX == NZ;
    static constexpr int LANES = BOTH ? NPL / 16 : NPL / 32;   // lanes of a phase
    static constexpr int THREADS = LANES < 64 ? 64 : LANES;    // whole waves (lane swaps)
    // LDS row stride: odd, so that the lanes of an x phase (one row each)
    // and of a z phase (one column each) fall on different banks
    static constexpr int S = NX + 1;
    static constexpr int LDS = NZ * S;
};

// One phase: g += kin T f (+ pot V f along x) over the plane's pencils of
// the axis (x rows or z columns); f and g in LDS (element (z, x) at z S + x),
// V the plane's potential in global memory (row z at z * vstride).  Lane
// group q carries rows q and q + NZ/2 (along x) or columns q and q + NX/2
// (along z) as one complex pencil: neighbouring lane groups read
// neighbouring rows or columns, which the odd row stride puts on different
// banks.
template <typename R, int N, bool ALONG_X, int NX, int NZ>
__device__ __forceinline__ void plane_phase(const R* f, R* g, const R* __restrict__ V, int64_t vstride, R kin,
                                            R pot, int nyq_zero, const cpx<double>* __restrict__ tw) {
    constexpr int T = N / 16, PPW = 64 / T;
    constexpr int S = plane_cfg<NX, NZ>::S;
    constexpr int PAIRS = (ALONG_X ? NZ : NX) / 2;
    static_assert(N == 16 || tail_swaps<N, PPW>::OK, "the last pass must run on lane swaps");
    static_assert(PAIRS * T <= plane_cfg<NX, NZ>::THREADS, "one pass over the plane's pencils");
    constexpr int STRIDE = ALONG_X ? 1 : S;          // between a pencil's points
    constexpr int OFF = ALONG_X ? PAIRS * S : PAIRS; // to the pencil's partner
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane % PPW, j = lane / PPW;
    const int q = wave * PPW + p;
    const bool on = q < PAIRS;
    const int base = ALONG_X ? q * S : q;
    cpx<R> v[1][16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = base + (j + T * e) * STRIDE;
        v[0][e] = on ? cpx<R>{f[i], f[i + OFF]} : cpx<R>{(R)0, (R)0};
    }
    fft_pencils<R, N, false, true, true, true, 1, PPW>(v, j, nullptr, 0, tw);
    apply_k2<R, N>(v[0], j, nyq_zero);
    fft_pencils<R, N, true, true, true, true, 1, PPW>(v, j, nullptr, 0, tw);
    if (!on) return;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = base + (j + T * e) * STRIDE;
        if constexpr (ALONG_X) {
            // rows q and q + NZ/2 at x = j + T e
            const int x = j + T * e, z0 = q, z1 = q + PAIRS;
            const R v0 = V[z0 * vstride + x], v1 = V[z1 * vstride + x];
            g[i] = g[i] + kin * v[0][e].x + pot * v0 * f[i];
            g[i + OFF] = g[i + OFF] + kin * v[0][e].y + pot * v1 * f[i + OFF];
        } else {
            g[i] = g[i] + kin * v[0][e].x;
            g[i + OFF] = g[i + OFF] + kin * v[0][e].y;
        }
    }
}

// Both axes of one half on a square plane: g += kx T_x f + pot V f + kz T_z f.
// The x and z terms read the same f, so lane groups q < N/2 transform the z
// column pairs (q, q + N/2) and the others the x row pairs (q - N/2, q) in
// one call; the x lanes add their terms to g first, the z lanes after a
// workgroup barrier.
template <typename R, int N>
__device__ __forceinline__ void plane_phase_both(const R* f, R* g, const R* __restrict__ V, int64_t vstride, R kx,
                                                 R kz, R pot, int nyq_zero, const cpx<double>* __restrict__ tw) {
    constexpr int T = N / 16, PPW = 64 / T;
    constexpr int S = plane_cfg<N, N>::S;
    constexpr int H = N / 2;
    static_assert(N == 16 || tail_swaps<N, PPW>::OK, "the last pass must run on lane swaps");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane % PPW, j = lane / PPW;
    const int q = wave * PPW + p;
    const bool on = q < N;
    const bool along_x = q >= H;
    const int qq = along_x ? q - H : q;
    const int stride = along_x ? 1 : S;            // between a pencil's points
    const int off = along_x ? H * S : H;           // to the pencil's partner
    const int base = along_x ? qq * S : qq;
    cpx<R> v[1][16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = base + (j + T * e) * stride;
        v[0][e] = on ? cpx<R>{f[i], f[i + off]} : cpx<R>{(R)0, (R)0};
    }
    fft_pencils<R, N, false, true, true, true, 1, PPW>(v, j, nullptr, 0, tw);
    apply_k2<R, N>(v[0], j, nyq_zero);
    fft_pencils<R, N, true, true, true, true, 1, PPW>(v, j, nullptr, 0, tw);
    if (on && along_x) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            // rows qq and qq + N/2 at x = j + T e; V row z starts at z * vstride
            const int x = j + T * e, i = base + x;
            const R v0 = V[qq * vstride + x], v1 = V[(qq + H) * vstride + x];
            g[i] = g[i] + kx * v[0][e].x + pot * v0 * f[i];
            g[i + off] = g[i + off] + kx * v[0][e].y + pot * v1 * f[i + off];
        }
    }
    __syncthreads();
    if (on && !along_x) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = base + (j + T * e) * S;
            g[i] = g[i] + kz * v[0][e].x;
            g[i + off] = g[i + off] + kz * v[0][e].y;
        }
    }
}

// Block b: instance b / ny, plane y = b % ny.  do_a, do_b: which halves
// of stage sc.l the launch applies (uniform).
template <typename R, int NX, int NZ>
__global__ __launch_bounds__((plane_cfg<NX, NZ>::THREADS)) void k_plane_zxz(
    R* __restrict__ psiR, R* __restrict__ psiI, const R* __restrict__ V, int64_t ny, ScaleRef sc, int do_a,
    int do_b, int nyq_zero, const cpx<double>* __restrict__ twx, const cpx<double>* __restrict__ twz) {
    using C = plane_cfg<NX, NZ>;
    __shared__ R sR[C::LDS];
    __shared__ R sI[C::LDS];
    const int64_t inst = blockIdx.x / ny, y = blockIdx.x % ny;
    const R kza = do_a ? scale_of<R>(sc, inst, SC_KZA) : (R)0, kxa = do_a ? scale_of<R>(sc, inst, SC_KXA) : (R)0;
    const R pa = do_a ? scale_of<R>(sc, inst, SC_PA) : (R)0;
    const R kzb = do_b ? scale_of<R>(sc, inst, SC_KZB) : (R)0, kxb = do_b ? scale_of<R>(sc, inst, SC_KXB) : (R)0;
    const R pb = do_b ? scale_of<R>(sc, inst, SC_PB) : (R)0;
    // a free slot (zero scales) stays as it is; uniform over the workgroup
    if (kza == (R)0 && kxa == (R)0 && pa == (R)0 && kzb == (R)0 && kxb == (R)0 && pb == (R)0) return;
    const int64_t zstride = (int64_t)NX * ny;                       // between the plane's rows
    const int64_t off = inst * (int64_t)NZ * zstride + y * NX;      // element (z, x) at off + z * zstride + x
    for (int k = threadIdx.x; k < C::NPL; k += C::THREADS) {
        const int z = k / NX, x = k % NX;
        const int64_t gi = off + z * zstride + x;
        sR[z * C::S + x] = psiR[gi];
        sI[z * C::S + x] = psiI[gi];
    }
    const R* Vp = V + off;
    __syncthreads();
    if constexpr (C::BOTH) {
        // the x and z transforms of a half in one phase (x and z tables of
        // one length are the same table)
        if (do_a) {
            plane_phase_both<R, NX>(sI, sR, Vp, zstride, kxa, kza, pa, nyq_zero, twx);
            __syncthreads();
        }
        if (do_b) {
            plane_phase_both<R, NX>(sR, sI, Vp, zstride, kxb, kzb, pb, nyq_zero, twx);
            __syncthreads();
        }
    } else {
        if (do_a) {
            plane_phase<R, NZ, false, NX, NZ>(sI, sR, Vp, zstride, kza, (R)0, nyq_zero, twz);
            __syncthreads();
            plane_phase<R, NX, true, NX, NZ>(sI, sR, Vp, zstride, kxa, pa, nyq_zero, twx);
            __syncthreads();
        }
        if (do_b) {
            plane_phase<R, NX, true, NX, NZ>(sR, sI, Vp, zstride, kxb, pb, nyq_zero, twx);
            __syncthreads();
            plane_phase<R, NZ, false, NX, NZ>(sR, sI, Vp, zstride, kzb, (R)0, nyq_zero, twz);
            __syncthreads();
        }
    }
    for (int k = threadIdx.x; k < C::NPL; k += C::THREADS) {
        const int z = k / NX, x = k % NX;
        const int64_t gi = off + z * zstride + x;
        psiR[gi] = sR[z * C::S + x];
        psiI[gi] = sI[z * C::S + x];
    }
}

template <typename R, int NX, int NZ>
static hipError_t plane_n(R* psiR, R* psiI, const R* V, int64_t ny, int64_t ninst, const ScaleRef& sc, int do_a,
                          int do_b, int nyq_zero, const void* twx, const void* twz, hipStream_t st) {
    hipLaunchKernelGGL((k_plane_zxz<R, NX, NZ>), dim3((unsigned)(ninst * ny)), dim3(plane_cfg<NX, NZ>::THREADS), 0,
                       st, psiR, psiI, V, ny, sc, do_a, do_b, nyq_zero, (const cpx<double>*)twx,
                       (const cpx<double>*)twz);
    return hipGetLastError();
}

template <typename R, int NX>
static hipError_t plane_z(int64_t nz, R* psiR, R* psiI, const R* V, int64_t ny, int64_t ninst, const ScaleRef& sc,
                          int do_a, int do_b, int nyq_zero, const void* twx, const void* twz, hipStream_t st) {
    switch (nz) {
        case 16: return plane_n<R, NX, 16>(psiR, psiI, V, ny, ninst, sc, do_a, do_b, nyq_zero, twx, twz, st);
        case 32: return plane_n<R, NX, 32>(psiR, psiI, V, ny, ninst, sc, do_a, do_b, nyq_zero, twx, twz, st);
        case 64: return plane_n<R, NX, 64>(psiR, psiI, V, ny, ninst, sc, do_a, do_b, nyq_zero, twx, twz, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_plane_zxz(int64_t nx, int64_t ny, int64_t nz, int64_t ninst, R* psiR, R* psiI, const R* V,
                            const ScaleRef& sc, int do_a, int do_b, int nyq_zero, const void* twx, const void* twz,
                            hipStream_t st) {
    if (!plane_ok(nx, nz) || ny < 1 || ninst < 1 || ninst * ny > 0x7fffffff) return hipErrorInvalidValue;
    if (!do_a && !do_b) return hipSuccess;
    switch (nx) {
        case 16: return plane_z<R, 16>(nz, psiR, psiI, V, ny, ninst, sc, do_a, do_b, nyq_zero, twx, twz, st);
        case 32: return plane_z<R, 32>(nz, psiR, psiI, V, ny, ninst, sc, do_a, do_b, nyq_zero, twx, twz, st);
        case 64: return plane_z<R, 64>(nz, psiR, psiI, V, ny, ninst, sc, do_a, do_b, nyq_zero, twx, twz, st);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_plane_zxz<double>(int64_t, int64_t, int64_t, int64_t, double*, double*, const double*,
                                             const ScaleRef&, int, int, int, const void*, const void*, hipStream_t);
template hipError_t launch_plane_zxz<float>(int64_t, int64_t, int64_t, int64_t, float*, float*, const float*,
                                            const ScaleRef&, int, int, int, const void*, const void*, hipStream_t);

}  // namespace spstd
