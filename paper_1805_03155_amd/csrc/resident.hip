// Resident 1D kernel: whole runs of short 1D instances in one launch.
//
// A lane group (T = N/16 lanes) keeps two instances of the same length N in
// registers for every step of the launch: instance a in the real parts and
// instance b in the imaginary parts of the complex arrays PR (psi_R) and PI
// (psi_I).  The kinetic operator T = IFFT(s(k) FFT(.)) has a real, even
// symbol, so T(f_a + i f_b) = T f_a + i T f_b; the transform applies the bare
// k^2 (bin index squared) and each instance's own scale
// c dt (hbar/2m*) (2 pi / L)^2 / N is applied after the inverse transform,
// which lets instances with different dt, L and V share a pencil.
//
// Substep of stage l (Eq. 17-18, A before B):
//   A: PR += kin_A * T PI + pot_A * V * PI      (kin_A from c_l dt, pot_A = c_l dt / hbar)
//   B: PI += kin_B * T PR + pot_B * V * PR      (kin_B, pot_B from -d_l dt)
// After every step each instance's probe samples (FP64) are written.
//
// Up to N = 4096 the state lives in registers.  Longer grids (GS: global
// state) keep psi_R and psi_I in the instances' own arrays -- each row is
// touched only by its own workgroup, so it stays in cache -- and read and
// write them around every substep, ordered by workgroup barriers; the step
// loop still runs inside one launch.
#include "fft_core.hpp"
#include "resident.hpp"

namespace spstd {

template <int N>
struct res_cfg {
    static constexpr int T = N / 16;
    static constexpr bool WAVE = T <= 64;
    static constexpr int GPW = WAVE ? 64 / T : 1;     // lane groups per wave
    static constexpr int WPB = WAVE ? 2 : 1;           // waves per block (wave-local groups)
    static constexpr int THREADS = WAVE ? 64 * WPB : T;
    static constexpr int GPB = WAVE ? WPB * GPW : 1;   // lane groups per block
    static constexpr int LS = lds_size<N>::value;
    static constexpr int LDS_REALS = N == 16 ? 1 : GPB * LS;   // split exchange
};

template <typename R, int N>
__device__ __forceinline__ void k2_symbol(cpx<R> (&v)[16], int j, int nyq_zero) {
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

template <typename R, int N, bool GS>
__global__ __launch_bounds__((res_cfg<N>::THREADS)) void k_resident_1d(
    const ResidentInst<R>* __restrict__ inst, int ninst, int m, int64_t nsteps, int nyq_zero,
    const cpx<double>* __restrict__ tw) {
    using C = res_cfg<N>;
    __shared__ R lds[C::LDS_REALS];
    int j, gib;
    if constexpr (C::WAVE) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        j = lane % C::T;
        gib = wave * C::GPW + lane / C::T;
    } else {
        j = threadIdx.x;
        gib = 0;
    }
    const int g = blockIdx.x * C::GPB + gib;
    const int ia = 2 * g, ib = 2 * g + 1;
    const bool ha = ia < ninst, hb = ib < ninst;
    // lanes of a group with no instance still take part in the exchanges
    const ResidentInst<R>* A = ha ? inst + ia : inst;
    const ResidentInst<R>* B = hb ? inst + ib : A;
    R* l0 = lds + (N == 16 ? 0 : gib * C::LS);
    const R* Va = A->V;
    const R* Vb = B->V;
    const int64_t slot_a = ha ? *A->counter : 0;
    const int64_t slot_b = hb ? *B->counter : 0;

    if constexpr (!GS) {
        cpx<R> PR[16], PI[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int x = j + C::T * e;
            PR[e] = cpx<R>{ha ? A->psiR[x] : (R)0, hb ? B->psiR[x] : (R)0};
            PI[e] = cpx<R>{ha ? A->psiI[x] : (R)0, hb ? B->psiI[x] : (R)0};
        }
        for (int64_t s = 0; s < nsteps; ++s) {
            for (int l = 0; l < m; ++l) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const R ka = ha ? A->kin[2 * l + half] : (R)0, kb = hb ? B->kin[2 * l + half] : (R)0;
                    const R pa = ha ? A->pot[2 * l + half] : (R)0, pb = hb ? B->pot[2 * l + half] : (R)0;
                    if (ka == (R)0 && kb == (R)0 && pa == (R)0 && pb == (R)0) continue;   // uniform
                    cpx<R>(&src)[16] = half == 0 ? PI : PR;
                    cpx<R>(&dst)[16] = half == 0 ? PR : PI;
                    cpx<R> v[1][16];
#pragma unroll
                    for (int e = 0; e < 16; ++e) v[0][e] = src[e];
                    fft_pencils<R, N, false, C::WAVE, true, true, 1, 1>(v, j, l0, C::LS, tw);
                    k2_symbol<R, N>(v[0], j, nyq_zero);
                    fft_pencils<R, N, true, C::WAVE, true, true, 1, 1>(v, j, l0, C::LS, tw);
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int x = j + C::T * e;
                        const R va = Va[x], vb = Vb[x];
                        dst[e].x += ka * v[0][e].x + pa * va * src[e].x;
                        dst[e].y += kb * v[0][e].y + pb * vb * src[e].y;
                    }
                }
            }
            // probe samples of this step
#pragma unroll
            for (int who = 0; who < 2; ++who) {
                const bool has = who == 0 ? ha : hb;
                const ResidentInst<R>* I = who == 0 ? A : B;
                if (!has) continue;
                for (int q = 0; q < I->nprobes; ++q) {
                    const int64_t pidx = I->probe_idx[q];
                    if (pidx < 0 || pidx >= N) {      // skipped, flagged for the host
                        if (j == 0) *I->fault = 1;
                        continue;
                    }
                    if ((int)(pidx % C::T) != j) continue;
                    const int pe = (int)(pidx / C::T);
                    R r = (R)0, im = (R)0;
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        if (e == pe) {
                            r = who == 0 ? PR[e].x : PR[e].y;
                            im = who == 0 ? PI[e].x : PI[e].y;
                        }
                    }
                    const int64_t slot = (who == 0 ? slot_a : slot_b) + s;
                    if (slot < I->capacity) {
                        I->probes[(slot * I->nprobes + q) * 2 + 0] = (double)r;
                        I->probes[(slot * I->nprobes + q) * 2 + 1] = (double)im;
                    }
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int x = j + C::T * e;
            if (ha) { A->psiR[x] = PR[e].x; A->psiI[x] = PI[e].x; }
            if (hb) { B->psiR[x] = PR[e].y; B->psiI[x] = PI[e].y; }
        }
    } else {
        // global state: every substep reads its source and destination rows
        for (int64_t s = 0; s < nsteps; ++s) {
            for (int l = 0; l < m; ++l) {
                for (int half = 0; half < 2; ++half) {
                    const R ka = ha ? A->kin[2 * l + half] : (R)0, kb = hb ? B->kin[2 * l + half] : (R)0;
                    const R pa = ha ? A->pot[2 * l + half] : (R)0, pb = hb ? B->pot[2 * l + half] : (R)0;
                    if (ka == (R)0 && kb == (R)0 && pa == (R)0 && pb == (R)0) continue;   // uniform
                    const R* sa = half == 0 ? A->psiI : A->psiR;
                    const R* sb = half == 0 ? B->psiI : B->psiR;
                    R* da = half == 0 ? A->psiR : A->psiI;
                    R* db = half == 0 ? B->psiR : B->psiI;
                    cpx<R> v[1][16];
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int x = j + C::T * e;
                        v[0][e] = cpx<R>{ha ? sa[x] : (R)0, hb ? sb[x] : (R)0};
                    }
                    fft_pencils<R, N, false, C::WAVE, true, true, 1, 1>(v, j, l0, C::LS, tw);
                    k2_symbol<R, N>(v[0], j, nyq_zero);
                    fft_pencils<R, N, true, C::WAVE, true, true, 1, 1>(v, j, l0, C::LS, tw);
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int x = j + C::T * e;
                        if (ha) da[x] = da[x] + ka * v[0][e].x + pa * Va[x] * sa[x];
                        if (hb) db[x] = db[x] + kb * v[0][e].y + pb * Vb[x] * sb[x];
                    }
                    // the next substep reads what other lanes of the group wrote
                    __threadfence_block();
                    if constexpr (C::WAVE) lds_sync<true>(); else __syncthreads();
                }
            }
#pragma unroll
            for (int who = 0; who < 2; ++who) {
                const bool has = who == 0 ? ha : hb;
                const ResidentInst<R>* I = who == 0 ? A : B;
                if (!has || j != 0) continue;
                const int64_t slot = (who == 0 ? slot_a : slot_b) + s;
                for (int q = 0; q < I->nprobes && slot < I->capacity; ++q) {
                    const int64_t pidx = I->probe_idx[q];
                    if (pidx < 0 || pidx >= N) {
                        *I->fault = 1;
                        continue;
                    }
                    I->probes[(slot * I->nprobes + q) * 2 + 0] = (double)I->psiR[pidx];
                    I->probes[(slot * I->nprobes + q) * 2 + 1] = (double)I->psiI[pidx];
                }
            }
        }
    }
    // every lane of the group has read the counters before lane 0 advances them
    if constexpr (C::WAVE) {
        lds_sync<true>();
    } else {
        __syncthreads();
    }
    if (j == 0) {
        if (ha) *A->counter = slot_a + nsteps;
        if (hb) *B->counter = slot_b + nsteps;
    }
}

// ---------------------------------------------------------------------------
// Resident 2D kernel: one workgroup per instance of NX by NY points (x
// fastest), psi_R and psi_I in LDS for the whole launch.  A substep is
//   g += kin_x T_x f + pot V f   (x phase: lane groups on row pairs 2q, 2q+1
//                                 packed as one complex pencil)
//   g += kin_y T_y f             (y phase: lane groups on column pairs)
// with f the source and g the destination field of Eq. (18) (A: f = psi_I,
// g = psi_R; B: f = psi_R, g = psi_I, kin and pot from -d_l dt), each phase
// a forward transform, the bare k^2 (bin index squared) and an inverse
// transform along its axis, separated by workgroup barriers.  f is not
// written within a substep; every element of g is written by one lane per
// phase.  After every step thread 0 records the probe samples (FP64).
// ---------------------------------------------------------------------------
template <int NX, int NY>
struct res2_cfg {
    static constexpr int TX = NX / 16, TY = NY / 16;   // lanes per pencil
    static constexpr int NPT = NX * NY;
    static constexpr int LANES = NPT / 32;             // lanes busy in either phase
    static constexpr int THREADS = LANES < 64 ? 64 : LANES;
    static constexpr int GX = THREADS / TX, GY = THREADS / TY;   // lane groups per phase
    static constexpr int SX = NX == 16 ? 0 : GX * lds_size<NX>::value;
    static constexpr int SY = NY == 16 ? 0 : GY * lds_size<NY>::value;
    static constexpr int SCR = (SX > SY ? SX : SY) > 0 ? (SX > SY ? SX : SY) : 1;
};

template <typename R, int NX, int NY>
__global__ __launch_bounds__((res2_cfg<NX, NY>::THREADS)) void k_resident_2d(
    const ResidentInst<R>* __restrict__ inst, int ninst, int m, int64_t nsteps, int nyq_zero,
    const cpx<double>* __restrict__ twx, const cpx<double>* __restrict__ twy) {
    using C = res2_cfg<NX, NY>;
    __shared__ R sR[C::NPT];
    __shared__ R sI[C::NPT];
    __shared__ R scr[C::SCR];
    if ((int)blockIdx.x >= ninst) return;   // uniform over the workgroup
    const ResidentInst<R>* I = inst + blockIdx.x;
    const int t = threadIdx.x;
    for (int k = t; k < C::NPT; k += C::THREADS) {
        sR[k] = I->psiR[k];
        sI[k] = I->psiI[k];
    }
    const R* __restrict__ V = I->V;
    const int64_t slot0 = *I->counter;
    // x phase: row pair qx, position jx; y phase: column pair qy, position jy
    const int jx = t % C::TX, qx = t / C::TX;
    const int jy = t % C::TY, qy = t / C::TY;
    const bool hx = qx < NY / 2, hy = qy < NX / 2;
    R* lx = scr + (NX == 16 ? 0 : qx * lds_size<NX>::value);
    R* ly = scr + (NY == 16 ? 0 : qy * lds_size<NY>::value);
    __syncthreads();
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int l = 0; l < m; ++l) {
            for (int half = 0; half < 2; ++half) {
                const R kx = I->kin[2 * l + half], ky = I->kin_y[2 * l + half], pt = I->pot[2 * l + half];
                if (kx == (R)0 && ky == (R)0 && pt == (R)0) continue;   // uniform
                const R* f = half == 0 ? sI : sR;
                R* g = half == 0 ? sR : sI;
                cpx<R> v[1][16];
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int k0 = 2 * qx * NX + jx + C::TX * e;
                    v[0][e] = hx ? cpx<R>{f[k0], f[k0 + NX]} : cpx<R>{(R)0, (R)0};
                }
                fft_pencils<R, NX, false, true, true, true, 1, 1>(v, jx, lx, lds_size<NX>::value, twx);
                k2_symbol<R, NX>(v[0], jx, nyq_zero);
                fft_pencils<R, NX, true, true, true, true, 1, 1>(v, jx, lx, lds_size<NX>::value, twx);
                if (hx) {
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int k0 = 2 * qx * NX + jx + C::TX * e, k1 = k0 + NX;
                        g[k0] += kx * v[0][e].x + pt * V[k0] * f[k0];
                        g[k1] += kx * v[0][e].y + pt * V[k1] * f[k1];
                    }
                }
                __syncthreads();
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int k0 = (jy + C::TY * e) * NX + 2 * qy;
                    v[0][e] = hy ? cpx<R>{f[k0], f[k0 + 1]} : cpx<R>{(R)0, (R)0};
                }
                fft_pencils<R, NY, false, true, true, true, 1, 1>(v, jy, ly, lds_size<NY>::value, twy);
                k2_symbol<R, NY>(v[0], jy, nyq_zero);
                fft_pencils<R, NY, true, true, true, true, 1, 1>(v, jy, ly, lds_size<NY>::value, twy);
                if (hy) {
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int k0 = (jy + C::TY * e) * NX + 2 * qy;
                        g[k0] += ky * v[0][e].x;
                        g[k0 + 1] += ky * v[0][e].y;
                    }
                }
                __syncthreads();
            }
        }
        if (t == 0) {
            const int64_t slot = slot0 + s;
            for (int q = 0; q < I->nprobes && slot < I->capacity; ++q) {
                const int64_t pidx = I->probe_idx[q];
                if (pidx < 0 || pidx >= NX * NY) {
                    *I->fault = 1;
                    continue;
                }
                I->probes[(slot * I->nprobes + q) * 2 + 0] = (double)sR[pidx];
                I->probes[(slot * I->nprobes + q) * 2 + 1] = (double)sI[pidx];
            }
        }
        // the next step writes the fields thread 0 has just sampled
        __syncthreads();
    }
    for (int k = t; k < C::NPT; k += C::THREADS) {
        I->psiR[k] = sR[k];
        I->psiI[k] = sI[k];
    }
    if (t == 0) *I->counter = slot0 + nsteps;
}

// ---------------------------------------------------------------------------
// Resident 3D kernel: one workgroup per instance of NX x NY x NZ points, a
// whole step chunk per launch (16^3 grids; at 32^3 one workgroup per
// instance is latency-bound: 611 against 126 us per step of the pass
// kernels, while at 16^3 it takes 67 against 120 us in FP64).  The
// fields are too large for LDS and stay in the instance's own arrays; only
// this workgroup touches them, so they stay in its cache.  A substep is
// three phases
//   g += kin_x T_x f + pot V f,   g += kin_y T_y f,   g += kin_z T_z f
// (A: f = psi_I, g = psi_R; B: f = psi_R, g = psi_I, kin and pot from
// -d_l dt), separated by workgroup barriers.  f is not written within a
// substep and every element of g is written by one lane per phase.  A lane
// group of N/16 lanes holds two neighbouring pencils as one complex pencil
// (rows 2q, 2q+1 along x; columns 2q, 2q+1 along y and z), with the pencil
// index fastest over the lanes, so that the transform's last pass runs on
// lane swaps and the kernel needs no LDS.  After every step thread 0
// records the probe samples (FP64).
// ---------------------------------------------------------------------------
template <typename R, int NX, int NY, int NZ>
struct res3_cfg {
    static constexpr int NPT = NX * NY * NZ;
    static constexpr int LANES = NPT / 32;                 // lanes one phase needs (any axis)
    // at most 8 waves: the transforms need more than the 128 registers a
    // lane has with 16 waves per CU
    static constexpr int THREADS = LANES > 512 ? 512 : LANES;
};

bool resident3d_ok(int64_t nx, int64_t ny, int64_t nz) { return nx == 16 && ny == 16 && nz == 16; }

template <typename R, int N, int AX, int NX, int NY, int NZ>
__device__ __forceinline__ void res3_phase(const R* __restrict__ f, R* __restrict__ g, const R* __restrict__ V,
                                           R kin, R pot, int nyq_zero, const cpx<double>* __restrict__ tw) {
    using C = res3_cfg<R, NX, NY, NZ>;
    constexpr int T = N / 16, PPW = 64 / T;
    constexpr int PAIRS = C::NPT / (2 * N);
    constexpr int GROUPS = C::THREADS / T;
    static_assert(N == 16 || tail_swaps<N, PPW>::OK, "the last pass must run on lane swaps");
    static_assert(PAIRS % GROUPS == 0, "whole waves per phase");
    constexpr int STRIDE = AX == 0 ? 1 : AX == 1 ? NX : NX * NY;   // between a pencil's points
    constexpr int OFF = AX == 0 ? NX : 1;                           // to the pencil's partner
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane % PPW, j = lane / PPW;
#pragma unroll 1
    for (int q0 = 0; q0 < PAIRS; q0 += GROUPS) {
        const int q = q0 + wave * PPW + p;
        int base;
        if constexpr (AX == 0) {
            base = 2 * q * NX;
        } else if constexpr (AX == 1) {
            base = (q / (NX / 2)) * NX * NY + 2 * (q % (NX / 2));
        } else {
            base = (q / (NX / 2)) * NX + 2 * (q % (NX / 2));
        }
        cpx<R> v[1][16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = base + (j + T * e) * STRIDE;
            const R a = f[i], b = f[i + OFF];
            v[0][e] = cpx<R>{a, b};
            if constexpr (AX == 0) {
                // the potential term now, so that f need not stay in
                // registers through the transforms
                g[i] += pot * V[i] * a;
                g[i + OFF] += pot * V[i + OFF] * b;
            }
            // a few elements' loads in flight at a time (registers)
            if ((e + 1) % 4 == 0) __builtin_amdgcn_sched_barrier(0);
        }
        fft_pencils<R, N, false, true, true, true, 1, PPW>(v, j, nullptr, 0, tw);
        k2_symbol<R, N>(v[0], j, nyq_zero);
        fft_pencils<R, N, true, true, true, true, 1, PPW>(v, j, nullptr, 0, tw);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = base + (j + T * e) * STRIDE;
            g[i] += kin * v[0][e].x;
            g[i + OFF] += kin * v[0][e].y;
            if ((e + 1) % 4 == 0) __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <typename R, int NX, int NY, int NZ>
__global__ __launch_bounds__((res3_cfg<R, NX, NY, NZ>::THREADS)) void k_resident_3d(
    const ResidentInst<R>* __restrict__ inst, int ninst, int m, int64_t nsteps, int nyq_zero,
    const cpx<double>* __restrict__ twx, const cpx<double>* __restrict__ twy, const cpx<double>* __restrict__ twz) {
    using C = res3_cfg<R, NX, NY, NZ>;
    if ((int)blockIdx.x >= ninst) return;   // uniform over the workgroup
    const ResidentInst<R>* I = inst + blockIdx.x;
    R* const pR = I->psiR;
    R* const pI = I->psiI;
    const R* __restrict__ V = I->V;
    const int64_t slot0 = *I->counter;
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int l = 0; l < m; ++l) {
            for (int half = 0; half < 2; ++half) {
                const R kx = I->kin[2 * l + half], ky = I->kin_y[2 * l + half], kz = I->kin_z[2 * l + half];
                const R pt = I->pot[2 * l + half];
                if (kx == (R)0 && ky == (R)0 && kz == (R)0 && pt == (R)0) continue;   // uniform
                const R* f = half == 0 ? pI : pR;
                R* g = half == 0 ? pR : pI;
                res3_phase<R, NX, 0, NX, NY, NZ>(f, g, V, kx, pt, nyq_zero, twx);
                __syncthreads();
                res3_phase<R, NY, 1, NX, NY, NZ>(f, g, V, ky, (R)0, nyq_zero, twy);
                __syncthreads();
                res3_phase<R, NZ, 2, NX, NY, NZ>(f, g, V, kz, (R)0, nyq_zero, twz);
                __syncthreads();
            }
        }
        if (threadIdx.x == 0) {
            const int64_t slot = slot0 + s;
            for (int q = 0; q < I->nprobes && slot < I->capacity; ++q) {
                const int64_t pidx = I->probe_idx[q];
                if (pidx < 0 || pidx >= C::NPT) {
                    *I->fault = 1;
                    continue;
                }
                I->probes[(slot * I->nprobes + q) * 2 + 0] = (double)pR[pidx];
                I->probes[(slot * I->nprobes + q) * 2 + 1] = (double)pI[pidx];
            }
        }
        // the next step writes the fields thread 0 has just sampled
        __syncthreads();
    }
    if (threadIdx.x == 0) *I->counter = slot0 + nsteps;
}

template <typename R, int NX, int NY, int NZ>
static hipError_t res3_n(const ResidentInst<R>* inst, int ninst, int m, int64_t nsteps, int nyq_zero,
                         const void* twx, const void* twy, const void* twz, hipStream_t st) {
    hipLaunchKernelGGL((k_resident_3d<R, NX, NY, NZ>), dim3(ninst), dim3(res3_cfg<R, NX, NY, NZ>::THREADS), 0, st,
                       inst, ninst, m, nsteps, nyq_zero, (const cpx<double>*)twx, (const cpx<double>*)twy,
                       (const cpx<double>*)twz);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_resident_3d(int64_t nx, int64_t ny, int64_t nz, const ResidentInst<R>* inst, int ninst, int m,
                              int64_t nsteps, int nyq_zero, const void* twx, const void* twy, const void* twz,
                              hipStream_t st) {
    if (ninst < 1 || m < 1 || m > kResMaxSubsteps / 2 || nsteps < 0) return hipErrorInvalidValue;
    if (!resident3d_ok(nx, ny, nz)) return hipErrorInvalidValue;
    return res3_n<R, 16, 16, 16>(inst, ninst, m, nsteps, nyq_zero, twx, twy, twz, st);
}

template hipError_t launch_resident_3d<double>(int64_t, int64_t, int64_t, const ResidentInst<double>*, int, int,
                                               int64_t, int, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_resident_3d<float>(int64_t, int64_t, int64_t, const ResidentInst<float>*, int, int,
                                              int64_t, int, const void*, const void*, const void*, hipStream_t);

bool resident_len_ok(int64_t n) { return n >= 16 && (n & (n - 1)) == 0 && n <= 16384; }

bool resident2d_ok(int64_t nx, int64_t ny) {
    return (nx == 16 || nx == 32 || nx == 64) && (ny == 16 || ny == 32 || ny == 64);
}

template <typename R, int NX, int NY>
static hipError_t res2_n(const ResidentInst<R>* inst, int ninst, int m, int64_t nsteps, int nyq_zero,
                         const void* twx, const void* twy, hipStream_t st) {
    hipLaunchKernelGGL((k_resident_2d<R, NX, NY>), dim3(ninst), dim3(res2_cfg<NX, NY>::THREADS), 0, st, inst,
                       ninst, m, nsteps, nyq_zero, (const cpx<double>*)twx, (const cpx<double>*)twy);
    return hipGetLastError();
}

template <typename R, int NX>
static hipError_t res2_x(int64_t ny, const ResidentInst<R>* inst, int ninst, int m, int64_t nsteps, int nyq_zero,
                         const void* twx, const void* twy, hipStream_t st) {
    switch (ny) {
        case 16: return res2_n<R, NX, 16>(inst, ninst, m, nsteps, nyq_zero, twx, twy, st);
        case 32: return res2_n<R, NX, 32>(inst, ninst, m, nsteps, nyq_zero, twx, twy, st);
        case 64: return res2_n<R, NX, 64>(inst, ninst, m, nsteps, nyq_zero, twx, twy, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_resident_2d(int64_t nx, int64_t ny, const ResidentInst<R>* inst, int ninst, int m,
                              int64_t nsteps, int nyq_zero, const void* twx, const void* twy, hipStream_t st) {
    if (ninst < 1 || m < 1 || m > kResMaxSubsteps / 2 || nsteps < 0) return hipErrorInvalidValue;
    switch (nx) {
        case 16: return res2_x<R, 16>(ny, inst, ninst, m, nsteps, nyq_zero, twx, twy, st);
        case 32: return res2_x<R, 32>(ny, inst, ninst, m, nsteps, nyq_zero, twx, twy, st);
        case 64: return res2_x<R, 64>(ny, inst, ninst, m, nsteps, nyq_zero, twx, twy, st);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_resident_2d<double>(int64_t, int64_t, const ResidentInst<double>*, int, int, int64_t,
                                               int, const void*, const void*, hipStream_t);
template hipError_t launch_resident_2d<float>(int64_t, int64_t, const ResidentInst<float>*, int, int, int64_t,
                                              int, const void*, const void*, hipStream_t);

template <typename R, int N>
static hipError_t res_n(const ResidentInst<R>* inst, int ninst, int m, int64_t nsteps, int nyq_zero,
                        const void* tw, hipStream_t st) {
    using C = res_cfg<N>;
    const int groups = (ninst + 1) / 2;
    const int blocks = (groups + C::GPB - 1) / C::GPB;
    hipLaunchKernelGGL((k_resident_1d<R, N, (N > 4096)>), dim3(blocks), dim3(C::THREADS), 0, st, inst,
                       ninst, m, nsteps, nyq_zero, (const cpx<double>*)tw);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_resident_1d(int64_t n, const ResidentInst<R>* inst, int ninst, int m, int64_t nsteps,
                              int nyq_zero, const void* tw, hipStream_t st) {
    switch (n) {
        case 16: return res_n<R, 16>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        case 32: return res_n<R, 32>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        case 64: return res_n<R, 64>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        case 128: return res_n<R, 128>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        case 256: return res_n<R, 256>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        case 512: return res_n<R, 512>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        case 1024: return res_n<R, 1024>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        case 2048: return res_n<R, 2048>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        case 4096: return res_n<R, 4096>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        case 8192: return res_n<R, 8192>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        case 16384: return res_n<R, 16384>(inst, ninst, m, nsteps, nyq_zero, tw, st);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_resident_1d<double>(int64_t, const ResidentInst<double>*, int, int, int64_t, int,
                                               const void*, hipStream_t);
template hipError_t launch_resident_1d<float>(int64_t, const ResidentInst<float>*, int, int, int64_t, int,
                                              const void*, hipStream_t);

}  // namespace spstd
