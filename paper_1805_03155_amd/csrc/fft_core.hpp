// Device building blocks of the spectral operator: complex arithmetic,
// register DFTs of length 2/4/8/16, and a Stockham FFT of one pencil of
// length N (a power of two, 16 <= N <= 16384) spread over T = N/16 lanes.
//
// Layout contract ("strided layout"): lane j of a pencil (0 <= j < T) holds
// in its 16 registers v[e] the elements j + T*e, e = 0..15.  The forward
// transform takes samples in this layout and leaves DFT bins in the same
// layout; the inverse transform does the converse.  Between radix passes the
// data goes through LDS; the last pass ends in registers.
//
// Passes: floor(log2 N / 4) radix-16 passes, then one radix-2/4/8 pass when
// log2 N is not a multiple of 4.  Pass p with radix R and running size Ns
// (product of the previous radices) maps butterfly b (inputs b + r*N/R) to
// outputs (b/Ns)*Ns*R + (b mod Ns) + r*Ns after the twiddles
// w_{Ns*R}^{r*(b mod Ns)} -- the self-sorting (Stockham) form, so no
// bit-reversal pass exists.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spstd {

template <typename R>
struct cpx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// multiply by -i (forward) or +i (inverse)
template <typename R, bool INV>
__device__ __forceinline__ cpx<R> rot90(cpx<R> a) {
    return INV ? cpx<R>{-a.y, a.x} : cpx<R>{a.y, -a.x};
}

// exp(-+ 2 pi i m / 16) for the internal twiddles of the 16-point DFT;
// cos(pi/8), sin(pi/8) and sqrt(1/2) to 20 digits.
template <typename R, bool INV, int M>
__device__ __forceinline__ cpx<R> w16mul(cpx<R> a) {
    constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
    constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
    constexpr double H = 0.70710678118654752440;   // sqrt(1/2)
    constexpr int m = M % 16;
    if constexpr (m == 0) return a;
    // angle theta = 2 pi m / 16; forward multiplies by cos - i sin
    constexpr double cs = (m == 1) ? C1 : (m == 2) ? H : (m == 3) ? S1 : (m == 4) ? 0.0
                        : (m == 6) ? -H : (m == 9) ? -C1 : 0.0;
    constexpr double sn = (m == 1) ? S1 : (m == 2) ? H : (m == 3) ? C1 : (m == 4) ? 1.0
                        : (m == 6) ? H : (m == 9) ? -S1 : 0.0;
    static_assert(m == 1 || m == 2 || m == 3 || m == 4 || m == 6 || m == 9, "unused");
    if constexpr (m == 4) return rot90<R, INV>(a);
    const R c = (R)cs;
    const R s = INV ? (R)sn : (R)(-sn);
    return {a.x * c - a.y * s, a.x * s + a.y * c};
}

template <typename R, bool INV>
__device__ __forceinline__ void dft2(cpx<R>& a, cpx<R>& b) {
    cpx<R> t = a - b;
    a = a + b;
    b = t;
}

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cpx<R>& a, cpx<R>& b, cpx<R>& c, cpx<R>& d) {
    cpx<R> s0 = a + c, d0 = a - c, s1 = b + d, d1 = rot90<R, INV>(b - d);
    a = s0 + s1;
    c = s0 - s1;
    b = d0 + d1;
    d = d0 - d1;
}

// natural order in, natural order out
template <typename R, bool INV>
__device__ __forceinline__ void dft8(cpx<R>& x0, cpx<R>& x1, cpx<R>& x2, cpx<R>& x3,
                                     cpx<R>& x4, cpx<R>& x5, cpx<R>& x6, cpx<R>& x7) {
    constexpr double H = 0.70710678118654752440;
    dft4<R, INV>(x0, x2, x4, x6);  // E[k] at x0,x2,x4,x6
    dft4<R, INV>(x1, x3, x5, x7);  // O[k] at x1,x3,x5,x7
    // O[k] *= w8^k
    const R h = (R)H;
    cpx<R> o1 = INV ? cpx<R>{(x3.x - x3.y) * h, (x3.x + x3.y) * h}
                    : cpx<R>{(x3.x + x3.y) * h, (x3.y - x3.x) * h};
    cpx<R> o2 = rot90<R, INV>(x5);
    cpx<R> o3 = INV ? cpx<R>{-(x7.x + x7.y) * h, (x7.x - x7.y) * h}
                    : cpx<R>{(x7.y - x7.x) * h, -(x7.x + x7.y) * h};
    cpx<R> e0 = x0, e1 = x2, e2 = x4, e3 = x6, o0 = x1;
    x0 = e0 + o0; x4 = e0 - o0;
    x1 = e1 + o1; x5 = e1 - o1;
    x2 = e2 + o2; x6 = e2 - o2;
    x3 = e3 + o3; x7 = e3 - o3;
}

// 16-point DFT as 4 x 4: natural order in v[0..15], natural order out.
template <typename R, bool INV, int S = 1>
__device__ __forceinline__ void dft16(cpx<R>* v) {
#define V_(i) v[(i) * S]
    dft4<R, INV>(V_(0), V_(4), V_(8), V_(12));
    dft4<R, INV>(V_(1), V_(5), V_(9), V_(13));
    dft4<R, INV>(V_(2), V_(6), V_(10), V_(14));
    dft4<R, INV>(V_(3), V_(7), V_(11), V_(15));
    // element r1 + 4 k1 holds A[r1][k1]; multiply by w16^(r1 k1)
    V_(5) = w16mul<R, INV, 1>(V_(5));
    V_(9) = w16mul<R, INV, 2>(V_(9));
    V_(13) = w16mul<R, INV, 3>(V_(13));
    V_(6) = w16mul<R, INV, 2>(V_(6));
    V_(10) = w16mul<R, INV, 4>(V_(10));
    V_(14) = w16mul<R, INV, 6>(V_(14));
    V_(7) = w16mul<R, INV, 3>(V_(7));
    V_(11) = w16mul<R, INV, 6>(V_(11));
    V_(15) = w16mul<R, INV, 9>(V_(15));
    dft4<R, INV>(V_(0), V_(1), V_(2), V_(3));
    dft4<R, INV>(V_(4), V_(5), V_(6), V_(7));
    dft4<R, INV>(V_(8), V_(9), V_(10), V_(11));
    dft4<R, INV>(V_(12), V_(13), V_(14), V_(15));
    // now element k2 + 4 k1 holds X[k1 + 4 k2]: transpose the 4x4 index
    cpx<R> t;
    t = V_(1); V_(1) = V_(4); V_(4) = t;
    t = V_(2); V_(2) = V_(8); V_(8) = t;
    t = V_(3); V_(3) = V_(12); V_(12) = t;
    t = V_(6); V_(6) = V_(9); V_(9) = t;
    t = V_(7); V_(7) = V_(13); V_(13) = t;
    t = V_(11); V_(11) = V_(14); V_(14) = t;
#undef V_
}

template <int N>
struct fft_shape {
    static constexpr int LOG = (N <= 1) ? 0 : 1 + fft_shape<N / 2>::LOG;
};
template <>
struct fft_shape<1> {
    static constexpr int LOG = 0;
};

// LDS index padding: one spare slot every 16 keeps the radix-16 scatter
// (stride-16 writes) off a single bank.  Where one pencil fills an LDS
// cycle (512- and 1024-point pencils with the position fastest over the
// lanes, JS = 1: 32 lanes on one pencil) the gather reads 32 consecutive
// positions, which one slot every 16 wraps onto the first bank again; one
// slot every 32 keeps both the scatter and the gather conflict-free there.
// (With the pencil index fastest, two 512-point pencils share a cycle and
// one slot every 16 is the conflict-free choice.)  lds_size is the larger
// of the two footprints.
template <int N, int JS>
struct lds_pad_shift {
    static constexpr int value = (JS == 1 && (N == 512 || N == 1024)) ? 5 : 4;
};
template <int N, int JS>
__device__ __forceinline__ int lpad(int i) { return i + (i >> lds_pad_shift<N, JS>::value); }
template <int N>
struct lds_size {
    static constexpr int value = N + N / 16;
};

// Wave-local or workgroup-wide LDS barrier.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}


// Twiddles are generated in FP64 in every precision: the table holds
// exp(-2 pi i t / N) in FP64 (from long-double cos/sin), any products of
// table entries are formed in FP64, and each twiddle is rounded once to the
// run precision where it is used.
template <typename R>
__device__ __forceinline__ cpx<R> to_run(cpx<double> a) {
    return cpx<R>{(R)a.x, (R)a.y};
}

// Twiddles w_N^{r*b}, r < RL, of the tail pass (RL = 2, 4, 8).
template <typename R, int RL, bool PRODUCTS>
__device__ __forceinline__ void twiddles_tail(const cpx<double>* __restrict__ tw, int b, cpx<R> (&w)[8]) {
    w[0] = cpx<R>{(R)1, (R)0};
    if constexpr (!PRODUCTS || RL == 2) {
#pragma unroll
        for (int r = 1; r < RL; ++r) w[r] = to_run<R>(tw[r * b]);
    } else {
        const cpx<double> t1 = tw[b], t2 = cmul(t1, t1), t3 = cmul(t2, t1);
        w[1] = to_run<R>(t1);
        w[2] = to_run<R>(t2);
        w[3] = to_run<R>(t3);
        if constexpr (RL == 8) {
            const cpx<double> t4 = tw[4 * b];
            w[4] = to_run<R>(t4);
            w[5] = to_run<R>(cmul(t1, t4));
            w[6] = to_run<R>(cmul(t2, t4));
            w[7] = to_run<R>(cmul(t3, t4));
        }
    }
}

// Transform of P pencils per lane group, forward (INV = false) or inverse
// (unnormalised).
// v[p]: the lane's 16 values of pencil p in strided layout; j: lane position
// in the pencil; lds: LDS of pencil 0, pencil p at lds + p * lds_stride;
// a pencil slice holds lds_size<N> reals (SPLIT) or twice that (re, im).
// tw: FP64 table of w_N^t = exp(-2 pi i t / N), t = 0..N-1.
// ---------------------------------------------------------------------------
// Reorder before a radix-RL tail pass without LDS (gfx950 lane swaps).
// After the last radix-16 pass, with S = N / (16 RL), lane j = m + S q
// (m < S, q < RL) holds in register t = a + RL c (a < RL) the output that
// the tail pass wants in lane m + S a, register (16/RL) q + c.  Each bit of
// q is exchanged with the same bit of a by one swap of register pairs
// between lanes D = S JS 2^s apart (JS: lane distance of neighbouring j),
// v_permlane16_swap for D = 16 and v_permlane32_swap for D = 32: in the
// lower lane the low register keeps its value and the high register
// receives the partner's low register, in the upper lane the low register
// receives the partner's high register.  A renaming of registers finishes
// the reorder.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void swap_dwords(uint32_t& lo, uint32_t& hi) {
    static_assert(D == 16 || D == 32, "lane swaps span 16 or 32 lanes");
    if constexpr (D == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(lo, hi, false, false);
        lo = r[0];
        hi = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
        lo = r[0];
        hi = r[1];
    }
}

template <int D>
__device__ __forceinline__ void swap_reals(float& lo, float& hi) {
    uint32_t a = __float_as_uint(lo), b = __float_as_uint(hi);
    swap_dwords<D>(a, b);
    lo = __uint_as_float(a);
    hi = __uint_as_float(b);
}

template <int D>
__device__ __forceinline__ void swap_reals(double& lo, double& hi) {
    const uint64_t a = (uint64_t)__double_as_longlong(lo), b = (uint64_t)__double_as_longlong(hi);
    uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    swap_dwords<D>(a0, b0);
    swap_dwords<D>(a1, b1);
    lo = __longlong_as_double((long long)(((uint64_t)a1 << 32) | a0));
    hi = __longlong_as_double((long long)(((uint64_t)b1 << 32) | b0));
}

// Whether the tail reorder of an N-point pencil with lane distance JS runs
// on lane swaps (every swap distance 16 or 32).
template <int N, int JS>
struct tail_swaps {
    static constexpr int LOG = fft_shape<N>::LOG;
    static constexpr int RL = 1 << (LOG % 4);
    static constexpr int S = N / (16 * RL);
    static constexpr int D0 = S * JS;
    static constexpr bool OK = JS > 0 && RL > 1 && N / 16 <= 64 &&
                               (RL == 2 ? (D0 == 16 || D0 == 32) : RL == 4 ? D0 == 16 : false);
};

template <typename R, int RL, int D0, int P>
__device__ __forceinline__ void tail_reorder(cpx<R> (&v)[P][16]) {
    constexpr int C = 16 / RL;
#pragma unroll
    for (int s = 0; (1 << s) < RL; ++s) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (r & (1 << s)) continue;
            const int h = r | (1 << s);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (s == 0) {
                    swap_reals<D0>(v[p][r].x, v[p][h].x);
                    swap_reals<D0>(v[p][r].y, v[p][h].y);
                } else {
                    swap_reals<(D0 == 16 ? 32 : 16)>(v[p][r].x, v[p][h].x);
                    swap_reals<(D0 == 16 ? 32 : 16)>(v[p][r].y, v[p][h].y);
                }
            }
        }
    }
    // register q + RL c now holds what belongs in register c + C q
#pragma unroll
    for (int p = 0; p < P; ++p) {
        cpx<R> t[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) t[r] = v[p][r];
#pragma unroll
        for (int q = 0; q < RL; ++q)
#pragma unroll
            for (int c = 0; c < C; ++c) v[p][c + C * q] = t[q + RL * c];
    }
}

// WAVE: the pencils lie inside one wavefront (T <= 64).
// SPLIT: exchange the real parts, then the imaginary parts (half the LDS,
// twice the barriers).
// PRODUCTS: build the twiddles of a pass from two table reads.
// JS: lane distance between neighbouring positions j of a pencil in the
// wave (0: unknown); where tail_swaps<N, JS>::OK the reorder before the
// tail pass uses lane swaps instead of LDS.
template <typename R, int N, bool INV, bool WAVE, bool SPLIT, bool PRODUCTS, int P, int JS = 0>
__device__ __forceinline__ void fft_pencils(cpx<R> (&v)[P][16], int j, R* lds, int lds_stride,
                                            const cpx<double>* __restrict__ tw) {
    constexpr int LOG = fft_shape<N>::LOG;
    constexpr int T = N / 16;
    constexpr int NP16 = LOG / 4;            // radix-16 passes
    constexpr int RL = 1 << (LOG % 4);       // radix of the tail pass (1: none)
    constexpr int NPASS = NP16 + (RL > 1 ? 1 : 0);
    constexpr int LS = lds_size<N>::value;
    static_assert(N >= 16 && (N & (N - 1)) == 0, "N must be a power of two >= 16");

    // pass 0: radix 16, Ns = 1, no twiddles
#pragma unroll
    for (int p = 0; p < P; ++p) dft16<R, INV>(v[p]);
    if constexpr (NPASS == 1) return;

    int Ns = 1;
#pragma unroll
    for (int ps = 1; ps < NPASS; ++ps) {
        // scatter the previous radix-16 pass outputs (Ns = 16^(ps-1)),
        // gather the strided layout
        bool swapped = false;
        if constexpr (WAVE && tail_swaps<N, JS>::OK) {
            if (ps == NPASS - 1) {
                tail_reorder<R, tail_swaps<N, JS>::RL, tail_swaps<N, JS>::D0, P>(v);
                swapped = true;
            }
        }
        if (!swapped) {
            const int k = j % Ns;
            const int base = (j / Ns) * Ns * 16 + k;
            lds_sync<WAVE>();   // earlier reads of these slices are complete
            if constexpr (!SPLIT) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    R* lre = lds + p * lds_stride;
                    R* lim = lre + LS;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int q = lpad<N, JS>(base + r * Ns);
                        lre[q] = v[p][r].x;
                        lim[q] = v[p][r].y;
                    }
                }
                lds_sync<WAVE>();
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    R* lre = lds + p * lds_stride;
                    R* lim = lre + LS;
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int q = lpad<N, JS>(j + T * e);
                        v[p][e].x = lre[q];
                        v[p][e].y = lim[q];
                    }
                }
            } else {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    R* lre = lds + p * lds_stride;
#pragma unroll
                    for (int r = 0; r < 16; ++r) lre[lpad<N, JS>(base + r * Ns)] = v[p][r].x;
                }
                lds_sync<WAVE>();
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    R* lre = lds + p * lds_stride;
                    R keep[16];
#pragma unroll
                    for (int e = 0; e < 16; ++e) keep[e] = lre[lpad<N, JS>(j + T * e)];
#pragma unroll
                    for (int e = 0; e < 16; ++e) v[p][e].x = keep[e];
                }
                // the imaginary parts still sit in v[p][r].y in scatter order
                lds_sync<WAVE>();
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    R* lre = lds + p * lds_stride;
#pragma unroll
                    for (int r = 0; r < 16; ++r) lre[lpad<N, JS>(base + r * Ns)] = v[p][r].y;
                }
                lds_sync<WAVE>();
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    R* lre = lds + p * lds_stride;
#pragma unroll
                    for (int e = 0; e < 16; ++e) v[p][e].y = lre[lpad<N, JS>(j + T * e)];
                }
            }
        }
        Ns *= 16;
        const bool last = (ps == NPASS - 1);
        if (!last || RL == 1) {
            // radix-16 pass: butterfly b = j, k = j mod Ns,
            // twiddle w_{16 Ns}^{r k} = w_N^{r k N / (16 Ns)}
            const int k = j % Ns;
            const int step = k * (N / (16 * Ns));
            if constexpr (PRODUCTS) {
                // w^{a step} w^{4 b step}, r = a + 4b, formed in FP64 where used
                const cpx<double> t1 = tw[step], t4 = tw[4 * step];
                const cpx<double> t2 = cmul(t1, t1), t3 = cmul(t2, t1);
                const cpx<double> t8 = cmul(t4, t4), t12 = cmul(t8, t4);
#pragma unroll
                for (int r = 1; r < 16; ++r) {
                    const int a = r & 3, b = r >> 2;
                    const cpx<double> lo = a == 1 ? t1 : a == 2 ? t2 : t3;
                    const cpx<double> hi = b == 1 ? t4 : b == 2 ? t8 : t12;
                    const cpx<R> w = to_run<R>(b == 0 ? lo : a == 0 ? hi : cmul(lo, hi));
#pragma unroll
                    for (int p = 0; p < P; ++p) v[p][r] = INV ? cmulc(v[p][r], w) : cmul(v[p][r], w);
                }
            } else {
#pragma unroll
                for (int r = 1; r < 16; ++r) {
                    const cpx<R> w = to_run<R>(tw[r * step]);
#pragma unroll
                    for (int p = 0; p < P; ++p) v[p][r] = INV ? cmulc(v[p][r], w) : cmul(v[p][r], w);
                }
            }
#pragma unroll
            for (int p = 0; p < P; ++p) dft16<R, INV>(v[p]);
        } else {
            // tail pass of radix RL: butterflies b = j + T u, u < 16/RL,
            // Ns * RL = N so the twiddle is w_N^{r b}
            constexpr int U = 16 / RL;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int b = j + T * u;
                cpx<R> w[8];
                twiddles_tail<R, RL, PRODUCTS>(tw, b, w);
#pragma unroll
                for (int p = 0; p < P; ++p) {
#pragma unroll
                    for (int r = 1; r < RL; ++r)
                        v[p][u + U * r] = INV ? cmulc(v[p][u + U * r], w[r]) : cmul(v[p][u + U * r], w[r]);
                    if constexpr (RL == 2) {
                        dft2<R, INV>(v[p][u], v[p][u + U]);
                    } else if constexpr (RL == 4) {
                        dft4<R, INV>(v[p][u], v[p][u + U], v[p][u + 2 * U], v[p][u + 3 * U]);
                    } else {
                        dft8<R, INV>(v[p][u], v[p][u + U], v[p][u + 2 * U], v[p][u + 3 * U],
                                     v[p][u + 4 * U], v[p][u + 5 * U], v[p][u + 6 * U], v[p][u + 7 * U]);
                    }
                }
            }
        }
    }
}

}  // namespace spstd
