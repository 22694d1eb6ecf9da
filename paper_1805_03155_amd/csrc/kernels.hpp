// Launchers of the SPSTD device kernels (host-callable C++; no C ABI here).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spstd {

// Pencils along y (axis 1) or z (axis 2): a complex pencil packs the real
// columns x = 2*px and 2*px + 1.  Element e of pencil (px, outer) lies at
// outer*outer_stride + 2*px + e*stride.
struct AxisGeom {
    int64_t half_x;        // nx / 2
    int64_t n_outer;       // nz for the y pass, ny for the z pass
    int64_t outer_stride;  // nx*ny for the y pass, nx for the z pass
    int64_t stride;        // nx for the y pass, nx*ny for the z pass
};

// Rows along x: complex pencil q packs rows 2q and 2q+1 (row r starts at r*nx);
// with an odd row count the last pencil has no imaginary row.
struct RowGeom {
    int64_t nrows;
};

// Supported pencil lengths.
bool axis_len_ok(int64_t n);   // y/z passes: 16..1024
bool row_len_ok(int64_t n);    // x pass:     16..16384

// dst += T_axis src, T_axis = IFFT_axis(scale * ks^2 * FFT_axis(.)).
template <typename R>
hipError_t launch_axis_acc(int64_t n, const R* src, R* dst, const void* tw,
                           const AxisGeom& g, double scale, int nyq_zero,
                           hipStream_t st);

// dst += T_x src + vscale * V * src  (one half-stage along x)
template <typename R>
hipError_t launch_x_acc(int64_t nx, const R* src, R* dst, const R* V,
                        const void* tw, const RowGeom& g, double scale,
                        double vscale, int nyq_zero, hipStream_t st);

// Fused A and B halves along x:
//   g  = g + T_x^a f + va * V f         (g = psi_R, f = psi_I)
//   f  = f + T_x^b g + vb * V g         (with the new g)
template <typename R>
hipError_t launch_x_ab(int64_t nx, R* psiR, R* psiI, const R* V, const void* tw,
                       const RowGeom& g, double sa, double va, double sb,
                       double vb, int nyq_zero, hipStream_t st);

// probe sample: out[slot][p] = (psiR[idx_p], psiI[idx_p]) as doubles, where
// slot = *counter; then (*counter)++.  Single thread block.
template <typename R>
hipError_t launch_probe(const R* psiR, const R* psiI, const int64_t* idx,
                        int nprobes, double* out, int64_t* counter,
                        int64_t capacity, hipStream_t st);

// per-block FP64 partial sums of psiR^2 + psiI^2 (fixed order)
template <typename R>
hipError_t launch_norm_partials(const R* psiR, const R* psiI, int64_t n,
                                double* partials, int nblocks, hipStream_t st);

// y = a*x + b*y (elementwise, used by the RK4 comparison run)
template <typename R>
hipError_t launch_axpby(int64_t n, double a, const R* x, double b, R* y,
                        hipStream_t st);
// z = x + a*y
template <typename R>
hipError_t launch_xpay(int64_t n, const R* x, double a, const R* y, R* z,
                       hipStream_t st);
template <typename R>
hipError_t launch_fill0(int64_t n, R* y, hipStream_t st);

}  // namespace spstd
