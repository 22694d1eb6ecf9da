// Probe samples at a step boundary whose two A halves run as one.
//
// When the last stage of a set has no B half (d_m = 0), the A half that ends
// step s and the A half that opens step s + 1 act on psi_R with the same
// psi_I (Eq. 18: nothing changes psi_I between them), so the engine applies
// them as one A half with coefficient c_m + c_1.  The state at the end of
// step s is then never formed in memory; its probe samples follow from the
// values around the merged half:
//   psi_R(s) = psi_R(before) + w (psi_R(after) - psi_R(before)),
//   w = c_m / (c_m + c_1),   psi_I(s) = psi_I before the merged half's B part.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace spstd {

// An index outside the grid skips its sample and sets *fault for the host.
template <typename R>
__global__ void k_probe_save(const R* __restrict__ psi, const int64_t* __restrict__ idx, int nprobes,
                             int64_t npts, double* __restrict__ save, int* __restrict__ fault) {
    const int t = threadIdx.x;
    if (t < nprobes) {
        const int64_t i = idx[t];
        if (i >= 0 && i < npts) save[t] = (double)psi[i];
        else *fault = 1;
    }
}

template <typename R>
__global__ void k_probe_merged(const R* __restrict__ psiR, const int64_t* __restrict__ idx, int nprobes,
                               int64_t npts, const double* __restrict__ saveR, const double* __restrict__ saveI,
                               double w, double* __restrict__ out, int64_t* __restrict__ counter, int64_t capacity,
                               int* __restrict__ fault) {
    const int64_t slot = *counter;
    const int t = threadIdx.x;
    if (slot < capacity && t < nprobes) {
        const int64_t i = idx[t];
        if (i >= 0 && i < npts) {
            const double r0 = saveR[t];
            out[(slot * nprobes + t) * 2 + 0] = r0 + w * ((double)psiR[i] - r0);
            out[(slot * nprobes + t) * 2 + 1] = saveI[t];
        } else {
            *fault = 1;
        }
    }
    __syncthreads();
    if (t == 0) *counter = slot + 1;
}

template <typename R>
hipError_t launch_probe_save(const R* psi, const int64_t* idx, int nprobes, int64_t npts, double* save,
                             int* fault, hipStream_t st) {
    if (nprobes < 1 || nprobes > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_probe_save<R>), dim3(1), dim3(64), 0, st, psi, idx, nprobes, npts, save, fault);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_probe_merged(const R* psiR, const int64_t* idx, int nprobes, int64_t npts, const double* saveR,
                               const double* saveI, double w, double* out, int64_t* counter, int64_t capacity,
                               int* fault, hipStream_t st) {
    if (nprobes < 1 || nprobes > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_probe_merged<R>), dim3(1), dim3(64), 0, st, psiR, idx, nprobes, npts, saveR, saveI, w,
                       out, counter, capacity, fault);
    return hipGetLastError();
}

#define SPSTD_INST_PROBES(R)                                                                                 \
    template hipError_t launch_probe_save<R>(const R*, const int64_t*, int, int64_t, double*, int*,          \
                                             hipStream_t);                                                   \
    template hipError_t launch_probe_merged<R>(const R*, const int64_t*, int, int64_t, const double*,        \
                                               const double*, double, double*, int64_t*, int64_t, int*,      \
                                               hipStream_t);
SPSTD_INST_PROBES(double)
SPSTD_INST_PROBES(float)
#undef SPSTD_INST_PROBES

}  // namespace spstd
