// Resident kernels (1D, small 2D): instance table and launchers (host-callable C++).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.hpp"

namespace spstd {

constexpr int kResMaxProbes = 8;
constexpr int kResMaxSubsteps = 32;   // 2 * SPSTD_MAX_STAGES

// One instance advanced by a resident kernel (device-resident table).
template <typename R>
struct ResidentInst {
    const R* V;            // N potential values
    R* psiR;               // N values: state in, state out
    R* psiI;
    double* probes;        // FP64 samples [capacity][nprobes][2]
    int64_t* counter;      // next free sample slot (advanced by nsteps)
    int* fault;            // set to 1 if a probe index lies outside the grid (sample skipped)
    int64_t capacity;      // sample slots available
    int nprobes;           // 0..kResMaxProbes
    int64_t probe_idx[kResMaxProbes];
    R kin[kResMaxSubsteps];   // substep 2l (A) and 2l+1 (B): coef dt (hbar/2m*) (2 pi/L)^2 / N
    R pot[kResMaxSubsteps];   // substep 2l (A) and 2l+1 (B): coef dt / hbar
    R kin_y[kResMaxSubsteps]; // 2D and 3D instances: kin of the y axis (L_y, N_y); kin is then the x axis's
    R kin_z[kResMaxSubsteps]; // 3D instances: kin of the z axis
};

bool resident_len_ok(int64_t n);
// 2D grids the resident kernel holds whole in LDS: n_x, n_y in {16, 32, 64}.
bool resident2d_ok(int64_t nx, int64_t ny);
// 3D grids the resident 3D kernel steps (fields in global memory, one
// workgroup per instance): 16^3.
bool resident3d_ok(int64_t nx, int64_t ny, int64_t nz);

// Advance every instance of the table (all of length n) by nsteps steps of
// m stages.  tw: twiddle table w_n^t, t < n, in the run precision.
template <typename R>
hipError_t launch_resident_1d(int64_t n, const ResidentInst<R>* inst, int ninst, int m, int64_t nsteps,
                              int nyq_zero, const void* tw, hipStream_t st);

// The same for 2D instances of nx by ny points (x fastest), one workgroup
// per instance with the state in LDS.  twx, twy: twiddle tables of the two
// axes (FP64).
template <typename R>
hipError_t launch_resident_2d(int64_t nx, int64_t ny, const ResidentInst<R>* inst, int ninst, int m,
                              int64_t nsteps, int nyq_zero, const void* twx, const void* twy, hipStream_t st);

// The same for 3D instances of nx by ny by nz points (x fastest), one
// workgroup per instance, fields in the instances' own arrays.
template <typename R>
hipError_t launch_resident_3d(int64_t nx, int64_t ny, int64_t nz, const ResidentInst<R>* inst, int ninst, int m,
                              int64_t nsteps, int nyq_zero, const void* twx, const void* twy, const void* twz,
                              hipStream_t st);

}  // namespace spstd
