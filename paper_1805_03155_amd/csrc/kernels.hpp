// Launchers of the SPSTD device kernels (host-callable C++; no C ABI here).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spstd {

// Pencils along y (axis 1) or z (axis 2) of a stack of instances of one
// shape: a complex pencil packs the real columns x = 2*px and 2*px + 1.
// Pencil (px, outer) starts at
//   (outer / n_in) * stride_hi + (outer % n_in) * stride_lo + 2 * px
// and element e lies stride further on; the instance is outer / n_in.
struct AxisGeom {
    int64_t half_x;      // nx / 2
    int64_t n_outer;     // instances * (nz for the y pass, ny for the z pass)
    int64_t n_in;        // nz (y pass) or ny (z pass)
    int64_t stride_lo;   // nx*ny (y pass) or nx (z pass)
    int64_t stride_hi;   // points per instance
    int64_t stride;      // nx (y pass) or nx*ny (z pass)
};

// Rows along x: complex pencil q packs rows 2q and 2q+1 (row r starts at
// r*nx; rows of one instance are consecutive, rows_per_inst of them); with
// an odd row count the last pencil has no imaginary row.
struct RowGeom {
    int64_t nrows;
    int64_t rows_per_inst;
};

// Per-instance, per-stage scales (run precision), row-major
// [instance][stage][SC_COLS]: kinetic scale of the A substep along x, y, z
// (c_l dt (hbar/2m*) (2 pi/L_d)^2 / n_d), potential scale of A (c_l dt/hbar),
// then the same four for B (with -d_l dt).  Each pass multiplies the
// inverse transform by its instance's scale, so instances with different
// dt, spacing and potential share launches (and complex pencils).
enum { SC_KXA = 0, SC_KYA, SC_KZA, SC_PA, SC_KXB, SC_KYB, SC_KZB, SC_PB, SC_COLS };
struct ScaleRef {
    const void* tab;   // device table, run precision
    int m;             // stages per instance
    int l;             // stage of this pass
};

// The pass launchers (y/z passes, stage-boundary sweep, x passes) take the
// waves per block as a last argument: 0 for the built-in choice per
// precision and length, or 2 or 4 (the batch autotuner's candidates).

// Supported pencil lengths.
bool axis_len_ok(int64_t n);   // y/z passes: 16..1024
bool row_len_ok(int64_t n);    // x pass:     16..16384
bool wall_dft_len_ok(int64_t n);   // walled axes of n <= 32 cells not transformed by the FFT passes

// dst += scale_inst * IFFT_axis(ks^2 FFT_axis(src)), scale column col.
template <typename R>
hipError_t launch_axis_acc(int64_t n, const R* src, R* dst, const void* tw,
                           const AxisGeom& g, const ScaleRef& sc, int col, int nyq_zero,
                           hipStream_t st, int wpb = 0);

// One sweep of y (or z) pencils at a stage boundary:
//   psiI += sB T psiR  (column colB of stage scB.l), then
//   psiR += sA T psiI  (column colA of stage scA.l), T the bare axis operator.
template <typename R>
hipError_t launch_axis_ba(int64_t n, R* psiR, R* psiI, const void* tw, const AxisGeom& g, const ScaleRef& scB,
                          const ScaleRef& scA, int colB, int colA, int nyq_zero, hipStream_t st, int wpb = 0);

// dst += k * IFFT_x(ks^2 FFT_x(src)) + p * V * src with (k, p) of columns
// (kcol, pcol): one half-stage along x.
template <typename R>
hipError_t launch_x_acc(int64_t nx, const R* src, R* dst, const R* V,
                        const void* tw, const RowGeom& g, const ScaleRef& sc,
                        int kcol, int pcol, int nyq_zero, hipStream_t st, int wpb = 0);

// 3D grids whose x-z planes the fused plane kernel holds in LDS: n_x, n_z
// in {16, 32, 64}.
bool plane_ok(int64_t nx, int64_t nz);
// The z and x terms of stage sc.l on every x-z plane of ninst stacked
// instances (nx by ny by nz, x fastest), one workgroup per plane:
// do_a: psi_R += T_z psi_I (SC_KZA), then += T_x psi_I + p_A V psi_I
// (SC_KXA, SC_PA); do_b: then psi_I += T_x psi_R + p_B V psi_R (SC_KXB,
// SC_PB), += T_z psi_R (SC_KZB).  Slots with zero scales are left alone.
template <typename R>
hipError_t launch_plane_zxz(int64_t nx, int64_t ny, int64_t nz, int64_t ninst, R* psiR, R* psiI, const R* V,
                            const ScaleRef& sc, int do_a, int do_b, int nyq_zero, const void* twx, const void* twz,
                            hipStream_t st);

// x passes of 1D rows of 8192 or 16384 points over many workgroups (the
// 128-column four-step factorisation of the transform; rows_per_inst 1).
// a, b: the A half (psi_R += T psi_I + p_A V psi_I, SC_KXA, SC_PA) and/or
// the B half (psi_I += T psi_R + p_B V psi_R, SC_KXB, SC_PB), A first.
// twN: the row's FP64 twiddle table (n entries); tw1: a 128-entry table;
// tw2: an (n / 128)-entry table; scratch: fourstep_scratch_bytes bytes of
// device memory the passes overwrite.  Pencils whose rows have zero
// kinetic scales in the applied halves are left alone.  fuse_next (b set):
// leave the column transforms of psi_I(new) in scratch; s_ready (a set):
// the previous pass on the same rows left them there, with psi_I unchanged
// since.
bool fourstep_ok(int64_t n);
size_t fourstep_scratch_bytes(int64_t n, int64_t nrows, size_t esz);
template <typename R>
hipError_t launch_x_fourstep(int64_t n, R* psiR, R* psiI, const R* V, const void* twN, const void* tw1,
                             const void* tw2, void* scratch, const RowGeom& rg, const ScaleRef& sc, int a, int b,
                             int nyq_zero, int s_ready, int fuse_next, hipStream_t st);

// Fused A and B halves along x (columns SC_KXA, SC_PA, SC_KXB, SC_PB):
//   psi_R += T_x^A psi_I + p_A V psi_I;  then  psi_I += T_x^B psi_R + p_B V psi_R
template <typename R>
hipError_t launch_x_ab(int64_t nx, R* psiR, R* psiI, const R* V, const void* tw,
                       const RowGeom& g, const ScaleRef& sc, int nyq_zero, hipStream_t st, int wpb = 0);

// Every probe kernel checks each device-side index against the grid size
// (npts): an index outside [0, npts) skips its sample and sets *fault = 1,
// which the host reads after the run and reports.
//
// Batched probe samples: for every instance i < ninst with active[i],
// out_i[slot][p] = (psiR[i*npts + idx[i*P + p]], psiI[...]) as doubles,
// slot = counter[i], then counter[i]++ (slots >= capacity are not written).
// out_i = probes + i * capacity * P * 2.
//
// part: the whole sample (PROBE_FULL), or one half of it: PROBE_R writes
// the psi_R values and keeps the counter, PROBE_I writes the psi_I values
// and advances it.  The halves serve a step boundary whose last pass runs
// fused with the next step's first: psi_R is final before that sweep,
// psi_I after it.
enum ProbePart { PROBE_R = 1, PROBE_I = 2, PROBE_FULL = 3 };
template <typename R>
hipError_t launch_probe_batch(const R* psiR, const R* psiI, int64_t npts, const int64_t* idx,
                              int nprobes, const int* active, int ninst, double* probes,
                              int64_t* counter, int64_t capacity, int* fault, hipStream_t st,
                              int part = PROBE_FULL);

// probe sample: out[slot][p] = (psiR[idx_p], psiI[idx_p]) as doubles, where
// slot = *counter; then (*counter)++.  Single thread block, nprobes 0..64.
template <typename R>
hipError_t launch_probe(const R* psiR, const R* psiI, const int64_t* idx,
                        int nprobes, int64_t npts, double* out, int64_t* counter,
                        int64_t capacity, int* fault, hipStream_t st);

// Merged step boundary (the last A half of a step and the first A half of
// the next as one): save[p] = psi[idx_p] as doubles; then the sample
// out[slot][p] = (saveR_p + w (psiR[idx_p] - saveR_p), saveI_p), slot =
// *counter, then (*counter)++.  Single thread block, nprobes 1..64.
template <typename R>
hipError_t launch_probe_save(const R* psi, const int64_t* idx, int nprobes, int64_t npts, double* save,
                             int* fault, hipStream_t st);
template <typename R>
hipError_t launch_probe_merged(const R* psiR, const int64_t* idx, int nprobes, int64_t npts, const double* saveR,
                               const double* saveI, double w, double* out, int64_t* counter, int64_t capacity,
                               int* fault, hipStream_t st);

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

// Windowed Fourier accumulation of the state (eigenstate reconstruction):
// with m = *count, if m < M: acc_k[i] += w_m exp(+i E_k m dt/hbar) psi[i]
// for k < nE, w_m the symmetric 4-term Blackman-Harris window of length M;
// acc_k is [npts] complex FP64 (re, im interleaved) at acc + 2 k npts.
struct EigParams {
    double E[8];
    int nE;
    int64_t M;
    double dt_over_hbar;
    double* acc;
    const int64_t* count;
};
template <typename R>
hipError_t launch_eig_acc(const R* psiR, const R* psiI, int64_t npts, const EigParams& ep, hipStream_t st);
// (*count)++ (one thread; after the accumulation of a step)
hipError_t launch_count_tick(int64_t* count, hipStream_t st);

// Three-point difference substep over all axes of one grid n[3]:
// dst += sum_d k_d (2 f - f[+e_d] - f[-e_d]) + p V f, periodic wrap, with
// k_d from scale columns kcol0 + d and p from pcol (instance 0).
template <typename R>
hipError_t launch_fd_acc(const R* src, R* dst, const R* V, const int64_t* n, const ScaleRef& sc, int kcol0,
                         int pcol, hipStream_t st);

// Boundary of a line (the same values as the C ABI's SPSTD_BC_*).
enum { WALL_NONE = 0, WALL_DIRICHLET = 1, WALL_NEUMANN = 2 };

// Lines of one axis for the energy sums: line L starts at
// (L / n_lo) * stride_hi + (L % n_lo); element e lies e * stride further on.
struct EnergyGeom {
    int64_t nlines;
    int64_t n_lo;
    int64_t stride_hi;
    int64_t stride;
};

// partials[b] (b < *nblocks <= max_blocks) = block sums of
// ks^2 |FFT_axis(psiR + i psiI)(k)|^2 over the lines of the axis (ks the
// signed bin index; the Nyquist bin counts 0 if nyq_zero).  rows: the lines
// are contiguous (x axis).  wall (WALL_*): a walled line of n samples is
// transformed as its mirrored extension of 2n points (tw then holds 2n
// twiddles), which counts every sample twice.  Transform length: 16..16384
// for rows, 16..1024 else.
template <typename R>
hipError_t launch_energy_axis(int64_t n, int rows, int wall, const R* psiR, const R* psiI,
                              const void* tw, const EnergyGeom& g, int nyq_zero, double* partials,
                              int max_blocks, int* nblocks, hipStream_t st);

// Pass along a walled axis (wall = WALL_DIRICHLET or WALL_NEUMANN)
// of n samples: dst += k * T src (+ p * V * src if pcol >= 0), with (k, p)
// from columns (kcol, pcol) of each line's instance (first sample / npts).
// T is the periodic operator of the mirrored line of 2n points (tw: 2n
// twiddles).  Lines come in pairs (2q, 2q + 1) sharing a complex pencil, so
// for columns n_lo must be even.  2n: 32..16384 for rows, 32..1024 else.
template <typename R>
hipError_t launch_wall_acc(int64_t n, int rows, int wall, const R* src, R* dst, const R* V,
                           const void* tw, const EnergyGeom& g, int64_t npts, const ScaleRef& sc,
                           int kcol, int pcol, int nyq_zero, hipStream_t st);

// pot[b], nrm[b] (b < nblocks) = block sums of V |psi|^2 and |psi|^2.
template <typename R>
hipError_t launch_energy_pot(const R* psiR, const R* psiI, const R* V, int64_t n, double* pot,
                             double* nrm, int nblocks, hipStream_t st);

// ---------------------------------------------------------------------------
// Mixed-shape groups: stacks of 2D instances of different shapes (one
// member per shape, n_x and n_y in {128, 256, 512}) advanced by one launch
// per pass over a table of tiles.
// ---------------------------------------------------------------------------
bool mix_len_ok(int64_t n);

// One member: a stack of `capacity` instances of nx by ny points (the
// fields, scales, twiddles and probe buffers of one single-shape batch).
template <typename R>
struct MixMember {
    int nx, ny;
    R* psiR;
    R* psiI;
    const R* V;
    const void* twx;         // FP64 twiddles of the x and y transforms
    const void* twy;
    const void* scales;      // [capacity][m][SC_COLS], run precision
    RowGeom rg;              // x rows of all slots
    AxisGeom gy;             // y pencils of all slots
    int64_t npts;            // points per instance
    const int64_t* pidx;     // [capacity][nprobes] probe indices
    const int* active;       // [capacity]
    double* probes;          // [capacity][capacity_samples][nprobes][2]
    int64_t* counter;        // [capacity] next sample slot
    int64_t samples;         // sample slots per instance
    int* fault;              // probe index fault flag
};

// Tile: block `blk` of member `member`'s own grid for one pass kind.
struct MixTile {
    int member;
    int blk;
};

// Schedule variants of the mixed kernels, chosen at run time: waves per
// block (2 or 4), the LDS exchange of the fused x pass (joint real and
// imaginary parts for rows shorter than 512 points, or split), and complex
// pencils per lane group of the y passes (1 or 2).
struct MixVariant {
    int wpb;
    int x_joint;
    int y_ppl;
};

// Blocks of one member's grid for a pass kind under variant v:
// kind 0 the fused x pass, 1 the y passes.
int64_t mix_blocks(int kind, int nx, int ny, int64_t capacity, int precision_bytes, const MixVariant& v);

// The launchers below run the tile-per-block kernels when grid >= ntiles,
// else the persistent kernels on `grid` blocks.
// Fused A and B halves along x for every member (stage l of m).
template <typename R>
hipError_t launch_mix_x_ab(const MixMember<R>* mem, const MixTile* tiles, int ntiles, int grid, int m, int l,
                           int nyq_zero, const MixVariant& v, hipStream_t st);
// The y pass of a half-stage for every member: b_half 0 (A: psi_R += T_y
// psi_I, column SC_KYA) or 1 (B: psi_I += T_y psi_R, column SC_KYB).
template <typename R>
hipError_t launch_mix_axis_acc(const MixMember<R>* mem, const MixTile* tiles, int ntiles, int grid, int m,
                               int l, int b_half, int nyq_zero, const MixVariant& v, hipStream_t st);
// The y sweep at a stage boundary (B half of stage lB, A half of lA).
template <typename R>
hipError_t launch_mix_axis_ba(const MixMember<R>* mem, const MixTile* tiles, int ntiles, int grid, int m,
                              int lB, int lA, int nyq_zero, const MixVariant& v, hipStream_t st);
// Probe samples of every active slot of every member (as launch_probe_batch,
// with its parts); slots[i] = (member, slot).
template <typename R>
hipError_t launch_mix_probe(const MixMember<R>* mem, const MixTile* slots, int nslots, int nprobes,
                            hipStream_t st, int part = PROBE_FULL);

}  // namespace spstd
