// Host engine behind the C ABI: plan validation, time step, workspace
// layout, stage sequencing of the directional passes, step-chunk HIP graphs,
// probe recording, norms, checkpoints and the RK4 comparison integrator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/spstd.h"
#include "host_common.hpp"
#include "kernels.hpp"
#include "resident.hpp"

namespace spstd {

// classical RK4 on an oscillation: stable while |x| <= 2 sqrt(2)
static const double kRK4Edge = 2.8284271247461900976;

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
// Rows of a plan's scale table: one per stage, the RK4 row, and the row of a
// merged step boundary.
static int scale_rows(const spstd_desc& d) { return d.m + 2; }

struct Layout {
    size_t psiR, psiI, V, rk[6], tw[3], pidx, probes, counter, psave, partials, rinst, scales, eig, ecount, total;
};

static const int kNormBlocks = 256;

// Axis whose passes are fused at stage boundaries (y; fusing z instead
// measured equal at 256^3).
static const int kFuseAxis = 1;
static const int kGraphChunk = 16;

struct Plan {
    spstd_desc d;
    double c[SPSTD_MAX_STAGES], dd[SPSTD_MAX_STAGES];
    int64_t probe_idx[SPSTD_MAX_PROBES];
    double dt, xmax, rho, norm0, norm, cellvol;
    int64_t N, nsteps_max, steps_done;
    size_t esz;
    char* ws;
    Layout L;
    // device fields psi_R, psi_I, V and the FP64 probe buffer: pieces of the
    // workspace, or the caller's own arrays (spstd_run_noalloc)
    char *fR, *fI, *fV;
    double* prb;
    hipStream_t st;
    hipGraphExec_t graph;
    bool graph_ready;
    bool eig_on = false;
    EigParams eig{};
    std::string err;
    // SPSTD_TIMING: events recorded on the stream in order, and the (start,
    // end, kind) of each timed pass; ev_open: the last event ends a timed
    // pass and nothing was enqueued after it, so it also starts the next one
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::array<int, 3>> ev_span;
    size_t ev_used = 0;
    bool ev_open = false;
    int64_t acc_n[SPSTD_NPASS_KINDS] = {0};
    double acc_ms[SPSTD_NPASS_KINDS] = {0.0};
};

// Record the next event of the pool on the plan's stream; -1 if none.
static int ev_record(Plan* p) {
    if (p->ev_used == p->ev_pool.size()) {
        // timing only: no system-scope fence (cache write-back and
        // invalidate) when an event completes, which would otherwise cost
        // every bracketed pass a few microseconds
        hipEvent_t a;
        if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess) return -1;
        p->ev_pool.push_back(a);
    }
    const int k = (int)p->ev_used;
    if (hipEventRecord(p->ev_pool[k], p->st) != hipSuccess) return -1;
    ++p->ev_used;
    return k;
}

// Work enqueued outside a timed pass: the next pass records its own start.
static void ev_break(Plan* p) { p->ev_open = false; }

// Brackets one pass launch with HIP events on the plan's stream when the
// plan times its passes (timing plans launch eagerly, never from a graph).
// Back-to-back passes share the event between them.
struct PassTimer {
    Plan* p;
    int start, kind;
    PassTimer(Plan* pl, int k) : p(pl), start(-1), kind(k) {
        if (!(p->d.flags & SPSTD_TIMING)) return;
        start = p->ev_open ? (int)p->ev_used - 1 : ev_record(p);
    }
    ~PassTimer() {
        if (start < 0) return;
        const int end = ev_record(p);
        p->ev_open = end >= 0;
        if (end >= 0) p->ev_span.push_back({start, end, kind});
    }
};

// Add the durations of completed passes to the per-kind totals.
static hipError_t harvest(Plan* p) {
    for (const auto& sp : p->ev_span) {
        float t = 0.0f;
        hipError_t e = hipEventElapsedTime(&t, p->ev_pool[sp[0]], p->ev_pool[sp[1]]);
        if (e != hipSuccess) return e;
        p->acc_n[sp[2]] += 1;
        p->acc_ms[sp[2]] += t;
    }
    return hipSuccess;
}


static bool pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

static spstd_status validate(const spstd_desc* d, std::string* why) {
    if (!d) { *why = "null descriptor"; return SPSTD_ERR_ARG; }
    if (d->ndim < 1 || d->ndim > 3) { *why = "ndim must be 1, 2 or 3"; return SPSTD_ERR_ARG; }
    for (int a = 0; a < 3; ++a) {
        if (d->bc[a] != SPSTD_BC_PERIODIC && d->bc[a] != SPSTD_BC_DIRICHLET && d->bc[a] != SPSTD_BC_NEUMANN) {
            *why = "bad boundary code"; return SPSTD_ERR_ARG;
        }
        if (a < d->ndim) {
            const bool wall = d->bc[a] != SPSTD_BC_PERIODIC;
            const int64_t nt = wall ? 2 * d->n[a] : d->n[a];
            bool ok = (a == 0) ? row_len_ok(nt) : axis_len_ok(nt);
            if (wall && d->n[a] < 16) ok = false;
            // a walled axis of at most 32 cells of any count
            if (wall && wall_dft_len_ok(d->n[a])) ok = true;
            if (!ok) {
                *why = "axis length must be a power of two (x: 16..16384, y/z: 16..1024; walled: half "
                       "that, or any 2..32 cells)";
                return SPSTD_ERR_ARG;
            }
            if (!(d->dx[a] > 0.0) || !std::isfinite(d->dx[a])) { *why = "dx must be positive"; return SPSTD_ERR_ARG; }
        } else if (d->n[a] != 1) {
            *why = "unused axes must have length 1";
            return SPSTD_ERR_ARG;
        }
    }
    if (!(d->hbar > 0.0) || !(d->mass > 0.0) || !std::isfinite(d->hbar) || !std::isfinite(d->mass)) {
        *why = "hbar and mass must be positive"; return SPSTD_ERR_ARG;
    }
    if (d->precision != SPSTD_FP64 && d->precision != SPSTD_FP32) { *why = "bad precision"; return SPSTD_ERR_ARG; }
    if (d->method != SPSTD_SYMPLECTIC && d->method != SPSTD_RK4) { *why = "bad method"; return SPSTD_ERR_ARG; }
    if (d->m < 0 || d->m > SPSTD_MAX_STAGES) { *why = "m must be 0..16"; return SPSTD_ERR_ARG; }
    if (d->method == SPSTD_SYMPLECTIC) {
        if (d->m < 1 || d->m > SPSTD_MAX_STAGES || !d->c || !d->d) { *why = "m must be 1..16 with c, d"; return SPSTD_ERR_ARG; }
        for (int l = 0; l < d->m; ++l)
            if (!std::isfinite(d->c[l]) || !std::isfinite(d->d[l])) { *why = "non-finite coefficient"; return SPSTD_ERR_ARG; }
    }
    if (d->nyquist != SPSTD_NYQ_FULL && d->nyquist != SPSTD_NYQ_ZERO) { *why = "bad nyquist"; return SPSTD_ERR_ARG; }
    if (d->laplacian != SPSTD_LAP_SPECTRAL && d->laplacian != SPSTD_LAP_FD3) { *why = "bad laplacian"; return SPSTD_ERR_ARG; }
    if (d->neig < 0 || d->neig > SPSTD_MAX_EIG) { *why = "neig must be 0..8"; return SPSTD_ERR_ARG; }
    if (d->laplacian == SPSTD_LAP_FD3)
        for (int a = 0; a < 3; ++a)
            if (d->bc[a] != SPSTD_BC_PERIODIC) { *why = "the difference operator is periodic only"; return SPSTD_ERR_ARG; }
    if (!(d->dt >= 0.0) || !std::isfinite(d->dt)) { *why = "dt must be >= 0"; return SPSTD_ERR_ARG; }
    if (d->dt == 0.0 && !(d->cfl_fraction > 0.0 && std::isfinite(d->cfl_fraction))) {
        *why = "cfl_fraction must be positive when dt is 0"; return SPSTD_ERR_ARG;
    }
    if (d->nprobes < 0 || d->nprobes > SPSTD_MAX_PROBES || (d->nprobes > 0 && !d->probe_idx)) {
        *why = "nprobes must be 0..64"; return SPSTD_ERR_ARG;
    }
    const int64_t N = d->n[0] * d->n[1] * d->n[2];
    for (int p = 0; p < d->nprobes; ++p)
        if (d->probe_idx[p] < 0 || d->probe_idx[p] >= N) { *why = "probe index out of range"; return SPSTD_ERR_ARG; }
    return SPSTD_OK;
}

static double rho_of(const spstd_desc* d, const double* V, int64_t N) {
    return rho_bound_of(d->ndim, d->dx, d->hbar, d->mass, V, N, d->laplacian == SPSTD_LAP_FD3);
}

static spstd_status edge_of(const spstd_desc* d, double* x) {
    if (d->method == SPSTD_RK4) { *x = kRK4Edge; return SPSTD_OK; }
    return xmax_symplectic(d->m, d->c, d->d, x) ? SPSTD_OK : SPSTD_ERR_ARG;
}

// Workspace pieces of a plan.  external: the fields and the probe buffer
// are the caller's own device arrays (spstd_run_noalloc) and take no room.
static Layout layout_of(const spstd_desc* d, int64_t nsteps_max, bool external = false) {
    Layout L{};
    const int64_t N = d->n[0] * d->n[1] * d->n[2];
    const size_t esz = d->precision == SPSTD_FP64 ? 8 : 4;
    const size_t fb = external ? 0 : align256((size_t)N * esz);
    size_t off = 0;
    // the fields sit back to back (padding between them, to shift their
    // placement across memory channels, measured neutral at 4 KB and 52 KB
    // and slower from 1 MB at 256^3)
    L.psiR = off; off += fb;
    L.psiI = off; off += fb;
    L.V = off; off += fb;
    for (int k = 0; k < 6; ++k) {
        L.rk[k] = off;
        if (d->method == SPSTD_RK4) off += fb;
    }
    for (int a = 0; a < 3; ++a) {
        // FP64 twiddle tables in every precision
        L.tw[a] = off;
        if (a < d->ndim) off += align256((size_t)transform_len(*d, a) * 2 * sizeof(double));
    }
    L.pidx = off; off += align256(sizeof(int64_t) * (size_t)(d->nprobes > 0 ? d->nprobes : 1));
    L.probes = off;
    if (!external)
        off += align256(sizeof(double) * 2 * (size_t)(d->nprobes > 0 ? d->nprobes : 1) * (size_t)(nsteps_max + 1));
    // the device step counter (int64), then the probe-index fault flag (int)
    L.counter = off; off += 256;
    // probe values saved around a merged step boundary: psi_R before, psi_I
    L.psave = off; off += align256(sizeof(double) * 2 * SPSTD_MAX_PROBES);
    // norm partials, then the energy sums: kinetic per axis, potential, norm
    L.partials = off; off += align256(sizeof(double) * kNormBlocks * 6);
    L.rinst = off; off += align256(sizeof(ResidentInst<double>));
    // per-stage pass scales, then one row for the RK4 operator applications
    L.scales = off; off += align256((size_t)scale_rows(*d) * SC_COLS * esz);
    // eigenstate accumulators: neig complex FP64 fields, then their step count
    L.eig = off; off += align256((size_t)d->neig * 2 * (size_t)N * sizeof(double));
    L.ecount = off; off += 256;
    L.total = off;
    return L;
}

template <typename R>
static R* F(Plan* p, size_t off) { return reinterpret_cast<R*>(p->ws + off); }
template <typename R>
static R* FR(Plan* p) { return reinterpret_cast<R*>(p->fR); }
template <typename R>
static R* FI(Plan* p) { return reinterpret_cast<R*>(p->fI); }
template <typename R>
static R* FV(Plan* p) { return reinterpret_cast<R*>(p->fV); }

// Set by a probe kernel that met a device-side probe index outside the grid.
static int* fault_flag(Plan* p) { return reinterpret_cast<int*>(p->ws + p->L.counter + sizeof(int64_t)); }

#define HIPCHK(x)                                                   \
    do {                                                            \
        hipError_t e_ = (x);                                        \
        if (e_ != hipSuccess) {                                     \
            p->err = std::string(#x) + ": " + hipGetErrorString(e_); \
            return SPSTD_ERR_DEVICE;                                \
        }                                                           \
    } while (0)

template <typename R>
static spstd_status upload(Plan* p, char* dst, const double* src) {
    const int64_t N = p->N;
    if (sizeof(R) == 8) {
        if (src) HIPCHK(hipMemcpyAsync(dst, src, N * 8, hipMemcpyHostToDevice, p->st));
        else HIPCHK(launch_fill0<R>(N, reinterpret_cast<R*>(dst), p->st));
    } else {
        if (src) {
            std::vector<float> tmp(N);
            for (int64_t i = 0; i < N; ++i) tmp[i] = (float)src[i];
            HIPCHK(hipMemcpyAsync(dst, tmp.data(), N * 4, hipMemcpyHostToDevice, p->st));
            HIPCHK(hipStreamSynchronize(p->st));   // tmp goes out of scope
        } else {
            HIPCHK(launch_fill0<R>(N, reinterpret_cast<R*>(dst), p->st));
        }
    }
    return SPSTD_OK;
}

static_assert(WALL_NONE == SPSTD_BC_PERIODIC && WALL_DIRICHLET == SPSTD_BC_DIRICHLET &&
                  WALL_NEUMANN == SPSTD_BC_NEUMANN,
              "kernel wall codes follow the ABI's boundary codes");

static bool walled(const Plan* p, int a) { return p->d.bc[a] != SPSTD_BC_PERIODIC; }

// Lines of axis a of the plan's grid, for the line-generic kernels.
static EnergyGeom lines_of(const Plan* p, int a) {
    const int64_t nx = p->d.n[0], ny = p->d.n[1], nz = p->d.n[2];
    if (a == 0) return EnergyGeom{ny * nz, 1, nx, 1};
    if (a == 1) return EnergyGeom{nz * nx, nx, nx * ny, nx};
    return EnergyGeom{ny * nx, nx * ny, p->N, nx * ny};
}

// dst += T_a src along axis a = 1 (y) or 2 (z), scale column col.
template <typename R>
static hipError_t axis_pass(Plan* p, int a, const R* src, R* dst, const ScaleRef& sc, int col) {
    PassTimer tm(p, a == 1 ? SPSTD_PASS_Y : SPSTD_PASS_Z);
    return walled(p, a)
        ? launch_wall_acc<R>(p->d.n[a], 0, p->d.bc[a], src, dst, nullptr, p->ws + p->L.tw[a], lines_of(p, a),
                             p->N, sc, col, -1, p->d.nyquist, p->st)
        : launch_axis_acc<R>(p->d.n[a], src, dst, p->ws + p->L.tw[a], axis_geom_of(p->d, a, 1), sc, col,
                             p->d.nyquist, p->st);
}

// dst += T_{y,z} src for every axis beyond x, with the scale columns of the
// A (ab = 0) or B (ab = 1) substep
template <typename R>
static hipError_t yz_passes(Plan* p, const R* src, R* dst, const ScaleRef& sc, int ab) {
    for (int a = 1; a < p->d.ndim; ++a) {
        hipError_t e = axis_pass<R>(p, a, src, dst, sc, (ab ? SC_KXB : SC_KXA) + a);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// dst += (three-point T) src + (V/hbar) src over all axes at once, with the
// kinetic columns of the A (ab = 0) or B (ab = 1) substep.
template <typename R>
static hipError_t fd_half(Plan* p, const R* src, R* dst, const ScaleRef& sc, int ab) {
    PassTimer tm(p, SPSTD_PASS_X);
    return launch_fd_acc<R>(src, dst, FV<R>(p), p->d.n, sc, ab ? SC_KXB : SC_KXA, ab ? SC_PB : SC_PA,
                            p->st);
}

// dst += T_x src + (V/hbar) src with the scale columns (kcol, pcol): one x
// half-stage.
template <typename R>
static hipError_t x_half(Plan* p, const R* src, R* dst, const ScaleRef& sc, int kcol, int pcol) {
    const R* V = FV<R>(p);
    const void* twx = p->ws + p->L.tw[0];
    if (walled(p, 0))
        return launch_wall_acc<R>(p->d.n[0], 1, p->d.bc[0], src, dst, V, twx, lines_of(p, 0), p->N, sc, kcol,
                                  pcol, p->d.nyquist, p->st);
    const RowGeom rg{p->N / p->d.n[0], p->N / p->d.n[0]};
    return launch_x_acc<R>(p->d.n[0], src, dst, V, twx, rg, sc, kcol, pcol, p->d.nyquist, p->st);
}

// When the last stage of the set has no B half (d_m = 0), the A half that
// ends a step and the A half that opens the next one act on psi_R with the
// same psi_I (Eq. 18), so consecutive steps of one enqueue share them as a
// single A half with coefficient c_m + c_1 (the scale row after the RK4
// row), fused with the B half of stage 1.  The boundary state is never
// formed; its probe samples are interpolated from psi_R around the merged
// half (probes.hip).  Not with eigenstate sums (they need every step's
// state) or the difference operator.
// When the last stage has a B half, a step ends with the B half's own pass
// along the fused axis; between consecutive steps of one enqueue that pass
// and the first A half's pass along the same axis run as one sweep
// (launch_axis_ba), exactly as at the stage boundaries inside a step.  The
// step's end state is then never complete in memory at once: its probe
// samples take psi_R before the sweep (it leaves psi_R of the step alone
// until the A half adds to it) and psi_I after it (the A half leaves psi_I
// alone until the x pass).  Not with eigenstate sums, the difference
// operator, a walled fused axis or SPSTD_NO_MERGE.
static bool chains_steps(const Plan* p) {
    const spstd_desc& d = p->d;
    if (d.method != SPSTD_SYMPLECTIC || d.laplacian != SPSTD_LAP_SPECTRAL || p->eig_on || d.ndim < 2 ||
        d.bc[kFuseAxis] != SPSTD_BC_PERIODIC || (d.flags & SPSTD_NO_MERGE))
        return false;
    return p->dd[d.m - 1] != 0.0 && p->c[0] != 0.0;
}

static bool merges_steps(const Plan* p) {
    const spstd_desc& d = p->d;
    if (d.method != SPSTD_SYMPLECTIC || d.laplacian != SPSTD_LAP_SPECTRAL || p->eig_on || d.m < 2 ||
        (d.flags & SPSTD_NO_MERGE))
        return false;
    const double cl = p->c[d.m - 1], c1 = p->c[0];
    return p->dd[d.m - 1] == 0.0 && cl != 0.0 && c1 != 0.0 && cl + c1 != 0.0;
}

// Probe samples and eigenstate sums of a completed step.
template <typename R>
static hipError_t step_end(Plan* p) {
    hipError_t e = hipSuccess;
    if (p->d.nprobes > 0)
        e = launch_probe<R>(FR<R>(p), FI<R>(p), reinterpret_cast<const int64_t*>(p->ws + p->L.pidx),
                            p->d.nprobes, p->N, p->prb,
                            reinterpret_cast<int64_t*>(p->ws + p->L.counter), p->nsteps_max + 1, fault_flag(p),
                            p->st);
    if (e == hipSuccess && p->eig_on) {
        e = launch_eig_acc<R>(FR<R>(p), FI<R>(p), p->N, p->eig, p->st);
        if (e == hipSuccess) e = launch_count_tick(reinterpret_cast<int64_t*>(p->ws + p->L.ecount), p->st);
    }
    ev_break(p);
    return e;
}

// k symplectic steps, each followed by its probe samples; with merge,
// consecutive steps share their boundary A half (merges_steps).
template <typename R>
static hipError_t enqueue_symplectic_steps(Plan* p, int64_t k, bool merge) {
    R* pr = FR<R>(p);
    R* pi = FI<R>(p);
    const R* V = FV<R>(p);
    const RowGeom rg{p->N / p->d.n[0], p->N / p->d.n[0]};
    const int64_t nx = p->d.n[0];
    const void* twx = p->ws + p->L.tw[0];
    const int m = p->d.m, rows = scale_rows(p->d);
    const int64_t* pidx = reinterpret_cast<const int64_t*>(p->ws + p->L.pidx);
    double* save = reinterpret_cast<double*>(p->ws + p->L.psave);
    hipError_t e = hipSuccess;
    // The B half ends with the pass along axis fa (y) and the A half starts
    // with it, so the pass owed by
    // the B half of one stage and the first pass of the next A half are one
    // sweep of those pencils (launch_axis_ba).  Steps end with the owed pass
    // on its own: the probes sample the completed step.
    const int fa = kFuseAxis, oa = 3 - fa;
    const bool fuse = p->d.ndim >= 2 && !walled(p, fa);
    int owed = -1;   // scale row whose B half still owes its pass along fa
    auto owed_pass = [&](int row) -> hipError_t {
        const ScaleRef so{p->ws + p->L.scales, rows, row};
        return axis_pass<R>(p, fa, pr, pi, so, SC_KXB + fa);
    };
    // one stage: A half (a) with row's A columns, B half (b) with its B
    // columns; boundary: a merged or chained step boundary, whose probe
    // samples are taken around it: psi_R interpolated with weight w between
    // its values before and after the stage's A half, psi_I before the x pass
    auto stage = [&](int row, bool a, bool b, bool boundary, double w) -> hipError_t {
        const ScaleRef sc{p->ws + p->L.scales, rows, row};
        const bool smp = boundary && p->d.nprobes > 0;
        hipError_t r = hipSuccess;
        if (p->d.laplacian == SPSTD_LAP_FD3) {
            if (a) r = fd_half<R>(p, pi, pr, sc, 0);
            if (b && r == hipSuccess) r = fd_half<R>(p, pr, pi, sc, 1);
            return r;
        }
        if (smp) {
            // psi_R before the merged A half (B passes leave it alone)
            r = launch_probe_save<R>(pr, pidx, p->d.nprobes, p->N, save, fault_flag(p), p->st);
            ev_break(p);
            if (r != hipSuccess) return r;
        }
        if (a && owed >= 0) {
            const ScaleRef so{p->ws + p->L.scales, rows, owed};
            {
                PassTimer tm(p, SPSTD_PASS_YBA);
                r = launch_axis_ba<R>(p->d.n[fa], pr, pi, p->ws + p->L.tw[fa], axis_geom_of(p->d, fa, 1), so, sc,
                                      SC_KXB + fa, SC_KXA + fa, p->d.nyquist, p->st);
            }
            owed = -1;
            if (r == hipSuccess && p->d.ndim == 3) r = axis_pass<R>(p, oa, pi, pr, sc, SC_KXA + oa);
        } else {
            if (owed >= 0) {
                r = owed_pass(owed);
                owed = -1;
            }
            if (a && r == hipSuccess) r = yz_passes<R>(p, pi, pr, sc, 0);
        }
        if (r != hipSuccess) return r;
        if (smp) {
            // psi_I of the boundary state: every B pass before it is done
            r = launch_probe_save<R>(pi, pidx, p->d.nprobes, p->N, save + SPSTD_MAX_PROBES, fault_flag(p), p->st);
            ev_break(p);
            if (r != hipSuccess) return r;
        }
        if (a && b && !walled(p, 0)) {
            PassTimer tm(p, SPSTD_PASS_XAB);
            r = launch_x_ab<R>(nx, pr, pi, V, twx, rg, sc, p->d.nyquist, p->st);
        } else {
            if (a) {
                PassTimer tm(p, SPSTD_PASS_X);
                r = x_half<R>(p, pi, pr, sc, SC_KXA, SC_PA);
            }
            if (b && r == hipSuccess) {
                PassTimer tm(p, SPSTD_PASS_X);
                r = x_half<R>(p, pr, pi, sc, SC_KXB, SC_PB);
            }
        }
        if (r != hipSuccess) return r;
        if (smp) {
            r = launch_probe_merged<R>(pr, pidx, p->d.nprobes, p->N, save, save + SPSTD_MAX_PROBES, w,
                                       p->prb,
                                       reinterpret_cast<int64_t*>(p->ws + p->L.counter), p->nsteps_max + 1,
                                       fault_flag(p), p->st);
            ev_break(p);
            if (r != hipSuccess) return r;
        }
        if (b) {
            if (fuse) {
                if (p->d.ndim == 3) r = axis_pass<R>(p, oa, pr, pi, sc, SC_KXB + oa);
                owed = row;
            } else {
                r = yz_passes<R>(p, pr, pi, sc, 1);
            }
        }
        return r;
    };
    const bool chain = !merge && fuse && chains_steps(p);
    const double w_merge = merge ? p->c[m - 1] / (p->c[m - 1] + p->c[0]) : 0.0;
    for (int64_t s = 0; s < k && e == hipSuccess; ++s) {
        const bool head = merge && s > 0;        // stage 1's A half ran at the boundary before
        const bool tail = merge && s + 1 < k;    // the last A half runs merged with the next
        const bool chained = chain && s > 0;     // the previous step's owed pass runs fused with stage 1's
        ev_break(p);
        for (int l = head ? 1 : 0; l < m && e == hipSuccess; ++l) {
            if (l == m - 1 && tail)
                e = stage(m + 1, true, p->dd[0] != 0.0, true, w_merge);
            else
                e = stage(l, p->c[l] != 0.0, p->dd[l] != 0.0, l == 0 && chained, 0.0);
        }
        if (e != hipSuccess || tail || (chain && s + 1 < k)) continue;
        if (owed >= 0) {
            e = owed_pass(owed);
            owed = -1;
        }
        if (e == hipSuccess) e = step_end<R>(p);
    }
    return e;
}

// kout = (+K or -K) src  (K of Eq. 16), into a cleared buffer; the RK4 row of
// the scale table holds coefficient +1 in its A columns and -1 in its B columns
template <typename R>
static hipError_t apply_K(Plan* p, const R* src, R* kout, double coef) {
    const ScaleRef sc{p->ws + p->L.scales, scale_rows(p->d), p->d.m};
    const int ab = coef > 0.0 ? 0 : 1;
    hipError_t e = launch_fill0<R>(p->N, kout, p->st);
    ev_break(p);
    if (p->d.laplacian == SPSTD_LAP_FD3) return e == hipSuccess ? fd_half<R>(p, src, kout, sc, ab) : e;
    if (e == hipSuccess) e = yz_passes<R>(p, src, kout, sc, ab);
    PassTimer tm(p, SPSTD_PASS_X);
    if (e == hipSuccess) e = x_half<R>(p, src, kout, sc, ab ? SC_KXB : SC_KXA, ab ? SC_PB : SC_PA);
    return e;
}

template <typename R>
static hipError_t enqueue_rk4_step(Plan* p) {
    R* pr = FR<R>(p);
    R* pi = FI<R>(p);
    R* kR = F<R>(p, p->L.rk[0]);
    R* kI = F<R>(p, p->L.rk[1]);
    R* yR = F<R>(p, p->L.rk[2]);
    R* yI = F<R>(p, p->L.rk[3]);
    R* aR = F<R>(p, p->L.rk[4]);
    R* aI = F<R>(p, p->L.rk[5]);
    const int64_t N = p->N;
    const double dt = p->dt;
    static const double wgt[4] = {1.0, 2.0, 2.0, 1.0};
    static const double nxt[3] = {0.5, 0.5, 1.0};
    hipError_t e = launch_fill0<R>(N, aR, p->st);
    if (e == hipSuccess) e = launch_fill0<R>(N, aI, p->st);
    for (int s = 0; s < 4 && e == hipSuccess; ++s) {
        const R* inR = s ? yR : pr;
        const R* inI = s ? yI : pi;
        e = apply_K<R>(p, inI, kR, 1.0);                 // d psi_R / dt =  K psi_I
        if (e == hipSuccess) e = apply_K<R>(p, inR, kI, -1.0);   // d psi_I / dt = -K psi_R
        if (e == hipSuccess) e = launch_axpby<R>(N, wgt[s], kR, 1.0, aR, p->st);
        if (e == hipSuccess) e = launch_axpby<R>(N, wgt[s], kI, 1.0, aI, p->st);
        if (s < 3) {
            if (e == hipSuccess) e = launch_xpay<R>(N, pr, nxt[s] * dt, kR, yR, p->st);
            if (e == hipSuccess) e = launch_xpay<R>(N, pi, nxt[s] * dt, kI, yI, p->st);
        }
        ev_break(p);
    }
    if (e == hipSuccess) e = launch_axpby<R>(N, dt / 6.0, aR, 1.0, pr, p->st);
    if (e == hipSuccess) e = launch_axpby<R>(N, dt / 6.0, aI, 1.0, pi, p->st);
    ev_break(p);
    return e;
}

static bool uses_resident(const Plan* p) {
    const spstd_desc& d = p->d;
    const bool shape = (d.ndim == 1 && resident_len_ok(d.n[0])) ||
                       (d.ndim == 2 && resident2d_ok(d.n[0], d.n[1]) && d.bc[1] == SPSTD_BC_PERIODIC);
    return shape && d.bc[0] == SPSTD_BC_PERIODIC && d.laplacian == SPSTD_LAP_SPECTRAL && d.neig == 0 &&
           d.method == SPSTD_SYMPLECTIC && d.nprobes <= kResMaxProbes && d.m <= SPSTD_MAX_STAGES &&
           !(d.flags & (SPSTD_NO_RESIDENT | SPSTD_TIMING));
}

// The resident kernel's one-entry instance table for a 1D or small 2D plan.
template <typename R>
static spstd_status upload_resident_inst(Plan* p) {
    ResidentInst<R> I{};
    I.V = FV<R>(p);
    I.psiR = FR<R>(p);
    I.psiI = FI<R>(p);
    I.probes = p->prb;
    I.counter = reinterpret_cast<int64_t*>(p->ws + p->L.counter);
    I.fault = fault_flag(p);
    I.capacity = p->nsteps_max + 1;
    I.nprobes = p->d.nprobes;
    for (int q = 0; q < p->d.nprobes; ++q) I.probe_idx[q] = p->probe_idx[q];
    // kinetic scale per axis: (hbar/2m*) (2 pi/L)^2 / N for the bare k^2
    double kin[2] = {0.0, 0.0};
    for (int ax = 0; ax < p->d.ndim && ax < 2; ++ax) {
        const double k1 = 2.0 * kPi / ((double)p->d.n[ax] * p->d.dx[ax]);
        kin[ax] = p->d.hbar / (2.0 * p->d.mass) * k1 * k1 / (double)p->d.n[ax];
    }
    for (int l = 0; l < p->d.m; ++l) {
        const double a = p->c[l] * p->dt, b = -p->dd[l] * p->dt;
        I.kin[2 * l] = (R)(a * kin[0]);
        I.kin[2 * l + 1] = (R)(b * kin[0]);
        I.kin_y[2 * l] = (R)(a * kin[1]);
        I.kin_y[2 * l + 1] = (R)(b * kin[1]);
        I.pot[2 * l] = (R)(a / p->d.hbar);
        I.pot[2 * l + 1] = (R)(b / p->d.hbar);
    }
    HIPCHK(hipMemcpyAsync(p->ws + p->L.rinst, &I, sizeof(I), hipMemcpyHostToDevice, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    return SPSTD_OK;
}

template <typename R>
static hipError_t enqueue_steps_eager(Plan* p, int64_t n) {
    hipError_t e = hipSuccess;
    if (p->d.method == SPSTD_SYMPLECTIC) {
        // in chunks of the graph's length, so that eager and graph-replayed
        // runs merge the same step boundaries
        const bool merge = merges_steps(p);
        for (int64_t done = 0; done < n && e == hipSuccess; done += kGraphChunk)
            e = enqueue_symplectic_steps<R>(p, std::min<int64_t>(kGraphChunk, n - done), merge);
        return e;
    }
    for (int64_t s = 0; s < n && e == hipSuccess; ++s) {
        ev_break(p);
        e = enqueue_rk4_step<R>(p);
        if (e == hipSuccess) e = step_end<R>(p);
    }
    return e;
}

template <typename R>
static spstd_status build_graph(Plan* p) {
    hipStream_t cap;
    HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t user = p->st;
    p->st = cap;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = enqueue_steps_eager<R>(p, kGraphChunk);
        e = hipStreamEndCapture(cap, &g);
        if (e == hipSuccess) e = e2;
    }
    p->st = user;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        p->err = std::string("graph capture: ") + hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    p->graph_ready = true;
    return SPSTD_OK;
}

template <typename R>
static spstd_status enqueue_steps(Plan* p, int64_t n) {
    if (uses_resident(p)) {
        const ResidentInst<R>* tab = reinterpret_cast<const ResidentInst<R>*>(p->ws + p->L.rinst);
        if (n > 0 && p->d.ndim == 1)
            HIPCHK(launch_resident_1d<R>(p->d.n[0], tab, 1, p->d.m, n, p->d.nyquist, p->ws + p->L.tw[0], p->st));
        else if (n > 0)
            HIPCHK(launch_resident_2d<R>(p->d.n[0], p->d.n[1], tab, 1, p->d.m, n, p->d.nyquist, p->ws + p->L.tw[0],
                                         p->ws + p->L.tw[1], p->st));
        return SPSTD_OK;
    }
    const bool use_graph = !(p->d.flags & (SPSTD_EAGER | SPSTD_TIMING)) && n >= kGraphChunk;
    if (use_graph && !p->graph_ready) {
        spstd_status s = build_graph<R>(p);
        if (s != SPSTD_OK) return s;
    }
    int64_t left = n;
    if (use_graph) {
        for (; left >= kGraphChunk; left -= kGraphChunk) HIPCHK(hipGraphLaunch(p->graph, p->st));
    }
    HIPCHK(enqueue_steps_eager<R>(p, left));
    return SPSTD_OK;
}

template <typename R>
static spstd_status compute_norm(Plan* p, double* out) {
    HIPCHK(launch_norm_partials<R>(FR<R>(p), FI<R>(p), p->N,
                                   reinterpret_cast<double*>(p->ws + p->L.partials), kNormBlocks, p->st));
    double part[kNormBlocks];
    HIPCHK(hipMemcpyAsync(part, p->ws + p->L.partials, sizeof(part), hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    double s = 0.0;
    for (int i = 0; i < kNormBlocks; ++i) s += part[i];
    *out = s * p->cellvol;
    return SPSTD_OK;
}

// <H> pieces (Sec. 2.2, Eq. 16 times hbar), each times the cell volume:
// out[0] kinetic, out[1] potential, out[2] norm.  Synchronises the stream.
template <typename R>
static spstd_status compute_energy(Plan* p, double* out) {
    double* part = reinterpret_cast<double*>(p->ws + p->L.partials) + kNormBlocks;
    int nb[3] = {0, 0, 0};
    for (int a = 0; a < p->d.ndim; ++a)
        HIPCHK(launch_energy_axis<R>(p->d.n[a], a == 0, p->d.bc[a], FR<R>(p), FI<R>(p),
                                     p->ws + p->L.tw[a], lines_of(p, a), p->d.nyquist == SPSTD_NYQ_ZERO,
                                     part + a * kNormBlocks, kNormBlocks, &nb[a], p->st));
    HIPCHK(launch_energy_pot<R>(FR<R>(p), FI<R>(p), FV<R>(p), p->N,
                                part + 3 * kNormBlocks, part + 4 * kNormBlocks, kNormBlocks, p->st));
    std::vector<double> h((size_t)5 * kNormBlocks);
    HIPCHK(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    const double hb = p->d.hbar, ms = p->d.mass;
    double kin = 0.0;
    for (int a = 0; a < p->d.ndim; ++a) {
        double s = 0.0;
        for (int b = 0; b < nb[a]; ++b) s += h[(size_t)a * kNormBlocks + b];
        // a walled line enters as its mirrored extension, which counts each
        // sample twice
        const double nt = (double)transform_len(p->d, a);
        const double k1 = 2.0 * kPi / (nt * p->d.dx[a]);
        kin += hb * hb / (2.0 * ms) * k1 * k1 / nt * s * (walled(p, a) ? 0.5 : 1.0);
    }
    double pot = 0.0, nrm = 0.0;
    for (int b = 0; b < kNormBlocks; ++b) {
        pot += h[(size_t)3 * kNormBlocks + b];
        nrm += h[(size_t)4 * kNormBlocks + b];
    }
    out[0] = kin * p->cellvol;
    out[1] = pot * p->cellvol;
    out[2] = nrm * p->cellvol;
    return SPSTD_OK;
}

// Twiddle and scale tables, probe indices, the zeroed step counter and
// fault flag, probe sample 0 of the current fields, and the resident
// kernel's instance table.
template <typename R>
static spstd_status init_tables(Plan* p) {
    for (int a = 0; a < p->d.ndim; ++a) {
        // FP64 in every precision: the kernels round each twiddle once
        std::vector<double> t = twiddles(transform_len(p->d, a));
        const size_t room = (a < 2 ? p->L.tw[a + 1] : p->L.pidx) - p->L.tw[a];
        if (t.size() * 8 > room) {
            p->err = "twiddle table larger than its workspace region";
            return SPSTD_ERR_WORKSPACE;
        }
        HIPCHK(hipMemcpyAsync(p->ws + p->L.tw[a], t.data(), t.size() * 8, hipMemcpyHostToDevice, p->st));
        HIPCHK(hipStreamSynchronize(p->st));
    }
    {
        // stage rows (A coefficient c_l dt, B coefficient -d_l dt), the RK4
        // row (+1, -1), then the merged step-boundary row: A (c_m + c_1) dt,
        // B of stage 1
        const int rows = scale_rows(p->d);
        std::vector<double> tab((size_t)rows * SC_COLS, 0.0);
        for (int l = 0; l < p->d.m && p->d.method == SPSTD_SYMPLECTIC; ++l)
            scale_row(p->d, p->c[l] * p->dt, -p->dd[l] * p->dt, &tab[(size_t)l * SC_COLS]);
        scale_row(p->d, 1.0, -1.0, &tab[(size_t)p->d.m * SC_COLS]);
        if (p->d.method == SPSTD_SYMPLECTIC && p->d.m >= 2)
            scale_row(p->d, (p->c[p->d.m - 1] + p->c[0]) * p->dt, -p->dd[0] * p->dt,
                      &tab[(size_t)(p->d.m + 1) * SC_COLS]);
        std::vector<R> tr(tab.size());
        for (size_t i = 0; i < tab.size(); ++i) tr[i] = (R)tab[i];
        HIPCHK(hipMemcpyAsync(p->ws + p->L.scales, tr.data(), tr.size() * sizeof(R), hipMemcpyHostToDevice, p->st));
        HIPCHK(hipStreamSynchronize(p->st));
    }
    if (p->d.nprobes > 0)
        HIPCHK(hipMemcpyAsync(p->ws + p->L.pidx, p->probe_idx, sizeof(int64_t) * p->d.nprobes,
                              hipMemcpyHostToDevice, p->st));
    // step counter and fault flag start at zero (a fill kernel, not a memset)
    HIPCHK(launch_fill0<int64_t>(2, reinterpret_cast<int64_t*>(p->ws + p->L.counter), p->st));
    if (p->d.nprobes > 0)
        HIPCHK(launch_probe<R>(FR<R>(p), FI<R>(p),
                               reinterpret_cast<const int64_t*>(p->ws + p->L.pidx), p->d.nprobes, p->N,
                               p->prb,
                               reinterpret_cast<int64_t*>(p->ws + p->L.counter), p->nsteps_max + 1, fault_flag(p),
                               p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    if (uses_resident(p)) {
        spstd_status s2 = upload_resident_inst<R>(p);
        if (s2 != SPSTD_OK) return s2;
    }
    return SPSTD_OK;
}

template <typename R>
static spstd_status plan_init(Plan* p, const double* V, const double* psiR0, const double* psiI0) {
    spstd_status s;
    if ((s = upload<R>(p, p->fR, psiR0)) != SPSTD_OK) return s;
    if ((s = upload<R>(p, p->fI, psiI0)) != SPSTD_OK) return s;
    if ((s = upload<R>(p, p->fV, V)) != SPSTD_OK) return s;
    if ((s = init_tables<R>(p)) != SPSTD_OK) return s;
    return compute_norm<R>(p, &p->norm0);
}

template <typename R>
static spstd_status get_state_t(Plan* p, double* psiR, double* psiI) {
    const int64_t N = p->N;
    std::vector<R> tmp(N);
    double* outs[2] = {psiR, psiI};
    const char* srcs[2] = {p->fR, p->fI};
    for (int k = 0; k < 2; ++k) {
        if (!outs[k]) continue;
        HIPCHK(hipMemcpyAsync(tmp.data(), srcs[k], N * sizeof(R), hipMemcpyDeviceToHost, p->st));
        HIPCHK(hipStreamSynchronize(p->st));
        for (int64_t i = 0; i < N; ++i) outs[k][i] = (double)tmp[i];
    }
    return SPSTD_OK;
}

}  // namespace spstd

using namespace spstd;

struct spstd_plan_s : Plan {};

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

spstd_status spstd_xmax(int m, const double* c, const double* d, double* xmax_out) {
    if (m < 1 || m > SPSTD_MAX_STAGES || !c || !d || !xmax_out) return SPSTD_ERR_ARG;
    for (int l = 0; l < m; ++l)
        if (!std::isfinite(c[l]) || !std::isfinite(d[l])) return SPSTD_ERR_ARG;
    return xmax_symplectic(m, c, d, xmax_out) ? SPSTD_OK : SPSTD_ERR_ARG;
}

spstd_status spstd_stable_dt(const spstd_desc* desc, const double* V, double* dt_out) {
    std::string why;
    spstd_status s = validate(desc, &why);
    if (s != SPSTD_OK) return s;
    if (!V || !dt_out) return SPSTD_ERR_ARG;
    double x;
    if ((s = edge_of(desc, &x)) != SPSTD_OK) return s;
    const int64_t N = desc->n[0] * desc->n[1] * desc->n[2];
    const double f = desc->cfl_fraction > 0.0 ? desc->cfl_fraction : 1.0;
    *dt_out = f * x / rho_of(desc, V, N);
    return SPSTD_OK;
}

spstd_status spstd_workspace_size(const spstd_desc* desc, int64_t nsteps_max, size_t* bytes) {
    std::string why;
    spstd_status s = validate(desc, &why);
    if (s != SPSTD_OK) return s;
    if (nsteps_max < 0 || !bytes) return SPSTD_ERR_ARG;
    *bytes = layout_of(desc, nsteps_max).total;
    return SPSTD_OK;
}

spstd_status spstd_plan(const spstd_desc* desc, const double* V, const double* psiR0, const double* psiI0,
                        void* d_workspace, size_t ws_bytes, int64_t nsteps_max, void* stream,
                        spstd_plan_t* out) {
    if (!out) return SPSTD_ERR_ARG;
    *out = nullptr;
    std::string why;
    spstd_status s = validate(desc, &why);
    if (s != SPSTD_OK) return s;
    if (!V || !psiR0 || nsteps_max < 0) return SPSTD_ERR_ARG;
    const int64_t N = desc->n[0] * desc->n[1] * desc->n[2];
    for (int64_t i = 0; i < N; ++i)
        if (!std::isfinite(V[i]) || !std::isfinite(psiR0[i]) || (psiI0 && !std::isfinite(psiI0[i])))
            return SPSTD_ERR_ARG;
    Layout L = layout_of(desc, nsteps_max);
    if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace & 255)) return SPSTD_ERR_WORKSPACE;
    double x;
    if ((s = edge_of(desc, &x)) != SPSTD_OK) return s;
    const double rho = rho_of(desc, V, N);
    double dt = desc->dt > 0.0 ? desc->dt : desc->cfl_fraction * x / rho;
    if (!(desc->flags & SPSTD_ALLOW_UNSTABLE) && dt * rho >= x) return SPSTD_ERR_UNSTABLE;

    spstd_plan_s* p = new (std::nothrow) spstd_plan_s();
    if (!p) return SPSTD_ERR_DEVICE;
    p->d = *desc;
    for (int l = 0; l < desc->m && desc->method == SPSTD_SYMPLECTIC; ++l) {
        p->c[l] = desc->c[l];
        p->dd[l] = desc->d[l];
    }
    p->d.c = p->c;
    p->d.d = p->dd;
    for (int q = 0; q < desc->nprobes; ++q) p->probe_idx[q] = desc->probe_idx[q];
    p->d.probe_idx = p->probe_idx;
    p->dt = dt;
    p->xmax = x;
    p->rho = rho;
    p->N = N;
    p->nsteps_max = nsteps_max;
    p->steps_done = 0;
    p->esz = desc->precision == SPSTD_FP64 ? 8 : 4;
    p->ws = (char*)d_workspace;
    p->L = L;
    p->fR = p->ws + L.psiR;
    p->fI = p->ws + L.psiI;
    p->fV = p->ws + L.V;
    p->prb = reinterpret_cast<double*>(p->ws + L.probes);
    p->st = (hipStream_t)stream;
    p->graph_ready = false;
    p->cellvol = 1.0;
    for (int a = 0; a < desc->ndim; ++a) p->cellvol *= desc->dx[a];
    s = (desc->precision == SPSTD_FP64) ? plan_init<double>(p, V, psiR0, psiI0)
                                        : plan_init<float>(p, V, psiR0, psiI0);
    if (s != SPSTD_OK) {
        delete p;
        return s;
    }
    p->norm = p->norm0;
    *out = p;
    return SPSTD_OK;
}

spstd_status spstd_step(spstd_plan_t p, int64_t nsteps) {
    if (!p || nsteps < 0) return SPSTD_ERR_ARG;
    if (p->steps_done + nsteps > p->nsteps_max) {
        p->err = "probe buffer capacity exceeded";
        return SPSTD_ERR_CAPACITY;
    }
    spstd_status s = (p->esz == 8) ? enqueue_steps<double>(p, nsteps) : enqueue_steps<float>(p, nsteps);
    if (s == SPSTD_OK) p->steps_done += nsteps;
    return s;
}

spstd_status spstd_run(spstd_plan_t p, int64_t nsteps, double* probe_out, spstd_stats* stats) {
    spstd_status s = spstd_step(p, nsteps);
    if (s != SPSTD_OK) return s;
    s = (p->esz == 8) ? compute_norm<double>(p, &p->norm) : compute_norm<float>(p, &p->norm);
    if (s != SPSTD_OK) return s;
    if (p->d.nprobes > 0) {
        int fault = 0;
        hipError_t e = hipMemcpyAsync(&fault, fault_flag(p), sizeof(int), hipMemcpyDeviceToHost, p->st);
        if (e == hipSuccess && probe_out) {
            const size_t bytes = sizeof(double) * 2 * p->d.nprobes * (size_t)(p->steps_done + 1);
            e = hipMemcpyAsync(probe_out, p->prb, bytes, hipMemcpyDeviceToHost, p->st);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(p->st);
        if (e != hipSuccess) {
            p->err = hipGetErrorString(e);
            return SPSTD_ERR_DEVICE;
        }
        if (fault) {
            p->err = "a probe index in device memory lies outside the grid (samples skipped)";
            return SPSTD_ERR_DEVICE;
        }
    }
    if (stats) spstd_plan_info(p, stats);
    if (!std::isfinite(p->norm)) {
        p->err = "state is not finite";
        return SPSTD_ERR_NONFINITE;
    }
    return SPSTD_OK;
}

spstd_status spstd_eig_begin(spstd_plan_t p, const double* E, int nE, int64_t nsteps) {
    if (!p || !E || p->d.neig == 0 || nE < 1 || nE > p->d.neig || nsteps < 2) return SPSTD_ERR_ARG;
    for (int k = 0; k < nE; ++k)
        if (!std::isfinite(E[k])) return SPSTD_ERR_ARG;
    EigParams ep{};
    for (int k = 0; k < nE; ++k) ep.E[k] = E[k];
    ep.nE = nE;
    ep.M = nsteps;
    ep.dt_over_hbar = p->dt / p->d.hbar;
    ep.acc = reinterpret_cast<double*>(p->ws + p->L.eig);
    ep.count = reinterpret_cast<const int64_t*>(p->ws + p->L.ecount);
    HIPCHK(launch_fill0<double>((int64_t)nE * 2 * p->N, ep.acc, p->st));
    HIPCHK(launch_fill0<int64_t>(1, reinterpret_cast<int64_t*>(p->ws + p->L.ecount), p->st));
    // the step graph holds the accumulation's arguments: capture it again
    if (p->graph_ready) {
        HIPCHK(hipStreamSynchronize(p->st));
        (void)hipGraphExecDestroy(p->graph);
        p->graph_ready = false;
    }
    p->eig = ep;
    p->eig_on = true;
    return SPSTD_OK;
}

spstd_status spstd_eig_read(spstd_plan_t p, int k, double* re, double* im) {
    if (!p || !re || !im || !p->eig_on || k < 0 || k >= p->eig.nE) return SPSTD_ERR_ARG;
    std::vector<double> tmp((size_t)2 * p->N);
    HIPCHK(hipMemcpyAsync(tmp.data(), p->eig.acc + (size_t)2 * k * p->N, tmp.size() * sizeof(double),
                          hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    for (int64_t i = 0; i < p->N; ++i) {
        re[i] = tmp[2 * i];
        im[i] = tmp[2 * i + 1];
    }
    return SPSTD_OK;
}

spstd_status spstd_energy(spstd_plan_t p, double* out) {
    if (!p || !out) return SPSTD_ERR_ARG;
    if (p->d.laplacian != SPSTD_LAP_SPECTRAL) {
        p->err = "energy diagnostics use the spectral second derivative";
        return SPSTD_ERR_ARG;
    }
    spstd_status s = (p->esz == 8) ? compute_energy<double>(p, out) : compute_energy<float>(p, out);
    if (s == SPSTD_OK && !(std::isfinite(out[0]) && std::isfinite(out[1]) && std::isfinite(out[2]))) {
        p->err = "state is not finite";
        return SPSTD_ERR_NONFINITE;
    }
    return s;
}

spstd_status spstd_plan_info(spstd_plan_t p, spstd_stats* st) {
    if (!p || !st) return SPSTD_ERR_ARG;
    st->steps_done = p->steps_done;
    st->dt = p->dt;
    st->xmax = p->xmax;
    st->rho = p->rho;
    st->norm0 = p->norm0;
    st->norm = p->norm;
    double subs = 0.0;
    if (p->d.method == SPSTD_RK4) subs = 8.0;
    else
        for (int l = 0; l < p->d.m; ++l) subs += (p->c[l] != 0.0) + (p->dd[l] != 0.0);
    st->substeps_per_step = subs;
    return SPSTD_OK;
}

spstd_status spstd_device_fields(spstd_plan_t p, void** psiR, void** psiI, void** V, double** probes) {
    if (!p) return SPSTD_ERR_ARG;
    if (psiR) *psiR = p->fR;
    if (psiI) *psiI = p->fI;
    if (V) *V = p->fV;
    if (probes) *probes = p->prb;
    return SPSTD_OK;
}

spstd_status spstd_get_state(spstd_plan_t p, double* psiR, double* psiI, int64_t* step) {
    if (!p || !psiR) return SPSTD_ERR_ARG;
    spstd_status s = (p->esz == 8) ? get_state_t<double>(p, psiR, psiI) : get_state_t<float>(p, psiR, psiI);
    if (s == SPSTD_OK && step) *step = p->steps_done;
    return s;
}

spstd_status spstd_set_state(spstd_plan_t p, const double* psiR, const double* psiI, int64_t step) {
    if (!p || !psiR || step < 0 || step > p->nsteps_max) return SPSTD_ERR_ARG;
    for (int64_t i = 0; i < p->N; ++i)
        if (!std::isfinite(psiR[i]) || (psiI && !std::isfinite(psiI[i]))) return SPSTD_ERR_ARG;
    spstd_status s = (p->esz == 8) ? upload<double>(p, p->fR, psiR) : upload<float>(p, p->fR, psiR);
    if (s == SPSTD_OK)
        s = (p->esz == 8) ? upload<double>(p, p->fI, psiI) : upload<float>(p, p->fI, psiI);
    if (s != SPSTD_OK) return s;
    // the next sample goes to slot step + 1; slot `step` holds this state
    int64_t next = step;
    hipError_t e = hipMemcpyAsync(p->ws + p->L.counter, &next, sizeof(next), hipMemcpyHostToDevice, p->st);
    if (e == hipSuccess && p->d.nprobes > 0) {
        e = (p->esz == 8)
                ? launch_probe<double>(FR<double>(p), FI<double>(p),
                                       reinterpret_cast<const int64_t*>(p->ws + p->L.pidx), p->d.nprobes, p->N,
                                       p->prb,
                                       reinterpret_cast<int64_t*>(p->ws + p->L.counter), p->nsteps_max + 1,
                                       fault_flag(p), p->st)
                : launch_probe<float>(FR<float>(p), FI<float>(p),
                                      reinterpret_cast<const int64_t*>(p->ws + p->L.pidx), p->d.nprobes, p->N,
                                      p->prb,
                                      reinterpret_cast<int64_t*>(p->ws + p->L.counter), p->nsteps_max + 1,
                                      fault_flag(p), p->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(p->st);
    if (e != hipSuccess) {
        p->err = hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    p->steps_done = step;
    return SPSTD_OK;
}

spstd_status spstd_destroy(spstd_plan_t p) {
    if (!p) return SPSTD_ERR_ARG;
    if (p->graph_ready) (void)hipGraphExecDestroy(p->graph);
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    delete p;
    return SPSTD_OK;
}

spstd_status spstd_pass_times(spstd_plan_t p, int64_t* launches, double* total_ms,
                              double* bytes_per_launch) {
    if (!p || !(p->d.flags & SPSTD_TIMING)) return SPSTD_ERR_ARG;
    const double fb = (double)p->N * (double)p->esz;
    // fields read + fields written once per launch
    const double per[SPSTD_NPASS_KINDS] = {3.0 * fb, 3.0 * fb, 5.0 * fb, 4.0 * fb, 4.0 * fb};
    hipError_t e = hipStreamSynchronize(p->st);
    if (e != hipSuccess) {
        p->err = hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    e = harvest(p);
    if (e != hipSuccess) {
        p->err = hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    p->ev_span.clear();
    p->ev_used = 0;
    p->ev_open = false;
    for (int k = 0; k < SPSTD_NPASS_KINDS; ++k) {
        if (launches) launches[k] = p->acc_n[k];
        if (total_ms) total_ms[k] = p->acc_ms[k];
        if (bytes_per_launch) bytes_per_launch[k] = per[k];
        p->acc_n[k] = 0;
        p->acc_ms[k] = 0.0;
    }
    return SPSTD_OK;
}

const char* spstd_strerror(spstd_status s) {
    switch (s) {
        case SPSTD_OK: return "ok";
        case SPSTD_ERR_ARG: return "invalid argument";
        case SPSTD_ERR_UNSTABLE: return "time step beyond the stability edge";
        case SPSTD_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
        case SPSTD_ERR_DEVICE: return "HIP runtime error";
        case SPSTD_ERR_NONFINITE: return "state is not finite";
        case SPSTD_ERR_CAPACITY: return "probe buffer capacity exceeded";
        case SPSTD_ERR_SCRATCH: return "working memory exceeds the fixed no-allocation scratch";
    }
    return "unknown status";
}

const char* spstd_last_error(spstd_plan_t p) { return p ? p->err.c_str() : "null plan"; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Run without allocation
// ---------------------------------------------------------------------------
// Working memory of spstd_run_noalloc: one file-scope device array, one copy
// per GPU, held until the process ends.  In host code its name stands for a
// host-side shadow, not a device address: the device address is looked up
// once per device (with that device current) and only that pointer is
// handed to kernels and copies.
static __device__ __align__(256) char scratch[SPSTD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

// Device address of the current device's scratch array.
static hipError_t scratch_of_current_device(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[dev] = ptr;
    }
    *out = static_cast<char*>(g_scratch[dev]);
    return hipSuccess;
}

extern "C" spstd_status spstd_run_noalloc(const spstd_desc* desc, const void* V, void* psiR, void* psiI,
                                          int64_t nsteps, double* probes, void* stream) {
    std::string why;
    spstd_status s = validate(desc, &why);
    if (s != SPSTD_OK) return s;
    if (desc->method != SPSTD_SYMPLECTIC || desc->neig != 0 || !(desc->dt > 0.0) ||
        (desc->flags & SPSTD_TIMING))
        return SPSTD_ERR_ARG;
    if (!V || !psiR || !psiI || nsteps < 0 || (desc->nprobes > 0 && !probes)) return SPSTD_ERR_ARG;
    const size_t esz = desc->precision == SPSTD_FP64 ? 8 : 4;
    if (((uintptr_t)V | (uintptr_t)psiR | (uintptr_t)psiI) & 255) return SPSTD_ERR_ARG;
    const Layout L = layout_of(desc, nsteps, true);
    if (L.total > SPSTD_NOALLOC_SCRATCH_BYTES) return SPSTD_ERR_SCRATCH;
    double x;
    if ((s = edge_of(desc, &x)) != SPSTD_OK) return s;
    char* ws = nullptr;
    if (scratch_of_current_device(&ws) != hipSuccess) return SPSTD_ERR_DEVICE;

    Plan p{};
    p.d = *desc;
    for (int l = 0; l < desc->m; ++l) {
        p.c[l] = desc->c[l];
        p.dd[l] = desc->d[l];
    }
    p.d.c = p.c;
    p.d.d = p.dd;
    for (int q = 0; q < desc->nprobes; ++q) p.probe_idx[q] = desc->probe_idx[q];
    p.d.probe_idx = p.probe_idx;
    // launches one by one: no graph is captured or instantiated
    p.d.flags |= SPSTD_EAGER;
    p.dt = desc->dt;
    p.xmax = x;
    p.rho = 0.0;
    p.N = desc->n[0] * desc->n[1] * desc->n[2];
    p.nsteps_max = nsteps;
    p.steps_done = 0;
    p.esz = esz;
    p.ws = ws;
    p.L = L;
    p.fR = static_cast<char*>(psiR);
    p.fI = static_cast<char*>(psiI);
    p.fV = const_cast<char*>(static_cast<const char*>(V));   // read only
    p.prb = probes;
    p.st = (hipStream_t)stream;
    p.graph_ready = false;
    p.cellvol = 1.0;
    Plan* pp = &p;
    s = esz == 8 ? init_tables<double>(pp) : init_tables<float>(pp);
    if (s == SPSTD_OK) s = esz == 8 ? enqueue_steps<double>(pp, nsteps) : enqueue_steps<float>(pp, nsteps);
    if (s != SPSTD_OK) return s;
    int fault = 0;
    hipError_t e = hipMemcpyAsync(&fault, fault_flag(pp), sizeof(int), hipMemcpyDeviceToHost, p.st);
    if (e == hipSuccess) e = hipStreamSynchronize(p.st);
    if (e != hipSuccess || fault) return SPSTD_ERR_DEVICE;
    return SPSTD_OK;
}
