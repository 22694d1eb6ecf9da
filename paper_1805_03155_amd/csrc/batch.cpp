// Batch engine: many independent instances of one shape advanced together.
//
// Slots are stacked in one buffer ([slot][z][y][x] for psi_R, psi_I, V) and
// every directional pass of a stage is one launch over all slots; each slot
// has its own row of the scale table (its dt, spacing, m* and hbar), its own
// probe points, probe buffer and step counter.  Free slots hold zero fields
// and zero scales, so they stay zero.  Short 1D batches, 2D batches of up
// to 64 x 64 points and 16^3 batches run a resident kernel (one launch per
// spstd_batch_step call for every active slot).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/spstd.h"
#include "host_common.hpp"
#include "kernels.hpp"
#include "resident.hpp"

namespace spstd {

struct BatchLayout {
    size_t psiR, psiI, V, tw[3], scales, pidx, active, counter, fault, probes, rinst;
    size_t twsub, fs;   // four-step x passes of long 1D rows: 128- and n/128-entry tables, scratch
    size_t total;
};

static const int kBatchGraphChunk = 16;

static BatchLayout batch_layout(const spstd_batch_desc* d) {
    BatchLayout L{};
    const int64_t npts = d->n[0] * d->n[1] * d->n[2];
    const size_t esz = d->precision == SPSTD_FP64 ? 8 : 4;
    const size_t cap = (size_t)d->capacity;
    const size_t fb = align256(cap * (size_t)npts * esz);
    const size_t np = (size_t)(d->nprobes > 0 ? d->nprobes : 1);
    size_t off = 0;
    L.psiR = off; off += fb;
    L.psiI = off; off += fb;
    L.V = off; off += fb;
    for (int a = 0; a < 3; ++a) {
        L.tw[a] = off;
        if (a < d->ndim) off += align256((size_t)d->n[a] * 2 * sizeof(double));
    }
    L.scales = off; off += align256(cap * (size_t)d->m * SC_COLS * esz);
    L.pidx = off; off += align256(cap * np * sizeof(int64_t));
    L.active = off; off += align256(cap * sizeof(int));
    L.counter = off; off += align256(cap * sizeof(int64_t));
    // set by a probe kernel that met a device-side probe index outside the grid
    L.fault = off; off += 256;
    L.probes = off; off += align256(cap * (size_t)(d->nsteps_max + 1) * np * 2 * sizeof(double));
    L.rinst = off; off += align256(cap * sizeof(ResidentInst<double>));
    if (d->ndim == 1 && fourstep_ok(d->n[0])) {
        L.twsub = off; off += align256((size_t)(128 + d->n[0] / 128) * 2 * sizeof(double));
        L.fs = off; off += align256(fourstep_scratch_bytes(d->n[0], d->capacity, esz));
    }
    L.total = off;
    return L;
}

struct Slot {
    bool active = false;
    double dt = 0.0, dx[3] = {1, 1, 1}, hbar = 1, mass = 1;
    int64_t steps = 0;
    int64_t probe_idx[kResMaxProbes] = {0};
};

struct Batch {
    spstd_batch_desc d;
    double c[SPSTD_MAX_STAGES], dd[SPSTD_MAX_STAGES];
    double xmax;
    int64_t npts;
    size_t esz;
    char* ws;
    BatchLayout L;
    hipStream_t st;
    std::vector<Slot> slots;
    bool resident;
    bool planes = false;        // 3D: the z and x passes of a stage as one launch per x-z plane
    bool fourstep = false;      // 1D long rows: x passes as four-step launches over many workgroups
    bool rtab_dirty = true;
    int nres = 0;               // active slots in the resident table
    hipGraphExec_t graph;
    bool graph_ready = false;
    int wpb = 0;                // waves per block of the pass kernels (0: built-in choice)
    double tuned_us[3] = {0.0, 0.0, 0.0};   // [resident, passes at 2 and 4 waves/block] per step
    std::string err;
};

#define BCHK(x)                                                      \
    do {                                                             \
        hipError_t e_ = (x);                                         \
        if (e_ != hipSuccess) {                                      \
            b->err = std::string(#x) + ": " + hipGetErrorString(e_); \
            return SPSTD_ERR_DEVICE;                                 \
        }                                                            \
    } while (0)

template <typename R>
static R* BF(Batch* b, size_t off) { return reinterpret_cast<R*>(b->ws + off); }

static spstd_status validate_batch(const spstd_batch_desc* d) {
    if (!d || d->ndim < 1 || d->ndim > 3) return SPSTD_ERR_ARG;
    for (int a = 0; a < 3; ++a) {
        if (a < d->ndim) {
            if (!((a == 0) ? row_len_ok(d->n[a]) : axis_len_ok(d->n[a]))) return SPSTD_ERR_ARG;
        } else if (d->n[a] != 1) {
            return SPSTD_ERR_ARG;
        }
    }
    if (d->precision != SPSTD_FP64 && d->precision != SPSTD_FP32) return SPSTD_ERR_ARG;
    if (d->m < 1 || d->m > SPSTD_MAX_STAGES || !d->c || !d->d) return SPSTD_ERR_ARG;
    for (int l = 0; l < d->m; ++l)
        if (!std::isfinite(d->c[l]) || !std::isfinite(d->d[l])) return SPSTD_ERR_ARG;
    if (d->nyquist != SPSTD_NYQ_FULL && d->nyquist != SPSTD_NYQ_ZERO) return SPSTD_ERR_ARG;
    if (d->capacity < 1 || d->capacity > (1 << 20)) return SPSTD_ERR_ARG;
    if (d->nprobes < 0 || d->nprobes > kResMaxProbes) return SPSTD_ERR_ARG;
    if (d->nsteps_max < 0) return SPSTD_ERR_ARG;
    if (d->waves_per_block != 0 && d->waves_per_block != 2 && d->waves_per_block != 4) return SPSTD_ERR_ARG;
    return SPSTD_OK;
}

template <typename R>
static hipError_t batch_axis(Batch* b, int a, const R* src, R* dst, const ScaleRef& sc, int col) {
    return launch_axis_acc<R>(b->d.n[a], src, dst, b->ws + b->L.tw[a],
                              axis_geom_of_n(b->d.ndim, b->d.n, a, b->d.capacity), sc, col, b->d.nyquist, b->st, b->wpb);
}

template <typename R>
static hipError_t batch_probe(Batch* b, int part) {
    if (b->d.nprobes == 0) return hipSuccess;
    return launch_probe_batch<R>(BF<R>(b, b->L.psiR), BF<R>(b, b->L.psiI), b->npts,
                                 reinterpret_cast<const int64_t*>(b->ws + b->L.pidx), b->d.nprobes,
                                 reinterpret_cast<const int*>(b->ws + b->L.active), b->d.capacity,
                                 reinterpret_cast<double*>(b->ws + b->L.probes),
                                 reinterpret_cast<int64_t*>(b->ws + b->L.counter), b->d.nsteps_max + 1,
                                 reinterpret_cast<int*>(b->ws + b->L.fault), b->st, part);
}

// One step and its probe samples.  *owed: on entry, the stage whose B half
// still owes its y pass from the previous step (-1: none); chain: leave the
// last B half's y pass owed to the next step, whose first y sweep then does
// it fused with its own.  A chained boundary writes the psi_R half of its
// sample at once (the owed pass changes psi_I alone) and the psi_I half
// after that sweep (A halves leave psi_I alone).
template <typename R>
static hipError_t batch_step_once(Batch* b, int* owed_io, bool chain) {
    R* pr = BF<R>(b, b->L.psiR);
    R* pi = BF<R>(b, b->L.psiI);
    const R* V = BF<R>(b, b->L.V);
    const int64_t rpi = b->npts / b->d.n[0];
    const RowGeom rg{rpi * b->d.capacity, rpi};
    const int64_t nx = b->d.n[0];
    const void* twx = b->ws + b->L.tw[0];
    hipError_t e = hipSuccess;
    // A half y, z, x; B half x, z, y: the B half's y pass and the next A
    // half's y pass are one sweep (as in the single-plan engine)
    int owed = *owed_io;
    const bool pending = owed >= 0;
    *owed_io = -1;
    bool fs_ready = false;   // four-step scratch holds the transforms of psi_I
    for (int l = 0; l < b->d.m && e == hipSuccess; ++l) {
        const bool a = b->c[l] != 0.0, bb = b->dd[l] != 0.0;
        const ScaleRef sc{b->ws + b->L.scales, b->d.m, l};
        if (b->d.ndim >= 2) {
            if (a && owed >= 0) {
                const ScaleRef so{b->ws + b->L.scales, b->d.m, owed};
                e = launch_axis_ba<R>(b->d.n[1], pr, pi, b->ws + b->L.tw[1],
                                      axis_geom_of_n(b->d.ndim, b->d.n, 1, b->d.capacity), so, sc, SC_KYB, SC_KYA,
                                      b->d.nyquist, b->st, b->wpb);
            } else {
                if (owed >= 0) {
                    const ScaleRef so{b->ws + b->L.scales, b->d.m, owed};
                    e = batch_axis<R>(b, 1, pr, pi, so, SC_KYB);
                }
                if (a && e == hipSuccess) e = batch_axis<R>(b, 1, pi, pr, sc, SC_KYA);
            }
            owed = -1;
            if (l == 0 && pending && e == hipSuccess) e = batch_probe<R>(b, PROBE_I);
            if (b->planes) {
                // z(A), x(A), x(B), z(B) in one launch per x-z plane
                if (e == hipSuccess)
                    e = launch_plane_zxz<R>(b->d.n[0], b->d.n[1], b->d.n[2], b->d.capacity, pr, pi, V, sc, a, bb,
                                            b->d.nyquist, twx, b->ws + b->L.tw[2], b->st);
                if (e == hipSuccess && bb) owed = l;
                continue;
            }
            if (a && e == hipSuccess && b->d.ndim == 3) e = batch_axis<R>(b, 2, pi, pr, sc, SC_KZA);
        }
        if (e != hipSuccess) break;
        if (b->fourstep) {
            // a B half followed by the next stage's A half leaves that half's
            // first transforms (of psi_I) in the scratch
            const bool fuse = bb && l + 1 < b->d.m && b->c[l + 1] != 0.0;
            if (a || bb)
                e = launch_x_fourstep<R>(nx, pr, pi, V, twx, b->ws + b->L.twsub, b->ws + b->L.twsub + 128 * 16,
                                         b->ws + b->L.fs, rg, sc, a, bb, b->d.nyquist, a && fs_ready, fuse, b->st);
            fs_ready = fuse;
            if (e != hipSuccess) break;
            continue;   // 1D: no y or z passes
        }
        if (a && bb) e = launch_x_ab<R>(nx, pr, pi, V, twx, rg, sc, b->d.nyquist, b->st, b->wpb);
        else if (a) e = launch_x_acc<R>(nx, pi, pr, V, twx, rg, sc, SC_KXA, SC_PA, b->d.nyquist, b->st, b->wpb);
        else if (bb) e = launch_x_acc<R>(nx, pr, pi, V, twx, rg, sc, SC_KXB, SC_PB, b->d.nyquist, b->st, b->wpb);
        if (e != hipSuccess) break;
        if (bb && b->d.ndim >= 2) {
            if (b->d.ndim == 3) e = batch_axis<R>(b, 2, pr, pi, sc, SC_KZB);
            owed = l;
        }
    }
    if (e != hipSuccess) return e;
    if (chain && owed >= 0) {
        *owed_io = owed;
        return batch_probe<R>(b, PROBE_R);
    }
    if (owed >= 0) {
        const ScaleRef so{b->ws + b->L.scales, b->d.m, owed};
        e = batch_axis<R>(b, 1, pr, pi, so, SC_KYB);
    }
    return e == hipSuccess ? batch_probe<R>(b, PROBE_FULL) : e;
}

// n steps, chained: every boundary between them but the last is fused.
template <typename R>
static hipError_t batch_steps(Batch* b, int64_t n) {
    int owed = -1;
    hipError_t e = hipSuccess;
    for (int64_t s = 0; s < n && e == hipSuccess; ++s) e = batch_step_once<R>(b, &owed, s + 1 < n);
    return e;
}

template <typename R>
static spstd_status batch_build_graph(Batch* b) {
    hipStream_t cap;
    BCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t user = b->st;
    b->st = cap;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t e2 = batch_steps<R>(b, kBatchGraphChunk);
        e = hipStreamEndCapture(cap, &g);
        if (e == hipSuccess) e = e2;
    }
    b->st = user;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        b->err = std::string("graph capture: ") + hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    b->graph_ready = true;
    return SPSTD_OK;
}

// Rebuild the resident kernel's table of active slots.
template <typename R>
static spstd_status upload_rtab(Batch* b) {
    std::vector<ResidentInst<R>> tab;
    const double k1base = 2.0 * kPi;
    for (int i = 0; i < b->d.capacity; ++i) {
        const Slot& s = b->slots[i];
        if (!s.active) continue;
        ResidentInst<R> I{};
        I.V = BF<R>(b, b->L.V) + (int64_t)i * b->npts;
        I.psiR = BF<R>(b, b->L.psiR) + (int64_t)i * b->npts;
        I.psiI = BF<R>(b, b->L.psiI) + (int64_t)i * b->npts;
        const size_t np = (size_t)(b->d.nprobes > 0 ? b->d.nprobes : 1);
        I.probes = reinterpret_cast<double*>(b->ws + b->L.probes) + (size_t)i * (b->d.nsteps_max + 1) * np * 2;
        I.counter = reinterpret_cast<int64_t*>(b->ws + b->L.counter) + i;
        I.fault = reinterpret_cast<int*>(b->ws + b->L.fault);
        I.capacity = b->d.nsteps_max + 1;
        I.nprobes = b->d.nprobes;
        for (int q = 0; q < b->d.nprobes; ++q) I.probe_idx[q] = s.probe_idx[q];
        // kinetic scale per axis: (hbar/2m*) (2 pi/L)^2 / N for the bare k^2
        double kin[3] = {0.0, 0.0, 0.0};
        for (int ax = 0; ax < b->d.ndim; ++ax) {
            const double k1 = k1base / ((double)b->d.n[ax] * s.dx[ax]);
            kin[ax] = s.hbar / (2.0 * s.mass) * k1 * k1 / (double)b->d.n[ax];
        }
        for (int l = 0; l < b->d.m; ++l) {
            const double a = b->c[l] * s.dt, bb = -b->dd[l] * s.dt;
            I.kin[2 * l] = (R)(a * kin[0]);
            I.kin[2 * l + 1] = (R)(bb * kin[0]);
            I.kin_y[2 * l] = (R)(a * kin[1]);
            I.kin_y[2 * l + 1] = (R)(bb * kin[1]);
            I.kin_z[2 * l] = (R)(a * kin[2]);
            I.kin_z[2 * l + 1] = (R)(bb * kin[2]);
            I.pot[2 * l] = (R)(a / s.hbar);
            I.pot[2 * l + 1] = (R)(bb / s.hbar);
        }
        tab.push_back(I);
    }
    b->nres = (int)tab.size();
    if (!tab.empty()) {
        BCHK(hipMemcpyAsync(b->ws + b->L.rinst, tab.data(), tab.size() * sizeof(ResidentInst<R>),
                            hipMemcpyHostToDevice, b->st));
        BCHK(hipStreamSynchronize(b->st));
    }
    b->rtab_dirty = false;
    return SPSTD_OK;
}

template <typename R>
static spstd_status batch_step_t(Batch* b, int64_t n) {
    if (b->resident) {
        if (b->rtab_dirty) {
            spstd_status s = upload_rtab<R>(b);
            if (s != SPSTD_OK) return s;
        }
        const ResidentInst<R>* tab = reinterpret_cast<const ResidentInst<R>*>(b->ws + b->L.rinst);
        if (b->nres > 0 && n > 0) {
            if (b->d.ndim == 1)
                BCHK(launch_resident_1d<R>(b->d.n[0], tab, b->nres, b->d.m, n, b->d.nyquist, b->ws + b->L.tw[0],
                                           b->st));
            else if (b->d.ndim == 2)
                BCHK(launch_resident_2d<R>(b->d.n[0], b->d.n[1], tab, b->nres, b->d.m, n, b->d.nyquist,
                                           b->ws + b->L.tw[0], b->ws + b->L.tw[1], b->st));
            else
                BCHK(launch_resident_3d<R>(b->d.n[0], b->d.n[1], b->d.n[2], tab, b->nres, b->d.m, n,
                                           b->d.nyquist, b->ws + b->L.tw[0], b->ws + b->L.tw[1],
                                           b->ws + b->L.tw[2], b->st));
        }
        return SPSTD_OK;
    }
    int64_t left = n;
    if (n >= kBatchGraphChunk) {
        if (!b->graph_ready) {
            spstd_status s = batch_build_graph<R>(b);
            if (s != SPSTD_OK) return s;
        }
        for (; left >= kBatchGraphChunk; left -= kBatchGraphChunk) BCHK(hipGraphLaunch(b->graph, b->st));
    }
    if (left > 0) BCHK(batch_steps<R>(b, left));
    return SPSTD_OK;
}

// ---------------------------------------------------------------------------
// Schedule autotuner: the resident kernel (batches that fit it) against
// the pass kernels with 2 and with 4 waves per block, timed on the empty
// batch (every slot stepping a zero state with the scales of a nominal
// instance) and remembered per (shape, precision, capacity).
// ---------------------------------------------------------------------------
struct TuneResult {
    bool resident;
    int wpb;
    double us[3];
};
static std::mutex g_tune_mu;
static std::map<std::tuple<int64_t, int64_t, int64_t, size_t, int>, TuneResult> g_tune;

template <typename R>
static spstd_status time_steps(Batch* b, int64_t warm, int64_t n, double* us) {
    spstd_status s = batch_step_t<R>(b, warm);
    if (s != SPSTD_OK) return s;
    hipEvent_t e0, e1;
    BCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SPSTD_ERR_DEVICE;
    }
    hipError_t e = hipEventRecord(e0, b->st);
    if (e == hipSuccess) s = batch_step_t<R>(b, n);
    if (e == hipSuccess && s == SPSTD_OK) e = hipEventRecord(e1, b->st);
    if (e == hipSuccess && s == SPSTD_OK) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess && s == SPSTD_OK) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        b->err = hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    *us = s == SPSTD_OK ? 1e3 * ms / (double)n : 0.0;
    return s;
}

// Drop the captured pass graph (its launches carry the old block size).
static void drop_graph(Batch* b) {
    if (b->graph_ready) (void)hipGraphExecDestroy(b->graph);
    b->graph_ready = false;
}

// Trial state for timing schedules on an empty batch: every slot active,
// stepping its (zero) state with the scales of a nominal instance (dx =
// hbar = m* = 1, V = 0, dt = 0.5 x_max / rho) and sampling point 0; and
// back to the empty batch (zero scales, counters and active flags; a zero
// state stays zero).
template <typename R>
static spstd_status batch_trial_begin(Batch* b) {
    spstd_desc one{};
    one.ndim = b->d.ndim;
    for (int a = 0; a < 3; ++a) {
        one.n[a] = b->d.n[a];
        one.dx[a] = 1.0;
    }
    one.hbar = one.mass = 1.0;
    const double dt = 0.5 * b->xmax / (0.5 * kPi * kPi * (double)b->d.ndim);
    std::vector<double> rows((size_t)b->d.m * SC_COLS);
    for (int l = 0; l < b->d.m; ++l) scale_row(one, b->c[l] * dt, -b->dd[l] * dt, &rows[(size_t)l * SC_COLS]);
    std::vector<R> rr(rows.size() * (size_t)b->d.capacity);
    for (int i = 0; i < b->d.capacity; ++i)
        for (size_t k = 0; k < rows.size(); ++k) rr[(size_t)i * rows.size() + k] = (R)rows[k];
    std::vector<int> act(b->d.capacity, 1);
    std::vector<int64_t> pz((size_t)b->d.capacity * (b->d.nprobes > 0 ? b->d.nprobes : 1), 0);
    BCHK(hipMemcpyAsync(b->ws + b->L.pidx, pz.data(), pz.size() * sizeof(int64_t), hipMemcpyHostToDevice, b->st));
    BCHK(hipMemcpyAsync(b->ws + b->L.scales, rr.data(), rr.size() * sizeof(R), hipMemcpyHostToDevice, b->st));
    BCHK(hipMemcpyAsync(b->ws + b->L.active, act.data(), act.size() * sizeof(int), hipMemcpyHostToDevice, b->st));
    BCHK(hipStreamSynchronize(b->st));
    for (Slot& sl : b->slots) {
        sl.active = true;
        sl.dt = dt;
        sl.hbar = sl.mass = 1.0;
        for (int a = 0; a < 3; ++a) sl.dx[a] = 1.0;
        for (int q = 0; q < b->d.nprobes; ++q) sl.probe_idx[q] = 0;
    }
    return SPSTD_OK;
}

template <typename R>
static spstd_status batch_trial_end(Batch* b) {
    const size_t nsc = (size_t)b->d.m * SC_COLS * (size_t)b->d.capacity;
    std::vector<R> zr(nsc, (R)0);
    std::vector<int> za(b->d.capacity, 0);
    std::vector<int64_t> zc(b->d.capacity, 0);
    BCHK(hipMemcpyAsync(b->ws + b->L.scales, zr.data(), zr.size() * sizeof(R), hipMemcpyHostToDevice, b->st));
    BCHK(hipMemcpyAsync(b->ws + b->L.active, za.data(), za.size() * sizeof(int), hipMemcpyHostToDevice, b->st));
    BCHK(hipMemcpyAsync(b->ws + b->L.counter, zc.data(), zc.size() * sizeof(int64_t), hipMemcpyHostToDevice, b->st));
    BCHK(hipStreamSynchronize(b->st));
    for (Slot& sl : b->slots) sl = Slot{};
    b->rtab_dirty = true;
    return SPSTD_OK;
}

template <typename R>
static spstd_status batch_autotune(Batch* b) {
    const auto key = std::make_tuple(b->d.n[0], b->d.n[1], b->d.n[2], b->esz, b->d.capacity);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            b->resident = it->second.resident;
            b->wpb = it->second.wpb;
            for (int k = 0; k < 3; ++k) b->tuned_us[k] = it->second.us[k];
            return SPSTD_OK;
        }
    }
    {
        spstd_status s0 = batch_trial_begin<R>(b);
        if (s0 != SPSTD_OK) return s0;
    }
    const int64_t trial = 2 * kBatchGraphChunk;
    double us[3] = {0.0, 0.0, 0.0};
    spstd_status s = SPSTD_OK;
    const bool can_resident = b->resident;
    if (can_resident) {
        b->rtab_dirty = true;
        s = time_steps<R>(b, kBatchGraphChunk, trial, &us[0]);
    }
    b->resident = false;
    // block size matters only where pencils of a wave share a block: every
    // y/z length does, x rows do up to 1024 points
    const bool both = b->d.ndim >= 2 || b->d.n[0] <= 1024;
    for (int k = 0; k < 2 && s == SPSTD_OK; ++k) {
        if (k == 1 && !both) {
            us[2] = us[1];
            break;
        }
        drop_graph(b);
        b->wpb = k == 0 ? 2 : 4;
        s = time_steps<R>(b, kBatchGraphChunk, trial, &us[1 + k]);
    }
    drop_graph(b);
    {
        spstd_status s1 = batch_trial_end<R>(b);
        if (s == SPSTD_OK) s = s1;
    }
    if (s != SPSTD_OK) return s;
    b->wpb = (both && us[2] < us[1]) ? 4 : 2;
    const double pass_us = us[b->wpb == 4 ? 2 : 1];
    b->resident = can_resident && us[0] <= pass_us;
    for (int k = 0; k < 3; ++k) b->tuned_us[k] = us[k];
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[key] = TuneResult{b->resident, b->wpb, {us[0], us[1], us[2]}};
    return SPSTD_OK;
}

template <typename R>
static spstd_status batch_upload_slot(Batch* b, int slot, const double* V, const double* pr, const double* pi,
                                      const double* row_tab) {
    const int64_t n = b->npts;
    const size_t off = (size_t)slot * n * sizeof(R);
    std::vector<R> tmp(n);
    const double* src[3] = {pr, pi, V};
    const size_t dst[3] = {b->L.psiR, b->L.psiI, b->L.V};
    for (int k = 0; k < 3; ++k) {
        for (int64_t i = 0; i < n; ++i) tmp[i] = src[k] ? (R)src[k][i] : (R)0;
        BCHK(hipMemcpyAsync(b->ws + dst[k] + off, tmp.data(), n * sizeof(R), hipMemcpyHostToDevice, b->st));
        BCHK(hipStreamSynchronize(b->st));
    }
    std::vector<R> rows((size_t)b->d.m * SC_COLS);
    for (size_t i = 0; i < rows.size(); ++i) rows[i] = row_tab ? (R)row_tab[i] : (R)0;
    BCHK(hipMemcpyAsync(b->ws + b->L.scales + (size_t)slot * rows.size() * sizeof(R), rows.data(),
                        rows.size() * sizeof(R), hipMemcpyHostToDevice, b->st));
    BCHK(hipStreamSynchronize(b->st));
    return SPSTD_OK;
}

}  // namespace spstd

using namespace spstd;

struct spstd_batch_s : Batch {};

extern "C" {

spstd_status spstd_batch_workspace_size(const spstd_batch_desc* d, size_t* bytes) {
    spstd_status s = validate_batch(d);
    if (s != SPSTD_OK) return s;
    if (!bytes) return SPSTD_ERR_ARG;
    *bytes = batch_layout(d).total;
    return SPSTD_OK;
}

spstd_status spstd_batch_create(const spstd_batch_desc* d, void* d_workspace, size_t ws_bytes, void* stream,
                                spstd_batch_t* out) {
    if (!out) return SPSTD_ERR_ARG;
    *out = nullptr;
    spstd_status s = validate_batch(d);
    if (s != SPSTD_OK) return s;
    BatchLayout L = batch_layout(d);
    if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace & 255)) return SPSTD_ERR_WORKSPACE;
    double x;
    if (!xmax_symplectic(d->m, d->c, d->d, &x)) return SPSTD_ERR_ARG;
    spstd_batch_s* b = new (std::nothrow) spstd_batch_s();
    if (!b) return SPSTD_ERR_DEVICE;
    b->d = *d;
    for (int l = 0; l < d->m; ++l) {
        b->c[l] = d->c[l];
        b->dd[l] = d->d[l];
    }
    b->d.c = b->c;
    b->d.d = b->dd;
    b->xmax = x;
    b->npts = d->n[0] * d->n[1] * d->n[2];
    b->esz = d->precision == SPSTD_FP64 ? 8 : 4;
    b->ws = (char*)d_workspace;
    b->L = L;
    b->st = (hipStream_t)stream;
    b->slots.resize(d->capacity);
    b->resident = ((d->ndim == 1 && resident_len_ok(d->n[0])) || (d->ndim == 2 && resident2d_ok(d->n[0], d->n[1])) ||
                   (d->ndim == 3 && resident3d_ok(d->n[0], d->n[1], d->n[2]))) &&
                  !(d->flags & SPSTD_NO_RESIDENT);
    b->wpb = d->waves_per_block;
    b->planes = d->ndim == 3 && plane_ok(d->n[0], d->n[2]) && !(d->flags & SPSTD_NO_PLANES);
    b->fourstep = d->ndim == 1 && fourstep_ok(d->n[0]) && !(d->flags & SPSTD_NO_FOURSTEP);
    // zero fields and scales, twiddles, probe slots inactive
    hipError_t e = hipSuccess;
    const size_t fb = (size_t)d->capacity * b->npts;
    if (b->esz == 8) {
        for (size_t off : {L.psiR, L.psiI, L.V})
            if (e == hipSuccess) e = launch_fill0<double>((int64_t)fb, BF<double>(b, off), b->st);
        if (e == hipSuccess)
            e = launch_fill0<double>((int64_t)d->capacity * d->m * SC_COLS, BF<double>(b, L.scales), b->st);
    } else {
        for (size_t off : {L.psiR, L.psiI, L.V})
            if (e == hipSuccess) e = launch_fill0<float>((int64_t)fb, BF<float>(b, off), b->st);
        if (e == hipSuccess)
            e = launch_fill0<float>((int64_t)d->capacity * d->m * SC_COLS, BF<float>(b, L.scales), b->st);
    }
    std::vector<int> act(d->capacity, 0);
    std::vector<int64_t> cnt(d->capacity, 0);
    // probe indices start at point 0 (in range) for every slot: the probe
    // kernel reads the indices of every slot it marks as sampled
    std::vector<int64_t> pz((size_t)d->capacity * (d->nprobes > 0 ? d->nprobes : 1), 0);
    if (e == hipSuccess) e = hipMemcpyAsync(b->ws + L.pidx, pz.data(), pz.size() * sizeof(int64_t),
                                            hipMemcpyHostToDevice, b->st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->ws + L.active, act.data(), act.size() * sizeof(int),
                                            hipMemcpyHostToDevice, b->st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->ws + L.counter, cnt.data(), cnt.size() * sizeof(int64_t),
                                            hipMemcpyHostToDevice, b->st);
    if (e == hipSuccess) e = launch_fill0<int>(1, reinterpret_cast<int*>(b->ws + L.fault), b->st);
    for (int a = 0; a < d->ndim && e == hipSuccess; ++a) {
        // FP64 in every precision: the kernels round each twiddle once
        std::vector<double> t = twiddles(d->n[a]);
        e = hipMemcpyAsync(b->ws + L.tw[a], t.data(), t.size() * 8, hipMemcpyHostToDevice, b->st);
        if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    }
    if (d->ndim == 1 && fourstep_ok(d->n[0]) && e == hipSuccess) {
        // the four-step passes' 128-point and n/128-point tables, in turn
        std::vector<double> t = twiddles(128), t2 = twiddles(d->n[0] / 128);
        t.insert(t.end(), t2.begin(), t2.end());
        e = hipMemcpyAsync(b->ws + L.twsub, t.data(), t.size() * 8, hipMemcpyHostToDevice, b->st);
        if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) {
        delete b;
        return SPSTD_ERR_DEVICE;
    }
    if (d->flags & SPSTD_AUTOTUNE) {
        s = (b->esz == 8) ? batch_autotune<double>(b) : batch_autotune<float>(b);
        if (s != SPSTD_OK) {
            drop_graph(b);
            delete b;
            return s;
        }
    }
    *out = b;
    return SPSTD_OK;
}

spstd_status spstd_batch_schedule(spstd_batch_t b, int* resident, int* waves_per_block, double* tuned_us) {
    if (!b || !resident) return SPSTD_ERR_ARG;
    *resident = b->resident ? 1 : 0;
    if (waves_per_block) *waves_per_block = b->wpb;
    if (tuned_us)
        for (int k = 0; k < 3; ++k) tuned_us[k] = b->tuned_us[k];
    return SPSTD_OK;
}

spstd_status spstd_batch_load(spstd_batch_t b, int slot, const double* dx, double hbar, double mass, double dt,
                              double cfl_fraction, const double* V, const double* psiR0, const double* psiI0,
                              const int64_t* probe_idx, double* dt_out) {
    if (!b || slot < 0 || slot >= b->d.capacity || !dx || !V || !psiR0) return SPSTD_ERR_ARG;
    if (b->slots[slot].active) return SPSTD_ERR_ARG;
    if (!(hbar > 0.0) || !(mass > 0.0) || !std::isfinite(hbar) || !std::isfinite(mass)) return SPSTD_ERR_ARG;
    for (int a = 0; a < b->d.ndim; ++a)
        if (!(dx[a] > 0.0) || !std::isfinite(dx[a])) return SPSTD_ERR_ARG;
    if (b->d.nprobes > 0 && !probe_idx) return SPSTD_ERR_ARG;
    for (int q = 0; q < b->d.nprobes; ++q)
        if (probe_idx[q] < 0 || probe_idx[q] >= b->npts) return SPSTD_ERR_ARG;
    for (int64_t i = 0; i < b->npts; ++i)
        if (!std::isfinite(V[i]) || !std::isfinite(psiR0[i]) || (psiI0 && !std::isfinite(psiI0[i])))
            return SPSTD_ERR_ARG;
    if (!(dt >= 0.0) || !std::isfinite(dt)) return SPSTD_ERR_ARG;
    const double rho = rho_bound_of(b->d.ndim, dx, hbar, mass, V, b->npts);
    if (dt == 0.0) {
        if (!(cfl_fraction > 0.0)) return SPSTD_ERR_ARG;
        dt = cfl_fraction * b->xmax / rho;
    }
    if (!(b->d.flags & SPSTD_ALLOW_UNSTABLE) && dt * rho >= b->xmax) return SPSTD_ERR_UNSTABLE;
    Slot& s = b->slots[slot];
    s.dt = dt;
    s.hbar = hbar;
    s.mass = mass;
    for (int a = 0; a < 3; ++a) s.dx[a] = a < b->d.ndim ? dx[a] : 1.0;
    for (int q = 0; q < b->d.nprobes; ++q) s.probe_idx[q] = probe_idx[q];
    s.steps = 0;
    // the slot's scale rows, from an instance descriptor with its spacing
    spstd_desc one{};
    one.ndim = b->d.ndim;
    for (int a = 0; a < 3; ++a) {
        one.n[a] = b->d.n[a];
        one.dx[a] = s.dx[a];
    }
    one.hbar = hbar;
    one.mass = mass;
    std::vector<double> rows((size_t)b->d.m * SC_COLS);
    for (int l = 0; l < b->d.m; ++l) scale_row(one, b->c[l] * dt, -b->dd[l] * dt, &rows[(size_t)l * SC_COLS]);
    spstd_status st = (b->esz == 8) ? batch_upload_slot<double>(b, slot, V, psiR0, psiI0, rows.data())
                                    : batch_upload_slot<float>(b, slot, V, psiR0, psiI0, rows.data());
    if (st != SPSTD_OK) return st;
    // probe indices, counter 0, sample 0, active flag
    hipError_t e = hipSuccess;
    if (b->d.nprobes > 0)
        e = hipMemcpyAsync(b->ws + b->L.pidx + (size_t)slot * b->d.nprobes * sizeof(int64_t), probe_idx,
                           b->d.nprobes * sizeof(int64_t), hipMemcpyHostToDevice, b->st);
    int64_t zero = 0;
    int one_i = 1;
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + b->L.counter + (size_t)slot * sizeof(int64_t), &zero, sizeof(zero),
                           hipMemcpyHostToDevice, b->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + b->L.active + (size_t)slot * sizeof(int), &one_i, sizeof(int),
                           hipMemcpyHostToDevice, b->st);
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    if (e == hipSuccess && b->d.nprobes > 0) {
        // record sample 0 for this slot alone: probe kernel on a one-slot view
        const size_t np = (size_t)b->d.nprobes;
        const size_t poff = (size_t)slot * (b->d.nsteps_max + 1) * np * 2 * sizeof(double);
        if (b->esz == 8)
            e = launch_probe_batch<double>(BF<double>(b, b->L.psiR) + (int64_t)slot * b->npts,
                                           BF<double>(b, b->L.psiI) + (int64_t)slot * b->npts, b->npts,
                                           reinterpret_cast<const int64_t*>(b->ws + b->L.pidx) + slot * np, b->d.nprobes,
                                           reinterpret_cast<const int*>(b->ws + b->L.active) + slot, 1,
                                           reinterpret_cast<double*>(b->ws + b->L.probes + poff),
                                           reinterpret_cast<int64_t*>(b->ws + b->L.counter) + slot,
                                           b->d.nsteps_max + 1, reinterpret_cast<int*>(b->ws + b->L.fault), b->st);
        else
            e = launch_probe_batch<float>(BF<float>(b, b->L.psiR) + (int64_t)slot * b->npts,
                                          BF<float>(b, b->L.psiI) + (int64_t)slot * b->npts, b->npts,
                                          reinterpret_cast<const int64_t*>(b->ws + b->L.pidx) + slot * np, b->d.nprobes,
                                          reinterpret_cast<const int*>(b->ws + b->L.active) + slot, 1,
                                          reinterpret_cast<double*>(b->ws + b->L.probes + poff),
                                          reinterpret_cast<int64_t*>(b->ws + b->L.counter) + slot,
                                          b->d.nsteps_max + 1, reinterpret_cast<int*>(b->ws + b->L.fault), b->st);
    } else if (e == hipSuccess) {
        int64_t one64 = 1;
        e = hipMemcpyAsync(b->ws + b->L.counter + (size_t)slot * sizeof(int64_t), &one64, sizeof(one64),
                           hipMemcpyHostToDevice, b->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) {
        b->err = hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    s.active = true;
    b->rtab_dirty = true;
    if (dt_out) *dt_out = dt;
    return SPSTD_OK;
}

spstd_status spstd_batch_step(spstd_batch_t b, int64_t nsteps) {
    if (!b || nsteps < 0) return SPSTD_ERR_ARG;
    for (const Slot& s : b->slots)
        if (s.active && s.steps + nsteps > b->d.nsteps_max) {
            b->err = "probe buffer capacity exceeded";
            return SPSTD_ERR_CAPACITY;
        }
    spstd_status st = (b->esz == 8) ? batch_step_t<double>(b, nsteps) : batch_step_t<float>(b, nsteps);
    if (st != SPSTD_OK) return st;
    for (Slot& s : b->slots)
        if (s.active) s.steps += nsteps;
    return SPSTD_OK;
}

spstd_status spstd_batch_read(spstd_batch_t b, int slot, double* probes_out, double* psiR, double* psiI,
                              int64_t* steps_done) {
    if (!b || slot < 0 || slot >= b->d.capacity) return SPSTD_ERR_ARG;
    const Slot& s = b->slots[slot];
    hipError_t e = hipStreamSynchronize(b->st);
    const size_t np = (size_t)b->d.nprobes;
    int fault = 0;
    // copies on the batch's own stream: a caller stepping other batches on
    // other streams is not made to wait for them
    if (e == hipSuccess && np > 0)
        e = hipMemcpyAsync(&fault, b->ws + b->L.fault, sizeof(int), hipMemcpyDeviceToHost, b->st);
    if (e == hipSuccess && np > 0) e = hipStreamSynchronize(b->st);
    if (e == hipSuccess && fault) {
        b->err = "a probe index in device memory lies outside the grid (samples skipped)";
        return SPSTD_ERR_DEVICE;
    }
    if (e == hipSuccess && probes_out && np > 0) {
        const size_t poff = (size_t)slot * (b->d.nsteps_max + 1) * np * 2 * sizeof(double);
        e = hipMemcpyAsync(probes_out, b->ws + b->L.probes + poff, (size_t)(s.steps + 1) * np * 2 * sizeof(double),
                           hipMemcpyDeviceToHost, b->st);
        if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    }
    double* outs[2] = {psiR, psiI};
    const size_t offs[2] = {b->L.psiR, b->L.psiI};
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        if (!outs[k]) continue;
        if (b->esz == 8) {
            e = hipMemcpyAsync(outs[k], b->ws + offs[k] + (size_t)slot * b->npts * 8, b->npts * 8,
                               hipMemcpyDeviceToHost, b->st);
            if (e == hipSuccess) e = hipStreamSynchronize(b->st);
        } else {
            std::vector<float> tmp(b->npts);
            e = hipMemcpyAsync(tmp.data(), b->ws + offs[k] + (size_t)slot * b->npts * 4, b->npts * 4,
                               hipMemcpyDeviceToHost, b->st);
            if (e == hipSuccess) e = hipStreamSynchronize(b->st);
            for (int64_t i = 0; i < b->npts && e == hipSuccess; ++i) outs[k][i] = tmp[i];
        }
    }
    if (e != hipSuccess) {
        b->err = hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    if (steps_done) *steps_done = s.steps;
    bool finite = true;
    for (int k = 0; k < 2; ++k)
        if (outs[k])
            for (int64_t i = 0; i < b->npts; ++i) finite = finite && std::isfinite(outs[k][i]);
    return finite ? SPSTD_OK : SPSTD_ERR_NONFINITE;
}

spstd_status spstd_batch_release(spstd_batch_t b, int slot) {
    if (!b || slot < 0 || slot >= b->d.capacity) return SPSTD_ERR_ARG;
    Slot& s = b->slots[slot];
    if (!s.active) return SPSTD_OK;
    spstd_status st = (b->esz == 8) ? batch_upload_slot<double>(b, slot, nullptr, nullptr, nullptr, nullptr)
                                    : batch_upload_slot<float>(b, slot, nullptr, nullptr, nullptr, nullptr);
    if (st != SPSTD_OK) return st;
    int zero = 0;
    hipError_t e = hipMemcpyAsync(b->ws + b->L.active + (size_t)slot * sizeof(int), &zero, sizeof(int),
                                  hipMemcpyHostToDevice, b->st);
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) {
        b->err = hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    s.active = false;
    s.steps = 0;
    b->rtab_dirty = true;
    return SPSTD_OK;
}

spstd_status spstd_batch_slot_info(spstd_batch_t b, int slot, int* active, int64_t* steps_done, double* dt) {
    if (!b || slot < 0 || slot >= b->d.capacity) return SPSTD_ERR_ARG;
    const Slot& s = b->slots[slot];
    if (active) *active = s.active ? 1 : 0;
    if (steps_done) *steps_done = s.steps;
    if (dt) *dt = s.dt;
    return SPSTD_OK;
}

spstd_status spstd_batch_destroy(spstd_batch_t b) {
    if (!b) return SPSTD_ERR_ARG;
    if (b->graph_ready) (void)hipGraphExecDestroy(b->graph);
    delete b;
    return SPSTD_OK;
}

const char* spstd_batch_last_error(spstd_batch_t b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Groups: 2D batches of different shapes stepped together, one launch per
// pass of the stage sequence for all of them (the mixed-shape kernels), or
// their own pass kernels one member after another on one stream.
// ---------------------------------------------------------------------------
namespace spstd {

static const int kMixMaxVariants = 16;

// Candidate k of the mixed kernels: waves per block 2 or 4 (bit 0), joint
// LDS exchange of the fused x pass for rows under 512 points (bit 1), one
// persistent block per compute unit instead of a grid that fills the device
// (bit 2), two complex pencils per lane group in the y passes (bit 3; FP32
// only).
static MixVariant mix_variant(int k) { return MixVariant{(k & 1) ? 4 : 2, (k >> 1) & 1, 1 + ((k >> 3) & 1)}; }
static bool mix_one_per_cu(int k) { return (k >> 2) & 1; }

struct Group {
    std::vector<Batch*> members;
    std::vector<hipStream_t> member_streams;   // the members' own streams, restored on destroy
    size_t esz = 8;
    int m = 0;
    bool mixable = false;   // every stage has both halves: the mixed kernels apply
    int nvar = 0;           // mixed-kernel candidates
    int choice = 0;         // candidate in use: < nvar a mixed variant, nvar the members' own kernels
    double tuned_us[kMixMaxVariants + 1] = {0.0};
    int cus = 256;          // compute units of the device
    char* ws = nullptr;
    hipStream_t st = nullptr;
    size_t mem_off = 0, tile_off = 0, slot_off = 0, total = 0;
    int64_t x_off[kMixMaxVariants] = {0}, x_n[kMixMaxVariants] = {0};
    int64_t y_off[kMixMaxVariants] = {0}, y_n[kMixMaxVariants] = {0};
    int nslots = 0;
    hipGraphExec_t graph;
    bool graph_ready = false;
    std::string err;
};

#define GCHK(x)                                                      \
    do {                                                             \
        hipError_t e_ = (x);                                         \
        if (e_ != hipSuccess) {                                      \
            g->err = std::string(#x) + ": " + hipGetErrorString(e_); \
            return SPSTD_ERR_DEVICE;                                 \
        }                                                            \
    } while (0)

// Members must be 2D pass-kernel batches of row and column lengths 128,
// 256 or 512 that share precision, coefficient set, Nyquist convention and
// probe count.
static spstd_status group_check(const spstd_batch_t* mem, int n, std::string* why) {
    if (!mem || n < 1 || n > 64) { *why = "1..64 members"; return SPSTD_ERR_ARG; }
    const Batch* b0 = mem[0];
    for (int i = 0; i < n; ++i) {
        const Batch* b = mem[i];
        if (!b) { *why = "null member"; return SPSTD_ERR_ARG; }
        if (b->d.ndim != 2 || !mix_len_ok(b->d.n[0]) || !mix_len_ok(b->d.n[1]) || b->resident) {
            *why = "members are 2D batches of 128, 256 or 512 points per axis";
            return SPSTD_ERR_ARG;
        }
        if (b->esz != b0->esz || b->d.m != b0->d.m || b->d.nyquist != b0->d.nyquist ||
            b->d.nprobes != b0->d.nprobes) {
            *why = "members differ in precision, stage count, Nyquist convention or probes";
            return SPSTD_ERR_ARG;
        }
        for (int l = 0; l < b->d.m; ++l)
            if (b->c[l] != b0->c[l] || b->dd[l] != b0->dd[l]) { *why = "members differ in coefficients"; return SPSTD_ERR_ARG; }
        for (int j = 0; j < i; ++j)
            if (mem[j] == b) { *why = "a member appears twice"; return SPSTD_ERR_ARG; }
    }
    return SPSTD_OK;
}

// Workspace pieces: the member table, the tile tables of every candidate
// (x tiles, then y tiles), the (member, slot) table of the probe kernel.
static void group_layout(Group* g) {
    const int nm = (int)g->members.size();
    size_t off = 0;
    g->mem_off = off;
    off += align256((size_t)nm * sizeof(MixMember<double>));
    g->tile_off = off;
    int64_t t = 0;
    for (int k = 0; k < g->nvar; ++k) {
        const MixVariant v = mix_variant(k);
        g->x_off[k] = t;
        g->x_n[k] = 0;
        for (Batch* b : g->members) g->x_n[k] += mix_blocks(0, (int)b->d.n[0], (int)b->d.n[1], b->d.capacity, (int)g->esz, v);
        t += g->x_n[k];
        g->y_off[k] = t;
        g->y_n[k] = 0;
        for (Batch* b : g->members) g->y_n[k] += mix_blocks(1, (int)b->d.n[0], (int)b->d.n[1], b->d.capacity, (int)g->esz, v);
        t += g->y_n[k];
    }
    off += align256((size_t)t * sizeof(MixTile));
    g->slot_off = off;
    g->nslots = 0;
    for (Batch* b : g->members) g->nslots += b->d.capacity;
    off += align256((size_t)(g->nslots > 0 ? g->nslots : 1) * sizeof(MixTile));
    g->total = off;
}

template <typename R>
static spstd_status group_upload(Group* g) {
    std::vector<MixMember<R>> mt;
    for (Batch* b : g->members) {
        MixMember<R> M{};
        M.nx = (int)b->d.n[0];
        M.ny = (int)b->d.n[1];
        M.psiR = BF<R>(b, b->L.psiR);
        M.psiI = BF<R>(b, b->L.psiI);
        M.V = BF<R>(b, b->L.V);
        M.twx = b->ws + b->L.tw[0];
        M.twy = b->ws + b->L.tw[1];
        M.scales = b->ws + b->L.scales;
        M.rg = RowGeom{b->d.n[1] * b->d.capacity, b->d.n[1]};
        M.gy = axis_geom_of_n(2, b->d.n, 1, b->d.capacity);
        M.npts = b->npts;
        M.pidx = reinterpret_cast<const int64_t*>(b->ws + b->L.pidx);
        M.active = reinterpret_cast<const int*>(b->ws + b->L.active);
        M.probes = reinterpret_cast<double*>(b->ws + b->L.probes);
        M.counter = reinterpret_cast<int64_t*>(b->ws + b->L.counter);
        M.samples = b->d.nsteps_max + 1;
        M.fault = reinterpret_cast<int*>(b->ws + b->L.fault);
        mt.push_back(M);
    }
    GCHK(hipMemcpyAsync(g->ws + g->mem_off, mt.data(), mt.size() * sizeof(MixMember<R>), hipMemcpyHostToDevice, g->st));
    std::vector<MixTile> tiles;
    for (int k = 0; k < g->nvar; ++k) {
        const MixVariant v = mix_variant(k);
        for (int kind = 0; kind < 2; ++kind)
            for (int i = 0; i < (int)g->members.size(); ++i) {
                const Batch* b = g->members[i];
                const int64_t nb = mix_blocks(kind, (int)b->d.n[0], (int)b->d.n[1], b->d.capacity, (int)g->esz, v);
                for (int64_t q = 0; q < nb; ++q) tiles.push_back(MixTile{i, (int)q});
            }
    }
    if (!tiles.empty())
        GCHK(hipMemcpyAsync(g->ws + g->tile_off, tiles.data(), tiles.size() * sizeof(MixTile), hipMemcpyHostToDevice,
                            g->st));
    std::vector<MixTile> slots;
    for (int i = 0; i < (int)g->members.size(); ++i)
        for (int s = 0; s < g->members[i]->d.capacity; ++s) slots.push_back(MixTile{i, s});
    if (!slots.empty())
        GCHK(hipMemcpyAsync(g->ws + g->slot_off, slots.data(), slots.size() * sizeof(MixTile), hipMemcpyHostToDevice,
                            g->st));
    GCHK(hipStreamSynchronize(g->st));
    return SPSTD_OK;
}

// Blocks of a launch: one per compute unit (a persistent launch striding
// over the tiles; the rest of the device stays free for other streams'
// kernels), or one per tile (the tile-per-block kernels).
static int group_grid(int64_t ntiles, bool one_per_cu, int cus) {
    return (int)(one_per_cu && ntiles > cus ? cus : ntiles);
}

// One step of every member: the stage sequence of batch_step_once (the y
// sweep owed by a B half fused with the next A half's, *owed and chain as
// there), each pass one launch over all members; then the probe samples.
template <typename R>
static hipError_t group_step_once(Group* g, int* owed_io, bool chain) {
    if (g->choice >= g->nvar) {
        // the members share one coefficient set: their owed stages agree
        int next = -1;
        for (Batch* b : g->members) {
            int o = *owed_io;
            const hipError_t e = batch_step_once<R>(b, &o, chain);
            if (e != hipSuccess) return e;
            next = o;
        }
        *owed_io = next;
        return hipSuccess;
    }
    const int k = g->choice;
    const MixVariant v = mix_variant(k);
    const MixMember<R>* mem = reinterpret_cast<const MixMember<R>*>(g->ws + g->mem_off);
    const MixTile* tiles = reinterpret_cast<const MixTile*>(g->ws + g->tile_off);
    const MixTile* tx = tiles + g->x_off[k];
    const MixTile* ty = tiles + g->y_off[k];
    const int nx = (int)g->x_n[k], ny = (int)g->y_n[k];
    const int gx = group_grid(nx, mix_one_per_cu(k), g->cus), gy = group_grid(ny, mix_one_per_cu(k), g->cus);
    const int nyq = g->members[0]->d.nyquist;
    const int nprobes = g->members[0]->d.nprobes;
    const MixTile* slots = reinterpret_cast<const MixTile*>(g->ws + g->slot_off);
    hipError_t e = hipSuccess;
    int owed = *owed_io;
    const bool pending = owed >= 0;
    *owed_io = -1;
    for (int l = 0; l < g->m && e == hipSuccess; ++l) {
        if (owed >= 0) e = launch_mix_axis_ba<R>(mem, ty, ny, gy, g->m, owed, l, nyq, v, g->st);
        else e = launch_mix_axis_acc<R>(mem, ty, ny, gy, g->m, l, 0, nyq, v, g->st);
        if (l == 0 && pending && e == hipSuccess) e = launch_mix_probe<R>(mem, slots, g->nslots, nprobes, g->st, PROBE_I);
        if (e == hipSuccess) e = launch_mix_x_ab<R>(mem, tx, nx, gx, g->m, l, nyq, v, g->st);
        owed = l;
    }
    if (e != hipSuccess) return e;
    if (chain) {
        *owed_io = owed;
        return launch_mix_probe<R>(mem, slots, g->nslots, nprobes, g->st, PROBE_R);
    }
    e = launch_mix_axis_acc<R>(mem, ty, ny, gy, g->m, owed, 1, nyq, v, g->st);
    return e == hipSuccess ? launch_mix_probe<R>(mem, slots, g->nslots, nprobes, g->st, PROBE_FULL) : e;
}

template <typename R>
static hipError_t group_steps(Group* g, int64_t n) {
    int owed = -1;
    hipError_t e = hipSuccess;
    for (int64_t s = 0; s < n && e == hipSuccess; ++s) e = group_step_once<R>(g, &owed, s + 1 < n);
    return e;
}

static void group_drop_graph(Group* g) {
    if (g->graph_ready) (void)hipGraphExecDestroy(g->graph);
    g->graph_ready = false;
}

template <typename R>
static spstd_status group_build_graph(Group* g) {
    hipStream_t cap;
    GCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t user = g->st;
    g->st = cap;
    for (Batch* b : g->members) b->st = cap;
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t e2 = group_steps<R>(g, kBatchGraphChunk);
        e = hipStreamEndCapture(cap, &gr);
        if (e == hipSuccess) e = e2;
    }
    g->st = user;
    for (Batch* b : g->members) b->st = user;
    if (e == hipSuccess) e = hipGraphInstantiate(&g->graph, gr, nullptr, nullptr, 0);
    if (gr) (void)hipGraphDestroy(gr);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        g->err = std::string("graph capture: ") + hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    g->graph_ready = true;
    return SPSTD_OK;
}

template <typename R>
static spstd_status group_step_t(Group* g, int64_t n) {
    int64_t left = n;
    if (n >= kBatchGraphChunk) {
        if (!g->graph_ready) {
            spstd_status s = group_build_graph<R>(g);
            if (s != SPSTD_OK) return s;
        }
        for (; left >= kBatchGraphChunk; left -= kBatchGraphChunk) GCHK(hipGraphLaunch(g->graph, g->st));
    }
    if (left > 0) GCHK(group_steps<R>(g, left));
    return SPSTD_OK;
}

template <typename R>
static spstd_status group_time(Group* g, double* us) {
    spstd_status s = group_step_t<R>(g, kBatchGraphChunk);
    if (s != SPSTD_OK) return s;
    hipEvent_t e0, e1;
    GCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SPSTD_ERR_DEVICE;
    }
    const int64_t trial = 2 * kBatchGraphChunk;
    hipError_t e = hipEventRecord(e0, g->st);
    if (e == hipSuccess) s = group_step_t<R>(g, trial);
    if (e == hipSuccess && s == SPSTD_OK) e = hipEventRecord(e1, g->st);
    if (e == hipSuccess && s == SPSTD_OK) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess && s == SPSTD_OK) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        g->err = hipGetErrorString(e);
        return SPSTD_ERR_DEVICE;
    }
    *us = s == SPSTD_OK ? 1e3 * ms / (double)trial : 0.0;
    return s;
}

// Time every candidate on the empty members (each slot stepping a zero
// state at a nominal instance's scales) and keep the fastest.
template <typename R>
static spstd_status group_autotune(Group* g) {
    spstd_status s = SPSTD_OK;
    for (Batch* b : g->members) {
        if (s == SPSTD_OK) s = batch_trial_begin<R>(b);
        b->rtab_dirty = true;
    }
    const int first = g->mixable ? 0 : g->nvar;
    for (int k = first; k <= g->nvar && s == SPSTD_OK; ++k) {
        group_drop_graph(g);
        for (Batch* b : g->members) drop_graph(b);
        g->choice = k;
        s = group_time<R>(g, &g->tuned_us[k]);
    }
    group_drop_graph(g);
    for (Batch* b : g->members) {
        drop_graph(b);
        const spstd_status s1 = batch_trial_end<R>(b);
        if (s == SPSTD_OK) s = s1;
    }
    if (s != SPSTD_OK) return s;
    // the fastest; within 3% of it, one block per compute unit (it leaves
    // the rest of the device to other streams' kernels)
    int best = g->nvar;
    for (int k = first; k < g->nvar; ++k)
        if (g->tuned_us[k] < g->tuned_us[best]) best = k;
    for (int k = first; k < g->nvar; ++k)
        if (mix_one_per_cu(k) && !mix_one_per_cu(best) && g->tuned_us[k] <= 1.03 * g->tuned_us[best]) best = k;
    g->choice = best;
    return SPSTD_OK;
}

}  // namespace spstd

struct spstd_batch_group_s : Group {};

extern "C" {

spstd_status spstd_batch_group_workspace_size(const spstd_batch_t* members, int nmembers, size_t* bytes) {
    std::string why;
    spstd_status s = group_check(members, nmembers, &why);
    if (s != SPSTD_OK) return s;
    if (!bytes) return SPSTD_ERR_ARG;
    Group g;
    g.esz = members[0]->esz;
    g.nvar = g.esz == 4 ? 16 : 8;
    for (int i = 0; i < nmembers; ++i) g.members.push_back(members[i]);
    group_layout(&g);
    *bytes = g.total;
    return SPSTD_OK;
}

spstd_status spstd_batch_group_create(const spstd_batch_t* members, int nmembers, uint32_t flags, void* d_workspace,
                                      size_t ws_bytes, void* stream, spstd_batch_group_t* out) {
    if (!out) return SPSTD_ERR_ARG;
    *out = nullptr;
    std::string why;
    spstd_status s = group_check(members, nmembers, &why);
    if (s != SPSTD_OK) return s;
    if ((flags & SPSTD_AUTOTUNE))
        for (int i = 0; i < nmembers; ++i)
            for (const Slot& sl : members[i]->slots)
                if (sl.active) return SPSTD_ERR_ARG;   // tuning steps every slot: members must be empty
    spstd_batch_group_s* g = new (std::nothrow) spstd_batch_group_s();
    if (!g) return SPSTD_ERR_DEVICE;
    g->esz = members[0]->esz;
    g->m = members[0]->d.m;
    g->nvar = g->esz == 4 ? 16 : 8;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            g->cus = cus;
    }
    g->mixable = true;
    for (int l = 0; l < g->m; ++l)
        if (members[0]->c[l] == 0.0 || members[0]->dd[l] == 0.0) g->mixable = false;
    for (int i = 0; i < nmembers; ++i) g->members.push_back(members[i]);
    group_layout(g);
    if (!d_workspace || ws_bytes < g->total || ((uintptr_t)d_workspace & 255)) {
        delete g;
        return SPSTD_ERR_WORKSPACE;
    }
    g->ws = (char*)d_workspace;
    g->st = (hipStream_t)stream;
    // the members' work runs on the group's stream from now on, so that
    // their slot loads, reads and releases order with the group's steps
    for (Batch* b : g->members) {
        if (hipStreamSynchronize(b->st) != hipSuccess) {
            delete g;
            return SPSTD_ERR_DEVICE;
        }
        g->member_streams.push_back(b->st);
        drop_graph(b);
    }
    for (Batch* b : g->members) b->st = g->st;
    // built-in choice: 4 waves per block, the fused x pass's exchange as
    // the single-shape kernels take it (joint in FP32, split in FP64), two
    // pencils per lane group in the FP32 y passes (one in FP64), one block
    // per tile; the members' own kernels where a stage has only one half.
    // (128^2, 256^2 and 512^2 FP32 members: 369 us per step, against 415
    // with one pencil per lane group.)
    g->choice = g->mixable ? (1 | (g->esz == 4 ? 2 | 8 : 0)) : g->nvar;
    s = g->esz == 8 ? group_upload<double>(g) : group_upload<float>(g);
    if (s == SPSTD_OK && (flags & SPSTD_AUTOTUNE))
        s = g->esz == 8 ? group_autotune<double>(g) : group_autotune<float>(g);
    if (s != SPSTD_OK) {
        for (size_t i = 0; i < g->members.size(); ++i) g->members[i]->st = g->member_streams[i];
        group_drop_graph(g);
        delete g;
        return s;
    }
    *out = g;
    return SPSTD_OK;
}

spstd_status spstd_batch_group_step(spstd_batch_group_t g, int64_t nsteps) {
    if (!g || nsteps < 0) return SPSTD_ERR_ARG;
    for (Batch* b : g->members)
        for (const Slot& sl : b->slots)
            if (sl.active && sl.steps + nsteps > b->d.nsteps_max) {
                g->err = "probe buffer capacity exceeded";
                return SPSTD_ERR_CAPACITY;
            }
    spstd_status s = g->esz == 8 ? group_step_t<double>(g, nsteps) : group_step_t<float>(g, nsteps);
    if (s != SPSTD_OK) return s;
    for (Batch* b : g->members)
        for (Slot& sl : b->slots)
            if (sl.active) sl.steps += nsteps;
    return SPSTD_OK;
}

spstd_status spstd_batch_group_schedule(spstd_batch_group_t g, int* choice, int* ncandidates, double* tuned_us) {
    if (!g) return SPSTD_ERR_ARG;
    if (choice) *choice = g->choice;
    if (ncandidates) *ncandidates = g->nvar + 1;
    if (tuned_us)
        for (int k = 0; k <= g->nvar; ++k) tuned_us[k] = g->tuned_us[k];
    return SPSTD_OK;
}

spstd_status spstd_batch_group_set_schedule(spstd_batch_group_t g, int choice) {
    if (!g || choice < 0 || choice > g->nvar || (choice < g->nvar && !g->mixable)) return SPSTD_ERR_ARG;
    if (hipStreamSynchronize(g->st) != hipSuccess) return SPSTD_ERR_DEVICE;
    group_drop_graph(g);
    for (Batch* b : g->members) drop_graph(b);
    g->choice = choice;
    return SPSTD_OK;
}

spstd_status spstd_batch_group_destroy(spstd_batch_group_t g) {
    if (!g) return SPSTD_ERR_ARG;
    (void)hipStreamSynchronize(g->st);
    group_drop_graph(g);
    for (size_t i = 0; i < g->members.size(); ++i) {
        drop_graph(g->members[i]);
        g->members[i]->st = g->member_streams[i];
    }
    delete g;
    return SPSTD_OK;
}

const char* spstd_batch_group_last_error(spstd_batch_group_t g) { return g ? g->err.c_str() : "null group"; }

}  // extern "C"
