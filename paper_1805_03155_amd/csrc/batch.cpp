// Batch engine: many independent instances of one shape advanced together.
//
// Slots are stacked in one buffer ([slot][z][y][x] for psi_R, psi_I, V) and
// every directional pass of a stage is one launch over all slots; each slot
// has its own row of the scale table (its dt, spacing, m* and hbar), its own
// probe points, probe buffer and step counter.  Free slots hold zero fields
// and zero scales, so they stay zero.  Short 1D batches and 2D batches of
// up to 64 x 64 points run a resident kernel (one launch per
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
    size_t psiR, psiI, V, tw[3], scales, pidx, active, counter, probes, rinst, total;
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
    L.probes = off; off += align256(cap * (size_t)(d->nsteps_max + 1) * np * 2 * sizeof(double));
    L.rinst = off; off += align256(cap * sizeof(ResidentInst<double>));
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
static hipError_t batch_step_once(Batch* b) {
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
    int owed = -1;
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
            if (a && e == hipSuccess && b->d.ndim == 3) e = batch_axis<R>(b, 2, pi, pr, sc, SC_KZA);
        }
        if (e != hipSuccess) break;
        if (a && bb) e = launch_x_ab<R>(nx, pr, pi, V, twx, rg, sc, b->d.nyquist, b->st, b->wpb);
        else if (a) e = launch_x_acc<R>(nx, pi, pr, V, twx, rg, sc, SC_KXA, SC_PA, b->d.nyquist, b->st, b->wpb);
        else if (bb) e = launch_x_acc<R>(nx, pr, pi, V, twx, rg, sc, SC_KXB, SC_PB, b->d.nyquist, b->st, b->wpb);
        if (e != hipSuccess) break;
        if (bb && b->d.ndim >= 2) {
            if (b->d.ndim == 3) e = batch_axis<R>(b, 2, pr, pi, sc, SC_KZB);
            owed = l;
        }
    }
    if (e == hipSuccess && owed >= 0) {
        const ScaleRef so{b->ws + b->L.scales, b->d.m, owed};
        e = batch_axis<R>(b, 1, pr, pi, so, SC_KYB);
    }
    if (e == hipSuccess && b->d.nprobes > 0)
        e = launch_probe_batch<R>(pr, pi, b->npts, reinterpret_cast<const int64_t*>(b->ws + b->L.pidx),
                                  b->d.nprobes, reinterpret_cast<const int*>(b->ws + b->L.active),
                                  b->d.capacity, reinterpret_cast<double*>(b->ws + b->L.probes),
                                  reinterpret_cast<int64_t*>(b->ws + b->L.counter), b->d.nsteps_max + 1, b->st);
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
        hipError_t e2 = hipSuccess;
        for (int s = 0; s < kBatchGraphChunk && e2 == hipSuccess; ++s) e2 = batch_step_once<R>(b);
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
        I.capacity = b->d.nsteps_max + 1;
        I.nprobes = b->d.nprobes;
        for (int q = 0; q < b->d.nprobes; ++q) I.probe_idx[q] = s.probe_idx[q];
        // kinetic scale per axis: (hbar/2m*) (2 pi/L)^2 / N for the bare k^2
        double kin[2] = {0.0, 0.0};
        for (int ax = 0; ax < b->d.ndim && ax < 2; ++ax) {
            const double k1 = k1base / ((double)b->d.n[ax] * s.dx[ax]);
            kin[ax] = s.hbar / (2.0 * s.mass) * k1 * k1 / (double)b->d.n[ax];
        }
        for (int l = 0; l < b->d.m; ++l) {
            const double a = b->c[l] * s.dt, bb = -b->dd[l] * s.dt;
            I.kin[2 * l] = (R)(a * kin[0]);
            I.kin[2 * l + 1] = (R)(bb * kin[0]);
            I.kin_y[2 * l] = (R)(a * kin[1]);
            I.kin_y[2 * l + 1] = (R)(bb * kin[1]);
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
            else
                BCHK(launch_resident_2d<R>(b->d.n[0], b->d.n[1], tab, b->nres, b->d.m, n, b->d.nyquist,
                                           b->ws + b->L.tw[0], b->ws + b->L.tw[1], b->st));
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
    for (; left > 0; --left) BCHK(batch_step_once<R>(b));
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
    // nominal instance: dx = hbar = m* = 1, V = 0, dt = 0.5 x_max / rho
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
    // every slot samples point 0 during the trial
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
    // back to an empty batch: zero scales, counters and active flags (the
    // fields stayed zero: a zero state steps to zero)
    std::vector<R> zr(rr.size(), (R)0);
    std::vector<int> za(b->d.capacity, 0);
    std::vector<int64_t> zc(b->d.capacity, 0);
    BCHK(hipMemcpyAsync(b->ws + b->L.scales, zr.data(), zr.size() * sizeof(R), hipMemcpyHostToDevice, b->st));
    BCHK(hipMemcpyAsync(b->ws + b->L.active, za.data(), za.size() * sizeof(int), hipMemcpyHostToDevice, b->st));
    BCHK(hipMemcpyAsync(b->ws + b->L.counter, zc.data(), zc.size() * sizeof(int64_t), hipMemcpyHostToDevice, b->st));
    BCHK(hipStreamSynchronize(b->st));
    for (Slot& sl : b->slots) sl = Slot{};
    b->rtab_dirty = true;
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
    b->resident = ((d->ndim == 1 && resident_len_ok(d->n[0])) || (d->ndim == 2 && resident2d_ok(d->n[0], d->n[1]))) &&
                  !(d->flags & SPSTD_NO_RESIDENT);
    b->wpb = d->waves_per_block;
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
    for (int a = 0; a < d->ndim && e == hipSuccess; ++a) {
        // FP64 in every precision: the kernels round each twiddle once
        std::vector<double> t = twiddles(d->n[a]);
        e = hipMemcpyAsync(b->ws + L.tw[a], t.data(), t.size() * 8, hipMemcpyHostToDevice, b->st);
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
                                           b->d.nsteps_max + 1, b->st);
        else
            e = launch_probe_batch<float>(BF<float>(b, b->L.psiR) + (int64_t)slot * b->npts,
                                          BF<float>(b, b->L.psiI) + (int64_t)slot * b->npts, b->npts,
                                          reinterpret_cast<const int64_t*>(b->ws + b->L.pidx) + slot * np, b->d.nprobes,
                                          reinterpret_cast<const int*>(b->ws + b->L.active) + slot, 1,
                                          reinterpret_cast<double*>(b->ws + b->L.probes + poff),
                                          reinterpret_cast<int64_t*>(b->ws + b->L.counter) + slot,
                                          b->d.nsteps_max + 1, b->st);
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
    if (e == hipSuccess && probes_out && np > 0) {
        const size_t poff = (size_t)slot * (b->d.nsteps_max + 1) * np * 2 * sizeof(double);
        e = hipMemcpy(probes_out, b->ws + b->L.probes + poff, (size_t)(s.steps + 1) * np * 2 * sizeof(double),
                      hipMemcpyDeviceToHost);
    }
    double* outs[2] = {psiR, psiI};
    const size_t offs[2] = {b->L.psiR, b->L.psiI};
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        if (!outs[k]) continue;
        if (b->esz == 8) {
            e = hipMemcpy(outs[k], b->ws + offs[k] + (size_t)slot * b->npts * 8, b->npts * 8, hipMemcpyDeviceToHost);
        } else {
            std::vector<float> tmp(b->npts);
            e = hipMemcpy(tmp.data(), b->ws + offs[k] + (size_t)slot * b->npts * 4, b->npts * 4,
                          hipMemcpyDeviceToHost);
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
