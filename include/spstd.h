/*
 * spstd.h -- C ABI of the MI355X SPSTD engine.
 *
 * The engine advances the time-dependent Schroedinger equation
 *     i hbar d(psi)/dt = -(hbar^2 / 2 m*) Laplacian psi + V(r) psi      (Eq. 1)
 * on a collocated grid (Eq. 5-6), periodic along each axis or between
 * Dirichlet or Neumann walls (Sec. 2.2), with psi = psi_R + i psi_I
 * (Eq. 2-4), the pseudospectral second derivative (Eq. 7-10; sine or cosine
 * modes between walls) and the partitioned symplectic stage update
 * (Eq. 13-18) of Shen, Sha, Kuang, Hu,
 * Huang and Wu, "Symplectic Pseudospectral Time-Domain Scheme for Solving
 * Time-Dependent Schroedinger Equation" (arXiv:1805.03155).  Eigenvalues are
 * read from the time spectrum of probe-point series (Sec. 3, Tables 2-4).
 *
 * Conventions shared by every call:
 *   - Every call returns spstd_status; 0 is success.  Nothing aborts or
 *     throws across the ABI.
 *   - Grids are row-major with x fastest: index = (z * ny + y) * nx + x.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the current device.  The library never allocates
 *     device memory: the caller passes one device workspace per plan
 *     (size from spstd_workspace_size) and owns it.
 *   - A plan is not thread-safe; distinct plans are independent.
 *   - Stage l of a step applies first  psi_R += c_l dt K psi_I  and then
 *     psi_I -= d_l dt K psi_R  (Eq. 17-18 with K of Eq. 16); stages whose
 *     coefficient is 0 are skipped.
 */
#ifndef SPSTD_H
#define SPSTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spstd_status {
    SPSTD_OK = 0,
    SPSTD_ERR_ARG = 1,        /* an argument is out of range or malformed */
    SPSTD_ERR_UNSTABLE = 2,   /* dt * rho >= x_max (Eq. 24-30) without SPSTD_ALLOW_UNSTABLE */
    SPSTD_ERR_WORKSPACE = 3,  /* workspace missing, too small or misaligned */
    SPSTD_ERR_DEVICE = 4,     /* a HIP runtime call failed */
    SPSTD_ERR_NONFINITE = 5,  /* the state holds NaN or Inf after a run */
    SPSTD_ERR_CAPACITY = 6,   /* more steps than the probe buffer holds */
    SPSTD_ERR_SCRATCH = 7     /* spstd_run_noalloc: working memory beyond its fixed scratch */
} spstd_status;

enum { SPSTD_FP64 = 0, SPSTD_FP32 = 1 };            /* storage and arithmetic of fields */
enum { SPSTD_NYQ_FULL = 0, SPSTD_NYQ_ZERO = 1 };    /* Nyquist bin convention, see below */
enum { SPSTD_SYMPLECTIC = 0, SPSTD_RK4 = 1 };        /* time integrator */
enum { SPSTD_BC_PERIODIC = 0, SPSTD_BC_DIRICHLET = 1, SPSTD_BC_NEUMANN = 2 };  /* per axis */
enum { SPSTD_LAP_SPECTRAL = 0, SPSTD_LAP_FD3 = 1 };  /* spatial second derivative */

#define SPSTD_ALLOW_UNSTABLE 0x1u                    /* flags: accept dt beyond the edge */
#define SPSTD_EAGER 0x2u                             /* flags: launch kernels one by one
                                                        instead of replaying step-chunk graphs */
#define SPSTD_TIMING 0x4u                            /* flags: eager launches, each pass kernel
                                                        bracketed by HIP events (spstd_pass_times) */
#define SPSTD_NO_RESIDENT 0x8u                       /* flags: 1D and small 2D plans and
                                                        batches use the pass kernels even
                                                        where a resident kernel applies */
#define SPSTD_AUTOTUNE 0x10u                         /* batch flags: time the candidate schedules
                                                        at creation and keep the faster */
#define SPSTD_NO_MERGE 0x20u                         /* flags: keep every step boundary whole:
                                                        neither merged (last stage without a B
                                                        half; then a run split over calls equals
                                                        the unsplit run bitwise) nor chained
                                                        (last stage with one) */
#define SPSTD_NO_PLANES 0x40u                        /* batch flags: 3D batches whose x and z
                                                        axes have 16, 32 or 64 points run the z
                                                        and x passes of a stage as separate
                                                        launches instead of one fused launch
                                                        per x-z plane */
#define SPSTD_NO_FOURSTEP 0x80u                      /* batch flags: 1D batches of 8192- or
                                                        16384-point rows run each x pass as one
                                                        workgroup per pair of rows instead of
                                                        the four-step launches over many */
#define SPSTD_MAX_STAGES 16
#define SPSTD_MAX_PROBES 64
#define SPSTD_MAX_EIG 8

/*
 * Problem descriptor (caller-owned; copied by spstd_plan).
 *   ndim         1, 2 or 3.
 *   n[3]         points per axis (unused axes must be 1).  Powers of two;
 *                periodic x: 16..16384, y, z: 16..1024; walled (see bc)
 *                x: 16..8192, y, z: 16..512.
 *   dx[3]        grid spacing per axis (> 0), so L_d = n_d * dx_d.
 *   hbar, mass   hbar and m* (> 0); the configs use 1 and 1.
 *   precision    SPSTD_FP64 or SPSTD_FP32 (fields, potential and transforms
 *                stored and computed in that type; probes, norms and the
 *                spectrum are always FP64).
 *   method       SPSTD_SYMPLECTIC (Eq. 17-18) or SPSTD_RK4 (classical
 *                fourth-order Runge-Kutta on d/dt(psi_R, psi_I) =
 *                (K psi_I, -K psi_R), the non-symplectic comparison of Sec. 3.1).
 *   m, c, d      stage count (1..16) and coefficients (host, length m) of
 *                Eq. (17); ignored for RK4.  The paper's set is
 *                c = (0.26833010, -0.18799162, 0.91966152), d_l = c_{m-l+1}.
 *   dt           time step; 0 selects dt = cfl_fraction * x_max / rho with
 *                x_max the first x where |tr L^d(x)| = 2 (Eq. 23-25) and
 *                rho = (hbar/2m*) sum_d (pi/dx_d)^2 + max|V|/hbar.
 *   cfl_fraction used when dt == 0 (0 < f < 1).
 *   nyquist      SPSTD_NYQ_FULL: symbol -k^2 with |k| = pi/dx at the Nyquist
 *                bin (direct second derivative); SPSTD_NYQ_ZERO: the Nyquist
 *                term removed, as Eq. (10) read literally (two first
 *                derivatives, real part kept after each inverse transform).
 *   nprobes      0..64 probe points; probe_idx (host) their linear indices.
 *   flags        SPSTD_ALLOW_UNSTABLE, SPSTD_EAGER, SPSTD_TIMING, SPSTD_NO_RESIDENT,
 *                SPSTD_NO_MERGE
 *                (OR-ed), or 0.  Periodic spectral symplectic plans in 1D,
 *                or in 2D with n_x, n_y in {16, 32, 64}, with at most 8
 *                probes, no eigenstate sums and no SPSTD_TIMING run each
 *                spstd_step call as one launch of a kernel that keeps the
 *                grid on chip.  Where the last stage has no B half, the A
 *                halves at the boundaries between the steps of one call run
 *                as one; where it has one, the y pass that ends a step and
 *                the one that opens the next run as one sweep (both unless
 *                SPSTD_NO_MERGE; the probe samples are those of the whole
 *                boundaries).
 *   bc[3]        boundary per axis (Sec. 2.2, last paragraph):
 *                SPSTD_BC_PERIODIC (DFT; sample j at j * dx), or walls at
 *                x = 0 and x = L_d with samples at cell centres (j + 1/2) dx:
 *                SPSTD_BC_DIRICHLET (psi = 0 at the walls, sine transform),
 *                SPSTD_BC_NEUMANN (zero normal derivative, cosine transform).
 *                A zero-initialised descriptor is periodic everywhere.
 *   laplacian    SPSTD_LAP_SPECTRAL (Eq. 9-10, the method) or SPSTD_LAP_FD3:
 *                the second-order central difference (f[j+1] - 2 f[j] +
 *                f[j-1]) / dx^2 per axis with periodic wrap, the FDTD
 *                comparison of Table 1 and Tables 2-3 (periodic axes only;
 *                rho then uses the difference operator's bound 4/dx^2 per
 *                axis in place of (pi/dx)^2; no spstd_energy).  With m = 1,
 *                c = d = (1) the spectral setting is the PSTD comparison
 *                (Eq. 11-12).
 *   neig         0..8: eigenstate accumulators reserved in the workspace
 *                (spstd_eig_begin); each costs 16 bytes per grid point.
 */
typedef struct spstd_desc {
    int ndim;
    int64_t n[3];
    double dx[3];
    double hbar, mass;
    int precision;
    int method;
    int m;
    const double *c, *d;
    double dt;
    double cfl_fraction;
    int nyquist;
    int nprobes;
    const int64_t *probe_idx;
    uint32_t flags;
    int bc[3];
    int laplacian;
    int neig;
} spstd_desc;

typedef struct spstd_plan_s *spstd_plan_t;

/* Run statistics (host, filled by spstd_run and spstd_plan_info). */
typedef struct spstd_stats {
    int64_t steps_done;    /* steps taken since the plan was made */
    double dt;             /* time step in use */
    double xmax;           /* stability edge x_max of the coefficient set */
    double rho;            /* the spectral-radius bound used for dt */
    double norm0;          /* sum |psi|^2 * cell volume at plan time */
    double norm;           /* the same after the last spstd_run */
    double substeps_per_step; /* non-zero A and B substeps per step (RK4: 8) */
} spstd_stats;

/*
 * Stability edge of a coefficient set: the smallest x > 0 beyond which
 * |tr L^d(x)| > 2, L^d the per-mode evolution matrix of Eq. (23)
 * (Eq. 24-25).  c, d: host arrays of length m.  Pure host computation.
 * Errors: SPSTD_ERR_ARG for m outside 1..16, null pointers or no edge below 1e3.
 */
spstd_status spstd_xmax(int m, const double *c, const double *d, double *xmax_out);

/*
 * The time step spstd_plan would choose: cfl_fraction * x_max / rho with
 * rho as described for spstd_desc.dt (Eq. 24-30 extended by max|V|/hbar).
 * V: host array of the grid's size.  Pure host computation.
 */
spstd_status spstd_stable_dt(const spstd_desc *desc, const double *V, double *dt_out);

/*
 * Exact device workspace size, in bytes, of a plan for desc that can record
 * up to nsteps_max steps of probe samples.  Pure host computation.
 */
spstd_status spstd_workspace_size(const spstd_desc *desc, int64_t nsteps_max, size_t *bytes);

/*
 * Create a plan: validate desc, fix dt, build the FP64 twiddle tables and
 * copy V, psi_R(0), psi_I(0) (host FP64 arrays of the grid's size; psi_I may
 * be NULL for zero) into d_workspace (device, ws_bytes >= the size returned
 * by spstd_workspace_size for the same nsteps_max, 256-byte aligned).
 * stream: a hipStream_t (NULL for the null stream) on which every kernel of
 * the plan runs.  Records probe sample 0 (the initial state).  Synchronises
 * the stream before returning.  *out receives the plan; release it with
 * spstd_destroy (the workspace stays the caller's).
 * Errors: SPSTD_ERR_ARG, SPSTD_ERR_UNSTABLE, SPSTD_ERR_WORKSPACE,
 * SPSTD_ERR_DEVICE.
 */
spstd_status spstd_plan(const spstd_desc *desc, const double *V, const double *psiR0,
                        const double *psiI0, void *d_workspace, size_t ws_bytes,
                        int64_t nsteps_max, void *stream, spstd_plan_t *out);

/*
 * Enqueue nsteps time steps (Eq. 17-18 per step, or RK4) on the plan's stream
 * and record one probe sample after each.  Asynchronous: returns once the
 * work is queued.  SPSTD_ERR_CAPACITY if the probe buffer would overflow
 * (nothing is queued then).
 */
spstd_status spstd_step(spstd_plan_t plan, int64_t nsteps);

/*
 * spstd_step(nsteps), then synchronise, check the state for NaN/Inf
 * (SPSTD_ERR_NONFINITE), update stats and copy the whole probe series
 * recorded so far to probe_out (host, [(steps_done + 1) * nprobes * 2]
 * doubles as (psi_R, psi_I) per probe per sample; may be NULL).
 * stats_out may be NULL.
 */
spstd_status spstd_run(spstd_plan_t plan, int64_t nsteps, double *probe_out,
                       spstd_stats *stats_out);

/*
 * Energy diagnostics of the current state psi = psi_R + i psi_I, the pieces
 * of <H> with H = hbar K (Sec. 2.2, Eq. 16), each summed over the grid and
 * multiplied by the cell volume:
 *   out[0] kinetic   sum psi* (-(hbar^2/2m*) Laplacian) psi, with the
 *                    plan's spectral second derivative (Eq. 9-10 and the
 *                    plan's Nyquist convention), by Parseval per axis;
 *   out[1] potential sum V |psi|^2;
 *   out[2] norm      sum |psi|^2.
 * <H> = (out[0] + out[1]) / out[2].  out: host array of 3 doubles.  Sums are
 * FP64 in a fixed order (deterministic).  Runs on the plan's stream after
 * the steps already queued and synchronises it.  Errors: SPSTD_ERR_ARG (null
 * pointers), SPSTD_ERR_NONFINITE (state not finite), SPSTD_ERR_DEVICE.
 */
spstd_status spstd_energy(spstd_plan_t plan, double *out);

/*
 * Eigenstate reconstruction (Sec. 3.1-3.2, Figs. 1, 2 and 4: eigenstates at
 * chosen eigenfrequencies from the same time-domain run).  After this call
 * each of the next nsteps steps adds its resulting state, weighted, into
 * one accumulator per energy:
 *   phi_k(r) = sum_{m=0}^{nsteps-1} w_m psi(r, t_m) exp(+i E_k m dt / hbar)
 * with psi(r, t_m) the state after m + 1 steps counted from this call and
 * w_m the symmetric 4-term Blackman-Harris window of length nsteps (the
 * spectrum's window).  E: host array of nE energies (nE <= the plan's
 * neig), e.g. levels returned by spstd_spectrum.  Steps beyond nsteps add
 * nothing.  Accumulators are FP64 in every precision.  Resets earlier
 * accumulations.  Errors: SPSTD_ERR_ARG (neig == 0, nE outside 1..neig,
 * nsteps < 2, non-finite E), SPSTD_ERR_DEVICE.
 */
spstd_status spstd_eig_begin(spstd_plan_t plan, const double *E, int nE, int64_t nsteps);

/*
 * Copy accumulator k (0 <= k < nE of the last spstd_eig_begin) to host
 * arrays re and im of the grid's size (row-major, x fastest).  Synchronises
 * the plan's stream.  Errors: SPSTD_ERR_ARG, SPSTD_ERR_DEVICE.
 */
spstd_status spstd_eig_read(spstd_plan_t plan, int k, double *re, double *im);

/* Statistics without running (steps_done, dt, x_max, rho, norm0). */
spstd_status spstd_plan_info(spstd_plan_t plan, spstd_stats *stats_out);

/*
 * Device pointers of the plan's fields (psi_R, psi_I, V) and of its FP64
 * probe buffer, for callers that read them in place (e.g. as tensors).
 * The element type of the fields follows desc.precision.
 */
spstd_status spstd_device_fields(spstd_plan_t plan, void **psiR, void **psiI, void **V,
                                 double **probes);

/*
 * Checkpoint: copy the state to host FP64 arrays (synchronising), with the
 * step count; and restore it (the probe series restarts at the given step
 * count: samples beyond it are discarded).  psiI may be NULL on get.
 */
spstd_status spstd_get_state(spstd_plan_t plan, double *psiR, double *psiI, int64_t *step);
spstd_status spstd_set_state(spstd_plan_t plan, const double *psiR, const double *psiI,
                             int64_t step);

/*
 * Eigenvalues from probe time series (Sec. 3: time-FFT of the recorded wave
 * function; Tables 2-4).  series: host [nsamples][nprobes][2] (psi_R, psi_I)
 * sampled every dt.  Reading of the unstated details: the conjugated complex
 * series per probe, a symmetric 4-term Blackman-Harris window, zero padding
 * to 2^ceil(log2(8 nsamples)), power summed over probes, local maxima above
 * 1e-8 of the largest, each refined to the zero of the derivative of the
 * windowed DTFT power; E = hbar * omega ascending.  Writes up to nlevels
 * energies to E_out and amplitudes to amp_out (may be NULL), the count to
 * *nfound (fewer than nlevels is not an error).  Pure host FP64.
 */
spstd_status spstd_spectrum(const double *series, int64_t nsamples, int nprobes, double dt,
                            double hbar, int nlevels, double *E_out, double *amp_out,
                            int *nfound);

/*
 * Kinds of pass kernels, for spstd_pass_times.  Y and Z: one directional
 * second-derivative pass along y or z added into a field; XAB: the fused A
 * and B halves along x of one stage (Eq. 18 and its psi_I mirror); X: one
 * half-stage along x; YBA: the y pass of the B half of a stage fused with
 * the y pass of the A half of the next stage (one sweep of the y pencils).
 */
enum { SPSTD_PASS_Y = 0, SPSTD_PASS_Z = 1, SPSTD_PASS_XAB = 2, SPSTD_PASS_X = 3,
       SPSTD_PASS_YBA = 4, SPSTD_NPASS_KINDS = 5 };

/*
 * Per-kind kernel timing of a plan made with SPSTD_TIMING: synchronises the
 * plan's stream and returns, for each kind k < SPSTD_NPASS_KINDS, the number
 * of launches since the previous call (launches[k]), their summed duration
 * in milliseconds measured with HIP events recorded on the plan's stream
 * around each launch (total_ms[k]; the events carry no system-scope fence,
 * and one event ends a launch and starts the next when nothing else was
 * enqueued between them), and the algorithmic HBM bytes of one
 * launch (bytes_per_launch[k]: every field read once and every field written
 * once).  Host arrays of SPSTD_NPASS_KINDS entries; any may be NULL.
 * SPSTD_ERR_ARG if the plan was made without SPSTD_TIMING.
 */
spstd_status spstd_pass_times(spstd_plan_t plan, int64_t *launches, double *total_ms,
                              double *bytes_per_launch);

spstd_status spstd_destroy(spstd_plan_t plan);
const char *spstd_strerror(spstd_status status);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work
 * of spstd_plan + spstd_run on fields the caller already holds on the
 * device, with every other piece of working memory (twiddle and scale
 * tables, probe indices, the step counter, merged-boundary samples, the
 * resident kernels' instance table) in one fixed static device array of the
 * library, SPSTD_NOALLOC_SCRATCH_BYTES per GPU, held until the process
 * ends.  No hipMalloc, hipFree or other device allocation is made.
 *   desc    as for spstd_plan, with method SPSTD_SYMPLECTIC, neig = 0, an
 *           explicit dt > 0 (V is not read on the host, so dt is neither
 *           derived nor checked against the stability edge; use
 *           spstd_stable_dt beforehand) and no SPSTD_TIMING; kernels launch
 *           one by one (no graph is captured).
 *   V       device, N values in desc->precision, read only.
 *   psiR, psiI  device, N values each in desc->precision: the initial state
 *           on entry, the state after nsteps steps on return.
 *   probes  device, (nsteps + 1) * nprobes * 2 doubles written as
 *           spstd_run's series (sample 0 = the initial state); may be NULL
 *           when nprobes = 0.
 *   The three fields are 256-byte aligned; all memory is on the current
 *   device; stream is a hipStream_t (NULL: null stream).  Synchronises the
 *   stream before returning.
 * The scratch array is shared by every call on a GPU and keeps the last
 * call's contents (each call re-initialises what it reads): calls that
 * overlap on one GPU (from several host threads or streams) race.
 * Errors: SPSTD_ERR_ARG (bad descriptor or pointers), SPSTD_ERR_SCRATCH (the
 * grid's tables exceed the scratch: x transforms of up to 16384 points fit),
 * SPSTD_ERR_DEVICE (HIP error, or a probe index found outside the grid).
 */
#define SPSTD_NOALLOC_SCRATCH_BYTES (384u * 1024u)
spstd_status spstd_run_noalloc(const spstd_desc *desc, const void *V, void *psiR, void *psiI,
                               int64_t nsteps, double *probes, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many independent instances of one grid shape advanced together
 * (each with its own spacing, hbar, m*, V, initial state, dt and probes; the
 * coefficient set is shared).  Instances live in slots of one stacked
 * buffer; every pass of a stage is one launch over all slots, so a step of
 * the whole batch costs what one large grid costs.  Slots are loaded and
 * released while others keep running, which is what the serving loop uses.
 * ------------------------------------------------------------------------ */
typedef struct spstd_batch_s *spstd_batch_t;

/*
 * Batch descriptor (caller-owned; copied by spstd_batch_create).
 *   ndim, n[3]    shape of every instance (as spstd_desc).
 *   precision     SPSTD_FP64 or SPSTD_FP32.
 *   m, c, d       stage coefficients of Eq. (17), shared by all slots.
 *   nyquist       as spstd_desc.
 *   capacity      number of slots (>= 1).
 *   nprobes       probe points per slot, 0..8.
 *   nsteps_max    probe samples kept per slot after sample 0.
 *   flags         SPSTD_ALLOW_UNSTABLE, SPSTD_NO_RESIDENT, SPSTD_AUTOTUNE,
 *                 SPSTD_NO_MERGE, SPSTD_NO_PLANES, SPSTD_NO_FOURSTEP.
 *                 The pass kernels of 1D batches of 8192 or 16384 points
 *                 run each x pass in four steps (Sec. 2, Eq. (9)-(10): the
 *                 row's transform factored as 128 columns by n/128 rows,
 *                 column, row and column launches over many workgroups,
 *                 with a scratch copy of each row pair in the workspace);
 *                 SPSTD_NO_FOURSTEP keeps one workgroup per row pair (one
 *                 launch per pass, fewer workgroups: the better neighbour
 *                 for other work on the device).
 *                 A 1D batch of up to 16384 points, a 2D batch of n_x,
 *                 n_y in {16, 32, 64}, or a 16^3 batch has two schedules:
 *                 the resident kernel (whole step chunks in one launch; a
 *                 2D instance lives in one workgroup's LDS, a 3D instance
 *                 is stepped by one workgroup in its own arrays) or the
 *                 pass kernels replayed as step graphs.  The pass kernels
 *                 run 2 or 4 waves per block.  SPSTD_AUTOTUNE runs every
 *                 candidate (resident where it applies; passes at 2 and at
 *                 4 waves per block) for a few steps on the empty batch at
 *                 creation (every slot stepping a zero state at a nominal
 *                 dt), keeps the fastest, and remembers the choice for this
 *                 (shape, precision, capacity) for the rest of the process.
 *   waves_per_block  block size of the pass kernels in 64-lane waves: 0
 *                 for the built-in choice per precision and length, or 2 or
 *                 4 (rows longer than 1024 points run one pencil per block,
 *                 or the four-step launches, whatever it says).
 *                 SPSTD_AUTOTUNE overrides it.
 */
typedef struct spstd_batch_desc {
    int ndim;
    int64_t n[3];
    int precision;
    int m;
    const double *c, *d;
    int nyquist;
    int capacity;
    int nprobes;
    int64_t nsteps_max;
    uint32_t flags;
    int waves_per_block;
} spstd_batch_desc;

/* Exact device workspace size of a batch.  Pure host computation. */
spstd_status spstd_batch_workspace_size(const spstd_batch_desc *desc, size_t *bytes);

/*
 * Create a batch over the caller's device workspace (256-byte aligned,
 * ws_bytes >= spstd_batch_workspace_size); all slots start free.  stream: a
 * hipStream_t (NULL for the null stream) for every kernel of the batch.
 * Synchronises the stream.  Errors: SPSTD_ERR_ARG, SPSTD_ERR_WORKSPACE,
 * SPSTD_ERR_DEVICE.
 */
spstd_status spstd_batch_create(const spstd_batch_desc *desc, void *d_workspace, size_t ws_bytes,
                                void *stream, spstd_batch_t *out);

/*
 * Load an instance into a free slot: spacing dx[ndim], hbar, m*, the time
 * step (dt > 0, or dt == 0 for cfl_fraction * x_max / rho of this instance,
 * as in spstd_desc), host FP64 arrays V, psi_R(0), psi_I(0) (NULL for zero)
 * of the shape's size, and nprobes linear probe indices.  Records sample 0,
 * marks the slot active and writes the time step used to *dt_out (may be
 * NULL).  Synchronises the batch stream.  Errors: SPSTD_ERR_ARG (slot busy or
 * out of range, bad values), SPSTD_ERR_UNSTABLE, SPSTD_ERR_DEVICE.
 */
spstd_status spstd_batch_load(spstd_batch_t batch, int slot, const double *dx, double hbar, double mass,
                              double dt, double cfl_fraction, const double *V, const double *psiR0,
                              const double *psiI0, const int64_t *probe_idx, double *dt_out);

/*
 * Enqueue nsteps steps of every active slot (asynchronous).  Each active
 * slot records one probe sample per step.  SPSTD_ERR_CAPACITY (nothing
 * queued) if a slot would pass nsteps_max.
 */
spstd_status spstd_batch_step(spstd_batch_t batch, int64_t nsteps);

/*
 * Synchronise and copy a slot's probe series ([(steps_done + 1) * nprobes * 2]
 * doubles) and state (host FP64, N values each); any output may be NULL.
 * SPSTD_ERR_NONFINITE if a copied state holds NaN or Inf.
 */
spstd_status spstd_batch_read(spstd_batch_t batch, int slot, double *probes_out, double *psiR,
                              double *psiI, int64_t *steps_done);

/* Free a slot (its fields and scales are cleared).  Synchronises. */
spstd_status spstd_batch_release(spstd_batch_t batch, int slot);

/* The schedule in use: *resident = 1 for a resident kernel, 0 for the
 * pass kernels; *waves_per_block = the pass kernels' block size in waves (0:
 * the built-in choice; may be NULL); tuned_us[0..2] = the measured
 * microseconds per step at creation of [resident, passes at 2 waves/block,
 * passes at 4 waves/block] (0 where not measured; may be NULL). */
spstd_status spstd_batch_schedule(spstd_batch_t batch, int *resident, int *waves_per_block,
                                  double *tuned_us);

/* Slot state: active flag, steps since its load, time step. */
spstd_status spstd_batch_slot_info(spstd_batch_t batch, int slot, int *active, int64_t *steps_done,
                                   double *dt);

spstd_status spstd_batch_destroy(spstd_batch_t batch);
const char *spstd_batch_last_error(spstd_batch_t batch);

/* ------------------------------------------------------------------------
 * Groups: 2D batches of different shapes (the uneven instances of the
 * batching form) advanced together.  Every pass of the stage sequence is
 * one persistent launch over all members: it walks a device table of tiles
 * (member, block of that member's own grid) and runs, per tile, the pass
 * body for that member's shape, fields, twiddles and scales.  A group
 * takes over its members: from its creation until its destruction the
 * members' kernels, and their slot loads, reads and releases, run on the
 * group's stream (so they order with the group's steps); step the members
 * through the group only.
 * ------------------------------------------------------------------------ */
typedef struct spstd_batch_group_s *spstd_batch_group_t;

/*
 * Members: 1..64 distinct 2D batches whose axes have 128, 256 or 512
 * points, with one precision, coefficient set, Nyquist convention and
 * probe count.  Exact device workspace of a group (tile tables).  Pure host
 * computation.  SPSTD_ERR_ARG for members that do not qualify.
 */
spstd_status spstd_batch_group_workspace_size(const spstd_batch_t *members, int nmembers, size_t *bytes);

/*
 * Create a group over the caller's device workspace (256-byte aligned).
 * Schedules (candidates): k < n (n = 16 in FP32, 8 in FP64) the mixed-shape
 * kernels with 2 << (k & 1) waves per block, the joint LDS exchange of the
 * fused x pass for rows under 512 points if k & 2 (else split), one
 * persistent block per compute unit striding over the tiles if k & 4 (else
 * one block per tile), and two complex pencils per lane group in the y
 * passes if k & 8 (FP32); k = n the members' own pass kernels one member
 * after another on the group's stream.  Sets whose stages do not all have both halves (a zero c_l or
 * d_l) run k = n only.  flags: SPSTD_AUTOTUNE times every candidate (16
 * warm-up and 32 timed steps, every slot stepping a zero state at a nominal
 * instance's scales; the members must have no active slot) and keeps the
 * fastest (within 3% of it, one block per compute unit, which leaves room
 * for other streams' kernels); otherwise the built-in choice (4 waves per
 * block, the exchange of the single-shape kernels, one block per tile, two
 * pencils per lane group in FP32 and one in FP64).  Synchronises the
 * members' streams.  Errors: SPSTD_ERR_ARG, SPSTD_ERR_WORKSPACE,
 * SPSTD_ERR_DEVICE.
 */
spstd_status spstd_batch_group_create(const spstd_batch_t *members, int nmembers, uint32_t flags,
                                      void *d_workspace, size_t ws_bytes, void *stream,
                                      spstd_batch_group_t *out);

/* Enqueue nsteps steps of every active slot of every member (asynchronous);
 * SPSTD_ERR_CAPACITY (nothing queued) if a slot would pass its nsteps_max. */
spstd_status spstd_batch_group_step(spstd_batch_group_t group, int64_t nsteps);

/* The schedule in use (*choice, as numbered for spstd_batch_group_create),
 * the number of candidates and, after SPSTD_AUTOTUNE, the measured
 * microseconds per step of each (0 where not measured); any may be NULL. */
spstd_status spstd_batch_group_schedule(spstd_batch_group_t group, int *choice, int *ncandidates,
                                        double *tuned_us);

/* Use schedule `choice` from now on (synchronises the group's stream). */
spstd_status spstd_batch_group_set_schedule(spstd_batch_group_t group, int choice);

/* Release the group (the members keep their slots and return to their own
 * streams; synchronises). */
spstd_status spstd_batch_group_destroy(spstd_batch_group_t group);
const char *spstd_batch_group_last_error(spstd_batch_group_t group);
/* Text of the last error recorded on the plan (never NULL). */
const char *spstd_last_error(spstd_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif /* SPSTD_H */
