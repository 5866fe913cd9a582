/*
 * bte.h -- C ABI of the MI355X solver for the 2-D spatially homogeneous
 * superlattice Boltzmann transport equation (D. Priimak, arXiv:1401.6047).
 *
 * The solver advances the Fourier-in-phi_x / finite-difference-in-phi_y
 * distribution (a_n(phi_y), b_n(phi_y)) with the paper's combined
 * Crank-Nicolson / staggered leap-frog scheme (Sec. 3: operator T, whole and
 * fractional grids, start-up half-step) under E(t) = E_dc + E_w cos(w t) and
 * constant B, relaxing towards the Boltzmann equilibrium (Sec. 2), and takes
 * the drift-velocity and absorption reductions every step (Sec. 2, v_dr and
 * A definitions).
 *
 * Conventions shared by every entry point:
 *   - N_x harmonics are kept: a_0 .. a_{N_x-1} and b_1 .. b_{N_x-1}; b_0 is a
 *     fixed zero.  phi_y(m) = phi_min + m (phi_max - phi_min)/(N_y - 1),
 *     m = 0 .. N_y-1.  Both are zero outside these ranges (Sec. 3 boundary
 *     conditions).
 *   - Time is in units of the relaxation time tau (Sec. 2 scaling), so tau
 *     must be 1.  The whole grid is at integer steps k (t = k dt), the
 *     fractional grid at k + 1/2.
 *   - Host arrays are row-major [n][m] doubles (m fastest), N_x * N_y long,
 *     copied in or out before the call returns; the caller keeps ownership.
 *   - Device memory is never allocated behind the caller's back when a
 *     workspace is passed: the caller owns the workspace and keeps it alive
 *     until bte_destroy.  Passing a NULL workspace makes the library allocate
 *     (and free on destroy) one of the size bte_workspace_bytes reports.
 *   - All device work is queued on the HIP stream given at creation (NULL =
 *     the null stream).  bte_step only queues work; bte_observables,
 *     bte_get_state and bte_set_state synchronise that stream.
 *   - Every call returns a bte_status; no exception or abort crosses the ABI.
 *     On failure bte_last_error() gives a message (thread-local, valid until
 *     the next failing call on the same thread).
 *   - A solver handle is not thread-safe; distinct handles are independent.
 */
#ifndef BTE_H
#define BTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BTE_OK = 0,
    BTE_EINVAL = -1,     /* invalid argument: nothing was changed */
    BTE_ENOMEM = -2,     /* workspace too small, or allocation failed */
    BTE_EDEVICE = -3,    /* a HIP runtime call failed */
    BTE_EUNSTABLE = -4,  /* sticky: norm drifted or an observable is not finite */
    BTE_ESTATE = -5      /* call not valid in the handle's current state */
} bte_status;

typedef enum {
    BTE_FP64 = 0,        /* state and arithmetic in FP64 */
    BTE_FP32_BULK = 1    /* state stored in FP32; cell update, scalars and
                            accumulators in FP64 */
} bte_precision;

/* Kernel form used by bte_step. */
typedef enum {
    BTE_KERNEL_FUSED = 0,    /* one launch per step: whole + fractional half-steps
                                fused, ping-pong state buffers */
    BTE_KERNEL_TWO_PASS = 1, /* two launches per step, each half-step in place
                                (the paper's two-kernel structure) */
    BTE_KERNEL_FUSED2 = 2,   /* one launch per two steps: four half-steps chained
                                in registers, ping-pong state buffers (an odd
                                step count ends with one BTE_KERNEL_FUSED step) */
    BTE_KERNEL_FUSED3 = 3    /* one launch per three steps: six half-steps
                                chained in registers, ping-pong state buffers
                                (a remainder of two or one steps runs as one
                                FUSED2 or FUSED launch) */
} bte_kernel;

typedef struct {
    int32_t n_x;         /* harmonics kept, >= 2 */
    int32_t n_y;         /* phi_y points, both ends included, >= 3 */
    double phiy_min;     /* box edges, phiy_max > phiy_min */
    double phiy_max;
} bte_grid;

typedef struct {
    double E_dc;         /* dc field (Sec. 2 field protocol) */
    double E_w;          /* ac amplitude */
    double omega;        /* ac angular frequency (> 0 when E_w != 0) */
    double B;            /* magnetic field */
    double mu;           /* Delta_1/(2 k_B T) > 0, sets f0 */
    double alpha;        /* m/m_x > 0; enters the normalisation of f0 and v_dr only */
    double tau;          /* must be 1: time is measured in units of tau */
    double dt;           /* time step > 0, with dt |B| / (2 dphi) < 1 (leap-frog bound) */
    int32_t precision;   /* bte_precision */
    uint32_t flags;      /* reserved, must be 0 */
} bte_params;

/* Launch shape of the step kernels.  Zero fields take the library default
   for the grid; bte_tune() picks one by measurement. */
typedef struct {
    int32_t kernel;          /* bte_kernel */
    int32_t rows_per_wave;   /* harmonics handled by one wavefront, 1 .. 62 (used up to 58
                                for FUSED2 and 54 for FUSED3) */
    int32_t waves_per_block; /* 1, 2, 4 or 8 (used up to 4 for FUSED2 and FUSED3) */
    int32_t graph_steps;     /* steps per captured HIP graph (even), 0 = no graph */
} bte_tuning;

typedef struct {
    int64_t step;        /* whole-grid step k of the current state */
    double t;            /* k dt */
    double v_dr;         /* pi sqrt(alpha) dphi sum_m b_1(m) at step k */
    double norm;         /* 2 pi sqrt(alpha) dphi sum_m a_0(m) at step k */
    int64_t n_avg;       /* steps accumulated in the current window */
    double S_v;          /* sum of v_dr over the window */
    double S_vc;         /* sum of v_dr cos(w t) over the window */
    double v_avg;        /* S_v / n_avg (0 if n_avg = 0) */
    double absorption;   /* (2 I_0(mu)/I_1(mu)) S_vc / n_avg  (Sec. 2 absorption) */
    double S_c;          /* sum of cos(w t) over the window's steps */
    double absorption_cov; /* (2 I_0/I_1) (S_vc - v_avg S_c) / n_avg: the same
                            average with the mean of v taken out, which removes
                            the leak of the dc drift into a window that is not
                            a whole number of periods (identical on exact
                            periods, where S_c = 0) */
    /* Resolution diagnostics of the whole grid at step k.  Both should stay
       small; when they do not, the phi_y box or the harmonic count is too
       small for the run. */
    double edge_mass;    /* the Sec. 2 normalisation integral 2 pi sqrt(alpha) dphi
                            sum |a_0(m)| taken over the outer max(1, ceil(N_y/64))
                            phi_y points at each end of the box */
    double top_harm_mass;/* share of the integral of f^2 over the Brillouin zone and
                            the box (Parseval: 2 a_0^2 + sum_{n>=1} a_n^2 + b_n^2,
                            summed over phi_y) held by the top max(1, N_x/8)
                            harmonics */
    int32_t status;      /* BTE_OK or BTE_EUNSTABLE */
    int32_t reserved;
} bte_obs;

typedef struct bte_solver bte_solver;

/* Device bytes a solver with this grid and parameters needs.  Validates the
   arguments the same way bte_create does (BTE_EINVAL also for a grid whose
   set of four state planes would reach 2 GiB: the step kernels address a
   set with 32-bit byte offsets). */
bte_status bte_workspace_bytes(const bte_grid* grid, const bte_params* params, size_t* bytes);

/* Create a solver: lay out the workspace, set the whole grid to the
   equilibrium a_n = a^(0)_n, b_n = 0 (Sec. 2 initial condition) and compute
   the fractional grid by the start-up half-step z^{1/2} = T(z^0) with time
   step dt/2 (Sec. 3).  The step counter starts at 0 and the averaging window
   is empty.  `workspace` is a device pointer of at least
   bte_workspace_bytes() bytes (256-byte aligned) or NULL; `hip_stream` is a
   hipStream_t or NULL. */
bte_status bte_create(const bte_grid* grid, const bte_params* params, void* workspace,
                      size_t workspace_bytes, void* hip_stream, bte_solver** out);

/* Advance n_steps >= 0 whole steps (Sec. 3 leap-frog: whole grid k -> k+1
   with coupling from the fractional grid, then fractional k+1/2 -> k+3/2
   with coupling from the new whole grid).  Steps whose new index k+1 lies in
   the averaging window add b_1(m) and b_1(m) cos(w (k+1) dt) to FP64
   per-phi_y accumulators.  Queues work only.
   Stability: after every captured run of steps (each graph replay) and every
   run of direct launches, the device checks the state's norm and drift
   velocity and, when either is not finite or the norm lies further from
   its equilibrium value (that of f0) than the initial state's norm did by
   more than 1e-2 of it (the norm-deviation bound reported in the paper's
   Sec. 4; relaxation alone moves the norm monotonically toward f0's, so a
   resolved run never exceeds this), sets a sticky flag in host-visible
   memory.  Every later
   bte_step reads that flag without synchronising and returns BTE_EUNSTABLE,
   queueing nothing, once the device has set it; bte_set_state clears it. */
bte_status bte_step(bte_solver* s, int64_t n_steps);

/* Set the averaging window to steps k with lo < k <= hi and clear the
   accumulators.  Steps already taken are not re-counted. */
bte_status bte_set_window(bte_solver* s, int64_t lo, int64_t hi);

/* Reduce and return the observables of the current state (synchronises).
   Flags the handle unstable (status BTE_EUNSTABLE, sticky) when an
   observable or the state's f^2 integral is not finite or the norm lies
   further from f0's norm than the initial state's did by more than 1e-2 of
   f0's norm. */
bte_status bte_observables(bte_solver* s, bte_obs* out);

/* Copy the state out as four [N_x][N_y] FP64 host arrays (whole grid a, b at
   step k; fractional grid a, b at k + 1/2).  Any pointer may be NULL. */
bte_status bte_get_state(bte_solver* s, double* a_h, double* b_h, double* a_f, double* b_f);

/* Replace the state.  With a_f and b_f given, the four arrays become the
   state at whole step `step` (a resume).  With a_f = b_f = NULL, (a_h, b_h)
   becomes the state at step 0 and the fractional grid is recomputed by the
   start-up half-step.  Row b[0] is ignored (b_0 is zero).  Clears the
   accumulators and the unstable flag. */
bte_status bte_set_state(bte_solver* s, const double* a_h, const double* b_h,
                         const double* a_f, const double* b_f, int64_t step);

/* Set or read the launch shape of the step kernels. */
bte_status bte_set_tuning(bte_solver* s, const bte_tuning* t);
bte_status bte_get_tuning(const bte_solver* s, bte_tuning* t);

/* Autotuner: pick the launch shape by measurement.  Builds a scratch solver
   for (grid, params) on `workspace` (bte_workspace_bytes of them; its contents
   are overwritten), times each candidate shape -- kernel form (`kernel_form`
   = a bte_kernel value, or -1 for all), 2..62 harmonics per wavefront, 1..8
   wavefronts per block -- for about `target_ms` milliseconds (<= 0: 2 ms)
   with HIP events on `hip_stream`, and writes the fastest to *best and its
   time per step to *best_us_per_step (may be NULL).  The paper tunes its
   kernels' block and grid sizes by hand (Sec. 7); this does it per grid.
   Synchronises the stream. */
bte_status bte_tune(const bte_grid* grid, const bte_params* params, void* workspace,
                    size_t workspace_bytes, void* hip_stream, int32_t kernel_form,
                    double target_ms, bte_tuning* best, double* best_us_per_step);

/* ------------------------------------------------------------------------ */
/* The distribution function itself                                         */
/* ------------------------------------------------------------------------ */
/* f(phi_x, phi_y) from Fourier coefficients (Sec. 2, Eq. f_fourier), on the
   uniform phi_x grid x_j = -pi + 2 pi j / n_phix, j = 0 .. n_phix-1 (the
   first Brillouin zone, right end excluded) at every phi_y point:

       out[j * n_y + m] = sum_{n < N_x} a_n(m) cos(n x_j) + b_n(m) sin(n x_j).

   `out` is a device array of n_phix * n_y doubles, owned by the caller and
   fully overwritten (rows are phi_x samples, phi_y contiguous).  Direct sum in
   FP64; every term's angle is reduced exactly from the integer phase
   (n j mod n_phix) / n_phix.  Any n_phix >= 1 is accepted (n_phix < 2 N_x
   samples alias harmonics, as any sampling does).  Queued on the stream;
   nothing is synchronised or allocated.
   Errors: BTE_EINVAL for NULL pointers, a misaligned `out` (8 bytes),
   n_phix outside 1 .. 2^20, or bad sizes. */

/* The solver's whole-grid state (step k).  FP32-bulk solvers' coefficients
   are widened to FP64.  Queued on the solver's stream after all work queued
   before it. */
bte_status bte_reconstruct(bte_solver* s, int32_t n_phix, double* out);

/* Caller coefficients: device arrays a and b of N_x rows of `ld` >= n_y
   doubles each (row n holds a_n or b_n at m = 0 .. n_y-1); row 0 of b is
   not read (b_0 = 0).  Queued on `hip_stream` (a hipStream_t, or NULL). */
bte_status bte_reconstruct_coeffs(const double* a, const double* b, int32_t n_x, int32_t n_y,
                                  int64_t ld, int32_t n_phix, double* out, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Observables of a state the caller holds                                  */
/* ------------------------------------------------------------------------ */
/* Device bytes of scratch bte_state_observables needs for n_x harmonics
   (partial sums, one row of three per harmonic plus a few).  BTE_EINVAL for
   n_x outside 2..16384. */
bte_status bte_state_observables_bytes(int32_t n_x, size_t* bytes);

/* The Sec. 2 observables of a whole-grid state in caller device arrays a and
   b (N_x rows of `ld` >= n_y doubles each; row n holds a_n or b_n at
   m = 0 .. n_y-1; row 0 of b is not read), on the grid phi_y(m) = phiy_min +
   m dphi, dphi = (phiy_max - phiy_min)/(n_y - 1):
       out[0] = norm = 2 pi sqrt(alpha) dphi sum_m a_0(m)
       out[1] = v_dr = pi sqrt(alpha) dphi sum_m b_1(m)
       out[2] = edge_mass, out[3] = top_harm_mass (as in bte_obs).
   `out` is a device array of 4 doubles.  The sums run in a fixed order (the
   result does not depend on timing).  `workspace` is device scratch of at
   least bte_state_observables_bytes(n_x) bytes, 256-byte aligned, that the
   call overwrites; queued on `hip_stream` (a hipStream_t or NULL) with no
   synchronisation.  A NULL workspace makes the call allocate and free one,
   synchronising the stream before and after.  Errors: BTE_EINVAL for NULL or
   misaligned pointers or bad sizes (n_y < 3, ld < n_y, alpha <= 0, phiy_max
   <= phiy_min), BTE_ENOMEM for a short workspace. */
bte_status bte_state_observables(const double* a, const double* b, int32_t n_x, int32_t n_y,
                                 int64_t ld, double phiy_min, double phiy_max, double alpha,
                                 void* workspace, size_t workspace_bytes, void* hip_stream,
                                 double* out);

/* bte_state_observables for callers that cannot allocate (code under HIP
   graph capture, serving loops, harnesses that forbid hipMalloc): the same
   kernels and results, with the scratch taken from a static device array of
   the library (about 385 KiB per GPU, held until the process ends) instead of
   a workspace argument.  Accepts n_x up to BTE_STATE_OBS_NOALLOC_MAX_NX
   (BTE_EINVAL beyond it) and otherwise the arguments and errors of
   bte_state_observables.  a, b, out and hip_stream must belong to the
   current device.  Queued on `hip_stream` with no synchronisation; calls no
   hipMalloc or hipFree.  Every call on one GPU shares that GPU's array and
   overwrites it entirely before reading it, so calls that overlap on one GPU
   (two streams, or two host threads) race and may return wrong sums;
   serialise them, e.g. on one stream. */
#define BTE_STATE_OBS_NOALLOC_MAX_NX 16384
bte_status bte_state_observables_noalloc(const double* a, const double* b, int32_t n_x,
                                         int32_t n_y, int64_t ld, double phiy_min,
                                         double phiy_max, double alpha, void* hip_stream,
                                         double* out);

/* ------------------------------------------------------------------------ */
/* Batched parameter sweeps                                                  */
/* ------------------------------------------------------------------------ */
/* Many independent instances (each its own fields, temperature and phi_y
   resolution) share the harmonic count, the phi_y box, dt and the precision.
   Every instance starts from the equilibrium (or a warm start), runs whole
   ac periods of T = 2 pi / omega, and stops when the absorption of two
   consecutive periods differs by less than `tol` (after at least
   `min_periods`), or after `max_periods`.  With L = round(T/dt) steps per
   period, period p covers the steps (p-1) L < k <= p L (windows of one
   length: a window of whole steps misses T by up to half a step, and equal
   windows keep that error the same from period to period instead of
   alternating); its absorption A_p and mean drift velocity follow the Sec. 2
   definitions over those steps.  Two schedules run the same per-cell
   arithmetic as the single-instance solver (bte_batch_schedule): the wide
   one (default) advances all running instances together, one launch per pass
   of one or two steps; the persistent one runs the whole sweep in one
   graph-captured launch in which each workgroup takes the next instance from
   a device work queue (largest expected cost first). */

typedef struct {
    double E_dc, E_w, omega, B, mu;   /* as in bte_params; omega > 0 */
    int32_t n_y;                       /* phi_y points of this instance, >= 3 */
    int32_t reserved;                  /* must be 0 */
} bte_instance;

typedef struct {
    int32_t n_x;            /* harmonics, shared, >= 2 */
    int32_t precision;      /* bte_precision */
    double phiy_min, phiy_max;
    double dt;              /* time step (tau = 1) */
    double alpha;           /* normalisation of f0 and v_dr, > 0 */
    double tol;             /* absolute |A_p - A_{p-1}| threshold, > 0 */
    int32_t min_periods;    /* >= 2 */
    int32_t max_periods;    /* >= min_periods */
    int32_t confirm;        /* consecutive periods that must each change A by less than
                               tol before an instance stops (>= 1; 1 = the single test) */
    int32_t reserved;       /* must be 0 */
} bte_batch_config;

/* How a batch is laid out on the GPU. */
typedef enum {
    /* One persistent launch; each workgroup takes the next instance from a
       device work queue and runs it to convergence.  Device memory: one state
       slot per workgroup.  A batch of few long instances runs at one
       workgroup per instance. */
    BTE_BATCH_PERSISTENT = 0,
    /* Every instance has its own state slot; each pass is one launch over the
       tiles of all instances still running (one or two steps each), followed
       by a bookkeeping launch that closes periods and sizes the next pass.
       The host replays captured groups of passes until no instance is left.
       Same per-cell arithmetic, step sequence and reductions as the
       persistent schedule: identical results. */
    BTE_BATCH_WIDE = 1
} bte_batch_schedule;

typedef struct {
    int32_t kernel;         /* BTE_KERNEL_FUSED or BTE_KERNEL_FUSED2 */
    int32_t rows_per_wave;  /* 1 .. 62 (58 for FUSED2) */
    int32_t waves_per_group;/* wavefronts per workgroup: 2, 4 or 8 */
    int32_t groups;         /* persistent workgroups (0: fill the GPU) */
    int32_t schedule;       /* a bte_batch_schedule */
} bte_batch_tuning;

typedef struct {
    double absorption;      /* A_p of the last period run: (2 I_0/I_1) times the
                               mean over the period's steps of (v - <v>) cos(w t)
                               (Sec. 2 absorption; the mean of v is taken out
                               because a period of whole steps is not exactly
                               2 pi / w long, as bte_obs.absorption_cov) */
    double v_avg;           /* mean drift velocity of that period */
    double dA;              /* |A_p - A_{p-1}| of that period (0 if p = 1) */
    int64_t steps;          /* whole steps taken */
    int32_t periods;        /* periods completed */
    int32_t converged;      /* 1 if dA < tol with p >= min_periods */
    int32_t status;         /* BTE_OK, or BTE_EUNSTABLE for a non-finite observable */
    int32_t reserved;
} bte_result;

typedef struct bte_batch bte_batch;

/* Device bytes for a batch (instance tables, state slots sized for the
   largest n_y -- one per workgroup, or one per instance for the wide
   schedule --, results), for the given tuning.  NULL tuning: FUSED2, 58
   harmonics per wave, 4 wavefronts per group, and the wide schedule unless
   its slots would take more than 64 GiB (then the persistent one).
   BTE_EINVAL as bte_batch_create, including a largest grid whose set of four
   state planes would reach 2 GiB. */
bte_status bte_batch_workspace_bytes(const bte_batch_config* cfg, int32_t n,
                                     const bte_instance* inst, const bte_batch_tuning* tuning,
                                     size_t* bytes);

/* Create a batch of n instances.  Host tables are copied; the workspace
   follows the same ownership rules as bte_create (NULL: library-allocated). */
bte_status bte_batch_create(const bte_batch_config* cfg, int32_t n, const bte_instance* inst,
                            const bte_batch_tuning* tuning, void* workspace,
                            size_t workspace_bytes, void* hip_stream, bte_batch** out);

/* Warm start: a device array of n x 64 x 128 floats (instance-major).  For
   instance i, rows 0..31 hold a_n - a^(0)_n (n = 0..31) and rows 32..63 hold
   b_n (n = 1..32), each sampled at 128 uniform points phi_min + j (phi_max -
   phi_min)/127 of the box.  Instances start from the state linearly
   interpolated back to their phi_y grid (harmonics >= 32 from the
   equilibrium) instead of f0, at t = 0 (phase 0 of the field); the start-up
   half-step then derives the fractional grid.  NULL restores the equilibrium
   start.  The array must stay valid until the next bte_batch_run completes. */
bte_status bte_batch_set_warm_start(bte_batch* b, const float* dev_coeffs);

/* State output: a device array of n x 64 x 128 floats that each run fills
   with every instance's whole-grid state at the end of its last period
   (phase 0 of the field), in the warm-start encoding above.  NULL: none. */
bte_status bte_batch_set_state_output(bte_batch* b, float* dev_coeffs);

/* Run the sweep.  Persistent schedule: queue it (one graph launch) and
   return immediately.  Wide schedule: set up, then replay groups of passes
   until every instance has stopped, synchronising the stream after each group;
   returns when the sweep is done (bte_batch_advance does the same in slices). */
bte_status bte_batch_run(bte_batch* b);

/* Wide schedule only: advance the sweep by at most `max_replays` >= 1 groups
   of passes (64 passes each), starting it first (set-up from the equilibrium
   or the warm start) when no sweep is in progress.  Synchronises the stream
   after each group and writes the number of instances still running to
   *remaining (host pointer); 0 means the sweep is done and its results are
   readable.  BTE_ESTATE for the persistent schedule; BTE_EDEVICE if the
   sweep exceeds the pass count that max_periods allows (it cannot). */
bte_status bte_batch_advance(bte_batch* b, int32_t max_replays, int32_t* remaining);

/* Wait for the sweep and copy the n results out (synchronises). */
bte_status bte_batch_results(bte_batch* b, bte_result* out);

/* Tuning of the batch kernel (takes effect at the next run). */
bte_status bte_batch_get_tuning(const bte_batch* b, bte_batch_tuning* t);

void bte_batch_destroy(bte_batch* b);

/* Sweep autotuner: pick the batch's tile (kernel form FUSED2 or FUSED,
   harmonics per wave among the values that split n_x into 1 to 8 equal
   chunks, wavefronts per group 2, 4 or 8; wide schedule) by measurement.
   The cost per step of an instance depends only on its grid, so the tuner
   runs samples whose N_y values follow the batch's share of cells, each
   instance with omega raised to periods of 400 steps and run for exactly
   two periods (a fixed amount of work), on `hip_stream`, timing the second
   of two runs (the first captures the graphs).  Stage one times every
   candidate on up to 128 instances; when the batch is larger, stage two
   re-times the three fastest on as many instances as the batch holds (at
   most 4096) and keeps the fastest there.  Neither sample takes more state
   slots than fit in 64 GiB (the wide schedule's default budget).  The
   library allocates and frees the samples' device memory itself.  With use_cache != 0 an earlier result for
   the same (n_x, set of N_y values, precision, batch-size class: the
   smallest power of two >= min(n, 4096)) in this process is returned
   without measuring.  *out receives the tuning; *cell_steps_per_s (may be
   NULL) the deciding sample's rate in cell-steps per second.  Errors as
   bte_batch_create. */
bte_status bte_batch_tune(const bte_batch_config* cfg, int32_t n, const bte_instance* inst,
                          void* hip_stream, int32_t use_cache, bte_batch_tuning* out,
                          double* cell_steps_per_s);

/* The sweep's stopping rule on one solver: run whole ac periods of
   L = round(2 pi / (omega dt)) steps from the current step k0 (period p
   covers k0 + (p-1) L < k <= k0 + p L; k0 = 0 starts at phase 0 of the
   field), take each period's absorption as bte_obs.absorption_cov over it,
   and stop when `confirm` consecutive periods each change it by less than
   `tol` (absolute, with p >= min_periods >= 2) or after max_periods periods.
   The averaging window is reset for every period.  Fills *out as
   bte_batch_results does (steps: whole steps taken by this call); an
   unstable run ends with out->status = BTE_EUNSTABLE and BTE_OK returned.
   Synchronises once per period.  BTE_EINVAL for omega = 0 or bad limits. */
bte_status bte_run_periods(bte_solver* s, double tol, int32_t min_periods, int32_t max_periods,
                           int32_t confirm, bte_result* out);

/* Destroy the handle; frees what the library allocated.  NULL is a no-op. */
void bte_destroy(bte_solver* s);

/* Plain device copy of `bytes` from src to dst (both 16-byte aligned, not
   overlapping, bytes a multiple of 16), queued on `hip_stream`.  Not part of
   the method: the read+write streaming rate it reaches (one 16 KiB run per
   workgroup, non-temporal loads and stores) is the practical HBM ceiling the
   step kernels are measured against.  BTE_EINVAL for bad pointers or
   sizes. */
bte_status bte_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Message of the last failing call on this thread ("" if none). */
const char* bte_last_error(void);

/* Library version string. */
const char* bte_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BTE_H */
