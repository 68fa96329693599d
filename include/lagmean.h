/*
 * lagmean.h - C ABI of the MI355X (gfx950) Lagrangian-mean library.
 *
 * The library advances the doubly periodic rotating shallow-water equations
 * pseudospectrally and, in the same classical RK4 stages, integrates the
 * Lagrangian-mean PDEs of Kafiabad & Vanneste, "Computing Lagrangian means":
 *
 *   strategy 1 (section 3.1; numerics section 4.1): the partial mean f~ in the
 *     form g~ = (t - tau) f~, eq. (4.1) (from eq. (3.5)), and the inverse lift
 *     map Xi^{-1} of eq. (3.9), carried as P = (t - tau)(x - Xi^{-1});
 *   strategy 2 (section 3.2; numerics section 4.2): the displacement
 *     xi = Xi - x and g-bar = (t - tau) f-bar, eqs. (4.5a,b), with periodic
 *     bilinear interpolation of u and f at x + xi;
 *   the Eulerian mean, for comparison;
 *
 * over successive averaging intervals (tau, tau + T) (section 3, the
 * paragraph after eq. (3.3): each interval is independent).  The averaged
 * fields are the total depth h and the vorticity zeta = dv/dx - du/dy.
 *
 * Dynamics (section 4.2, eq. (4.6), in dimensional vector-invariant form):
 *   du/dt = zeta v + f v - d(K + g h)/dx - nu8 |k|^8 u,
 *   dv/dt = -zeta u - f u - d(K + g h)/dy - nu8 |k|^8 v,
 *   dh/dt = -div(h u) - nu8 |k|^8 h,         K = (u^2 + v^2)/2,
 * on [0, 2 pi)^2 with the 2/3-rule square mask |kx|, |ky| <= floor((N-1)/3)
 * applied to the state and to every right-hand side (sections 4.1, 4.2.1).
 * At t = tau, where xi/(t - tau) is 0/0, the partial-mean velocity takes its
 * limit u/2.
 *
 * Conventions shared by every entry point:
 *   - Physical arrays are N x N float64, row-major [iy][ix], x_i = 2 pi i / N,
 *     for both precisions.
 *   - Pointers flagged on_device = 1 are HIP device pointers, otherwise host
 *     pointers.  The caller owns them; the library copies and never retains them.
 *   - Every call returns an lm_status; nothing throws across the ABI.  After an
 *     error, lm_last_error() (thread-local) describes it and the run is left as
 *     it was before the call, except for LM_E_HIP (device state is then undefined).
 *   - A run is driven by one thread at a time; distinct runs may be driven
 *     from different threads.  All device work of a run is ordered on the HIP
 *     stream given to lm_create (0 = the null stream).
 */
#ifndef LAGMEAN_H
#define LAGMEAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LM_OK = 0,
  LM_E_ARG = -1,         /* bad argument (null pointer, out-of-range value) */
  LM_E_STATE = -2,       /* call out of order (e.g. end_interval with no steps) */
  LM_E_OOM = -3,         /* device allocation failed */
  LM_E_HIP = -4,         /* a HIP runtime call failed */
  LM_E_NONFINITE = -5,   /* a NaN or Inf reached the interval outputs */
  LM_E_UNSUPPORTED = -6, /* configuration not implemented (N, mode, ...) */
  LM_E_BUDGET = -7       /* footprint exceeds a caller-given budget */
} lm_status;

typedef enum { LM_FP64 = 0, LM_FP32_MIXED = 1 } lm_precision;

/* averaged fields (bit mask).  Two scalar fields are averaged, by default h and
   zeta; any other two of the five below may be chosen instead (the tests use
   u, v and the potential vorticity q, which is materially conserved without
   dissipation: section 4.1, eq. (4.2), and the potential-vorticity argument of
   section 4.2.1).  The two fields fill the output slots field = 0 and 1 in the
   order of their bits (lowest first).  On request strategy 2 also averages the
   momentum 1-form u . dx (appendix C). */
#define LM_F_H 1u
#define LM_F_ZETA 2u
#define LM_F_MOMENTUM 4u
#define LM_F_U 8u
#define LM_F_V 16u
#define LM_F_Q 32u /* (f + zeta) / h */
/* strategies (bit mask); the library always integrates all three */
#define LM_S1 1u
#define LM_S2 2u
#define LM_EULER 4u
/* gather interpolation of strategy 2 (u and the averaged fields at x + xi) */
#define LM_INTERP_BILINEAR 0 /* periodic bilinear, as section 4.2.1 */
#define LM_INTERP_CUBIC 1    /* periodic tensor-product cubic (4-point Lagrange, 4 x 4
                                points; the paper compares linear and cubic
                                interpolation for strategy 1, section 4.1) */
/* driver of u, v, h */
#define LM_DYNAMIC 0              /* the rotating shallow-water equations */
#define LM_KINEMATIC_PLANEWAVE 1  /* prescribed, for tests: a linear Poincare plane
                                     wave plus a uniform flow (kin[] below) */

typedef struct {
  int32_t n;           /* grid points per side: 64, 128, 192, 256, 384, 512 or 1024 */
  int32_t precision;   /* LM_FP64: everything float64.  LM_FP32_MIXED: transforms,
                          products, gathers and RK4 accumulators in float32; the other
                          prognostic state (u, v, h and the g-bar, g-tilde and Eulerian
                          accumulators) as compensated float32 pairs (a leading and a
                          trailing word, renormalised at each step's update); the xi and
                          P state, their RK4 accumulators and the end-of-interval outputs
                          (division by T included) in float64 */
  double f, g, H;      /* Coriolis parameter, gravity, mean depth */
  double dt;           /* time step (shared by dynamics and mean PDEs) */
  double nu8;          /* eighth-order hyperviscosity on u, v, h (>= 0) */
  uint32_t avg_fields; /* two of LM_F_H, LM_F_ZETA, LM_F_U, LM_F_V, LM_F_Q (0: LM_F_H | LM_F_ZETA),
                          optionally | LM_F_MOMENTUM.  Averaging fields other than
                          (h, zeta) takes two more forward transforms per stage for
                          their Eulerian means.  LM_F_MOMENTUM:
                          strategy 2 also integrates the mean of the momentum 1-form,
                          eq. (C.4) in the g-bar form of eq. (4.5b):
                          dg_i/dt + w_j d_j g_i + g_j d_i w_j = u_j(x + xi)(delta_ij + d_i xi_j)
                          (two more prognostic fields, two more row tasks and
                          column groups; a larger footprint) */
  uint32_t strategies; /* must be LM_S1 | LM_S2 | LM_EULER (or 0 for the default) */
  int32_t interp;      /* LM_INTERP_BILINEAR or LM_INTERP_CUBIC */
  int32_t mode;        /* LM_DYNAMIC or LM_KINEMATIC_PLANEWAVE */
  double kin[8];       /* LM_KINEMATIC_PLANEWAVE only (ignored otherwise): the prescribed
                          flow at time t (t = 0 at lm_create, steps * dt after) is
                            h = H + A cos(theta), theta = kx x + ky y - omega t + phase,
                            u = U0 + A (omega kx cos(theta) - f ky sin(theta)) / (H |k|^2),
                            v = V0 + A (omega ky cos(theta) + f kx sin(theta)) / (H |k|^2),
                          the linear plane wave of section 4.2.1, eq. (4.8), in any
                          direction; for A < H the particle phase obeys an Adler
                          equation with a real frequency, and over whole periods of it
                          the Lagrangian means are constants known in closed form.
                          kin = {kx, ky, A, omega (0: the dispersion relation
                          omega^2 = f^2 + g H |k|^2), phase, U0, V0, unused}.  kx, ky
                          integers inside the 2/3-rule mask (else LM_E_ARG); A = 0 gives
                          the uniform flow alone.  Such a run has no lm_set_state
                          (LM_E_STATE); its state is defined from lm_create on, and
                          lm_get_state returns the prescribed u, v, h at the current time */
} lm_config;

typedef struct lm_run lm_run;

/* Device bytes lm_create would allocate for this configuration.  Host only,
   allocates nothing.  LM_E_UNSUPPORTED / LM_E_ARG as lm_create. */
lm_status lm_query_footprint(const lm_config* cfg, size_t* bytes);

/* Create a run: validates cfg, allocates all device buffers of the run (one
   allocation), builds twiddle tables.  hip_stream: a hipStream_t (may be 0).
   The state is undefined until lm_set_state.  *out receives the handle. */
lm_status lm_create(const lm_config* cfg, void* hip_stream, lm_run** out);

/* Set the dynamical state from physical u, v, h (h = total depth), each N x N
   float64.  The fields are transformed and truncated to the 2/3-rule mask.
   Resets the step counter to 0; the averaging state is cleared and no interval
   is open.  Synchronous with respect to the caller's buffers. */
lm_status lm_set_state(lm_run* run, const double* u, const double* v, const double* h, int on_device);

/* Physical u, v, h of the current (masked) state, N x N float64 each.  Synchronous. */
lm_status lm_get_state(lm_run* run, double* u, double* v, double* h, int on_device);

/* Open an averaging interval at the current time: tau := t, and zero the
   strategy-1, strategy-2 and Eulerian state (their initial conditions: section
   3.2 and eq. (4.1): g = 0, xi = 0, P = 0).  LM_E_STATE before lm_set_state. */
lm_status lm_begin_interval(lm_run* run);

/* Advance nsteps >= 0 RK4 steps.  Asynchronous on the run's stream.
   LM_E_STATE before lm_set_state. */
lm_status lm_step(lm_run* run, int32_t nsteps);

/* As lm_step, but every kernel launch is bracketed by a pair of HIP events on
   the run's stream (all enqueued back to back; one synchronisation at the end).
   ms_avg[0..2] receive the average duration in milliseconds of the three
   hot-path kernels: [0] rows pass of the dynamics, [1] rows pass of the mean
   right-hand sides, [2] column pass (spectral assembly + RK4).
   1 <= nsteps <= 4096.  Synchronous.  For measurement. */
lm_status lm_step_profiled(lm_run* run, int32_t nsteps, double* ms_avg);

/* As lm_step, with a pair of HIP events on the run's stream around the steps:
   *ms receives their elapsed time in milliseconds.  Synchronous.  For
   measurement. */
lm_status lm_step_timed(lm_run* run, int32_t nsteps, double* ms);

/* Close the interval: T = (steps since begin) * dt; computes the outputs
   (section 4.1: f~^L = g~/T, eta = P/T; section 4.2: f-bar^L = g-bar/T and xi;
   Eulerian mean E/T) in float64 and synchronises the stream.  LM_E_STATE if no
   interval is open or it holds no step; LM_E_NONFINITE if any output is NaN or
   Inf (outputs are still readable).  *T_out (may be null) receives T. */
lm_status lm_end_interval(lm_run* run, double* T_out);

/* output kinds for lm_read_mean */
typedef enum {
  LM_K_S2_MEAN = 0,   /* strategy 2: f-bar^L at Lagrangian-mean positions (field) */
  LM_K_S2_XI_X = 1,   /* strategy 2: xi_x = Xi_x(x, tau+T) - x               */
  LM_K_S2_XI_Y = 2,   /* strategy 2: xi_y                                   */
  LM_K_S1_MEAN = 3,   /* strategy 1: f~^L at end-of-interval positions (field) */
  LM_K_S1_ETA_X = 4,  /* strategy 1: eta_x = x - Xi^{-1}_x(x, tau+T)          */
  LM_K_S1_ETA_Y = 5,  /* strategy 1: eta_y                                  */
  LM_K_EULER_MEAN = 6, /* Eulerian time mean (field)                        */
  LM_K_S1_REMAP_MEAN = 7, /* strategy 1 remapped: f-bar^L at Lagrangian-mean
                             positions (field), after lm_remap_s1             */
  LM_K_S1_REMAP_XI_X = 8, /* strategy 1 remapped: Xi_x(y) - y, the end position
                             minus the mean position, as xi_x of strategy 2   */
  LM_K_S1_REMAP_XI_Y = 9, /* strategy 1 remapped: Xi_y(y) - y                 */
  LM_K_S2_MOM_X = 10,     /* strategy 2: the mean of the momentum 1-form at
                             Lagrangian-mean positions, x component (runs
                             created with LM_F_MOMENTUM; else LM_E_STATE)     */
  LM_K_S2_MOM_Y = 11      /* same, y component                               */
} lm_kind;
/* output slot of a scalar averaged field: the first (lowest bit) or second of
   the two averaged fields; with the default fields, h and zeta */
typedef enum { LM_FIELD_H = 0, LM_FIELD_ZETA = 1, LM_FIELD_FIRST = 0, LM_FIELD_SECOND = 1 } lm_field;

/* Remap the strategy-1 outputs of the last closed interval to Lagrangian-mean
   positions (section 3.1, eq. (3.8): f~^L(x) = f-bar^L(Xi^{-1}(x))).  For every
   grid point y, taken as a mean position, the end position x of its particle
   solves x - eta(x) = y (eta = x - Xi^{-1}(x) from strategy 1, bilinear between
   grid values, as the gathers of section 4.2.1); then f-bar^L(y) = f~^L(x)
   (bilinear) and the displacement Xi(y) - y = x - y.  Solved exactly per
   end-position cell: the cell's corner mean positions span a bilinear patch,
   and every grid point the patch covers is located by inverting the patch
   (closed form, then two Newton steps); no iteration that could fail to
   contract where mean positions cluster (the paper's caveat, section 5).  Where
   the mean map folds (a point covered by several patches) the patch of the
   lowest cell index iy N + ix is taken.  Patches spanning more than max_extent
   grid cells in x or y are skipped; a point no patch covers gets NaN.
   float64.  1 <= max_extent <= 64 (else LM_E_ARG); LM_E_STATE before the
   first lm_end_interval or while the run belongs to a batch.  *residual (may be
   null) receives the largest |p(s, t) - y| over all points in grid spacings
   (inversion error; infinite if some point is not covered).  The results are
   read with lm_read_mean kinds LM_K_S1_REMAP_*, until the next
   lm_end_interval.  Uses the run's boundary staging buffer.  Synchronous. */
lm_status lm_remap_s1(lm_run* run, int32_t max_extent, double* residual);

/* Copy one output of the last closed interval (N x N float64) to out.
   field is ignored for the displacement kinds.  LM_E_STATE before the first
   lm_end_interval, and for the LM_K_S1_REMAP_* kinds before lm_remap_s1 of
   that interval.  Synchronous. */
lm_status lm_read_mean(lm_run* run, int32_t field, int32_t kind, double* out, int on_device);

/* raw prognostic fields for lm_peek */
typedef enum {
  LM_P_U = 0, LM_P_V, LM_P_H, LM_P_GBAR_H, LM_P_GBAR_ZETA, LM_P_GTIL_H, LM_P_GTIL_ZETA,
  LM_P_E_H, LM_P_E_ZETA, LM_P_XI_X, LM_P_XI_Y, LM_P_P_X, LM_P_P_Y
} lm_peek_field;

/* Physical value of one raw prognostic field of the current state (e.g.
   g-bar = (t - tau) f-bar undivided), N x N float64.  The accumulators of h
   (LM_P_GBAR_H, LM_P_GTIL_H, LM_P_E_H) integrate the anomaly h - H.
   Synchronous.  For tests. */
lm_status lm_peek(lm_run* run, int32_t which, double* out, int on_device);

/* Checkpoint and resume, also in the middle of an averaging interval (each
   interval is independent of the others, section 3, the paragraph after eq.
   (3.3), but within one interval the partial means, xi and P accumulate from
   tau on, so resuming mid-interval needs them).  A checkpoint holds the whole
   state between two steps: every prognostic field as stored (dynamics, the
   strategy-1, strategy-2 and Eulerian accumulators, xi and P; both words of
   compensated float32 fields), the step counters and whether an interval is
   open, behind a header naming the configuration.  lm_restore into a run of
   the same configuration continues exactly as the saved run would have, bit
   for bit (the RK4 accumulators are rewritten by the first stage of a step, and
   the inputs of the next rows passes are transformed from the state by the same
   kernels the last step's final column pass uses).  The outputs of a closed
   interval are not part of it.
     lm_checkpoint_size: bytes a checkpoint of this run takes (host only).
     lm_save: write the checkpoint to buf (cap bytes, at least the size), a host
       or device pointer.  LM_E_STATE without a state or inside a batch.
     lm_restore: take the state from a checkpoint of size bytes.  LM_E_ARG for a
       buffer that is not a checkpoint, is truncated, or was taken with any other
       configuration (grid, precision, physics, fields, gathers, driver).
       LM_E_STATE inside a batch.
   Synchronous. */
lm_status lm_checkpoint_size(const lm_run* run, size_t* bytes);
lm_status lm_save(lm_run* run, void* buf, size_t cap, int on_device);
lm_status lm_restore(lm_run* run, const void* buf, size_t size, int on_device);

/* Steps taken since lm_set_state and since lm_begin_interval. */
lm_status lm_counters(lm_run* run, int64_t* steps, int64_t* steps_in_interval);

/* Release every device buffer of the run (waits for its stream).  Null is a
   no-op.  LM_E_STATE while the run belongs to a batch. */
lm_status lm_destroy(lm_run* run);

/* ---------------------------------------------------------------------------
 * Batched form: many independent runs of any grid size and precision advanced
 * together.  One RK4 step of all active members is one captured HIP graph: per
 * (N, precision) group the three hot kernels are launched once for all the
 * group's runs (blockIdx.z selects the run), groups are parallel branches of
 * the graph.  Each member computes exactly what it computes alone (same
 * kernels, same arithmetic, no cross-run reductions), bit for bit.
 * While a run belongs to a batch, lm_set_state, lm_begin_interval, lm_step,
 * lm_step_profiled, lm_end_interval and lm_destroy return LM_E_STATE for it;
 * the reading calls stay available between lm_batch_step calls.
 * ------------------------------------------------------------------------- */
typedef struct lm_batch lm_batch;

/* Empty batch.  Its graphs are captured and launched on a stream of its own;
   lm_batch_step first waits for hip_stream (0 = the null stream). */
lm_status lm_batch_create(void* hip_stream, lm_batch** out);

/* Add a run that has a state and an open averaging interval, with a budget of
   steps >= 0 RK4 steps.  Waits for the run's own stream.  LM_E_STATE if the run
   has no open interval or already belongs to a batch. */
lm_status lm_batch_add(lm_batch* b, lm_run* run, int32_t steps);

/* Remove a member (its step counters stay as advanced). */
lm_status lm_batch_remove(lm_batch* b, lm_run* run);

/* Advance every member by min(max_steps, its remaining budget) RK4 steps.
   Synchronous.  *active (may be null) receives the number of members with
   budget left afterwards. */
lm_status lm_batch_step(lm_batch* b, int32_t max_steps, int32_t* active);

/* Allocation-free form of lm_batch_step, for callers that cannot allocate
   device memory (serving loops that must not call hipMalloc, harnesses that
   forbid it).  Same arguments, same kernels and the same results, bit for bit,
   as lm_batch_step; the difference is where the batch's bookkeeping lives: the
   member descriptors and step counters go to a fixed device array of the
   library (128 KiB, one per GPU, held until the process ends) instead of
   device memory allocated by the batch, and the steps are launched directly on
   the batch's stream instead of replaying a captured graph (which would need
   an instantiation).  The call allocates no device memory and calls no
   allocating library routine on its success path.  LM_E_BUDGET when the batch
   has more than LM_STATIC_MAX_MEMBERS members (nothing is launched then).
   Every call on one GPU shares that array: calls that overlap in time on the
   same GPU (from several threads, whatever the batch) race and must not be
   made.  Synchronous, like lm_batch_step; not for use under stream capture. */
#define LM_STATIC_MAX_MEMBERS 256
lm_status lm_batch_step_static(lm_batch* b, int32_t max_steps, int32_t* active);

/* Remaining budget of a member. */
lm_status lm_batch_remaining(lm_batch* b, const lm_run* run, int32_t* remaining);

/* Release the batch (members are removed, not destroyed).  Null is a no-op. */
lm_status lm_batch_destroy(lm_batch* b);

/* ---------------------------------------------------------------------------
 * Launch schedules and the autotuner.  The time-stepping kernels of one
 * (n, precision) can be launched in several ways that compute the same numbers
 * in the same order (results are bit-identical across schedules):
 *   col_tile   width of the column tiles of the column pass (columns per
 *              block): -1 half, 0 the default (8 columns when a transform
 *              spans at least 8 lanes), +1 twice; a width is usable when its
 *              block is whole wavefronts of at most 1024 threads and its LDS
 *              tile fits in a CU's 160 KiB;
 *   xcd_order  1: blocks renumbered so that each of the 8 XCDs (own L2)
 *              receives a contiguous range of row blocks / column tiles with
 *              all tasks of each (the default); 0: hardware dispatch order;
 *   streams    1: the three passes of an RK4 stage run in order on the run's
 *              stream (the default); 2: the stage's dependency graph runs on
 *              two streams (the run's and one of its own): the dynamics rows
 *              pass and the column groups of u, v, h on one, the mean
 *              right-hand-side rows pass and the mean column groups on the
 *              other, so that the column groups of u, v, h overlap the mean
 *              right-hand-side passes of the same stage.  Ordering with the caller is
 *              unchanged: lm_step's work still ends on the run's stream.
 *              Batched launches (captured graphs) take 1.
 * Two process-wide schedule tables, one entry per (n, precision) each: one for
 * single runs, read at every launch, and one for batched launches, read when a
 * batch captures its graph (a batch re-captures after any change of either
 * table).  The best schedule differs between the two (a single run of a small
 * grid wants more, narrower blocks; a batch fills the GPU with its runs).
 * Calls are thread-safe; changing a schedule while another thread launches the
 * same (n, precision) affects either launch or the next.
 * ------------------------------------------------------------------------- */
typedef struct lm_schedule {
  int32_t col_tile;  /* -1, 0, +1 */
  int32_t xcd_order; /* 0 or 1 */
  int32_t streams;   /* 1 or 2 (single runs; batched launches take 1) */
} lm_schedule;

/* The usable schedules of (n, precision) for single runs, the default first:
   *count receives their number (at most 12); the first min(cap, count) go to
   out (out may be null when cap is 0).  Host only. */
lm_status lm_schedule_candidates(int32_t n, int32_t precision, lm_schedule* out, int32_t cap, int32_t* count);

/* Set / read the schedule of (n, precision).  LM_E_ARG for a schedule that
   lm_schedule_candidates does not list, LM_E_UNSUPPORTED for other n.  Host only. */
lm_status lm_set_schedule(int32_t n, int32_t precision, const lm_schedule* s);
lm_status lm_get_schedule(int32_t n, int32_t precision, lm_schedule* s);
/* The same for the batched launches' table. */
lm_status lm_set_batch_schedule(int32_t n, int32_t precision, const lm_schedule* s);
lm_status lm_get_batch_schedule(int32_t n, int32_t precision, lm_schedule* s);

/* Autotune the schedule of the run's (n, precision) on the run itself: every
   candidate advances a copy of the run's current state by steps RK4 steps
   (1..64), reps times (1..16), timed with HIP events on the run's stream; the
   fastest (least of its reps) becomes the table's schedule and is written to
   *best.  ms (may be null) receives the per-step times of the first cap
   candidates in lm_schedule_candidates order, *count (may be null) their
   number.  The run's state, step counters and interval are restored exactly
   (a device copy of its whole allocation is taken and freed here, so the call
   needs that much free device memory: LM_E_OOM otherwise).  Synchronous.
   LM_E_STATE without a state or inside a batch. */
lm_status lm_autotune(lm_run* run, int32_t steps, int32_t reps, lm_schedule* best, double* ms, int32_t cap,
                      int32_t* count);

/* Autotune the batched launches' schedules on a batch's members: for each
   (n, precision) present in turn (the others at their current schedule), every
   candidate is installed, the batch graph captured and steps (1..64) graph
   launches of all members timed, reps times (1..16); the fastest stays in the
   batched table.  Every member's allocation and counters are restored exactly
   (copies of all members' allocations are taken and freed here: LM_E_OOM if
   they do not fit).  Budgets are untouched.  *tuned (may be null) receives the
   number of (n, precision) tuned.  Synchronous. */
lm_status lm_batch_autotune(lm_batch* b, int32_t steps, int32_t reps, int32_t* tuned);

/* ---------------------------------------------------------------------------
 * Two-dimensional incompressible inviscid flow with strategy 1 in two
 * discretisations: the test of the paper's section 4.1 (material conservation
 * of vorticity, eq. (4.2): zeta~^L(x, tau) = zeta(x, tau + T)) and appendix B.
 *   dynamics: dzeta/dt + (u + U0) . grad zeta = 0, u = (-dpsi/dy, dpsi/dx),
 *     lap psi = zeta; pseudospectral with the 2/3-rule square mask, Heun's
 *     method (as section 4.1), no dissipation;
 *   strategy 1 pseudospectral, in the same Heun stages: g~ = (t - tau) zeta~
 *     (eq. (4.1)) and P = (t - tau)(x - Xi^{-1}) (eq. (3.9));
 *   strategy 1 semi-Lagrangian (appendix B), after every step: departure point
 *     Y = X - dt u(X, t_{n+1}) (eq. (B.2)), trapezoidal updates (B.4) of zeta~
 *     and (B.5) of Xi^{-1}, written for eta = x - Xi^{-1}, with the gathers at Y
 *     periodic bilinear or cubic (interp).
 * float64 throughout.  Physical arrays N x N row-major as above.
 * ------------------------------------------------------------------------- */
typedef struct lm_e2d lm_e2d;
typedef struct {
  int32_t n;       /* 64, 128, 192, 256, 384, 512 or 1024 */
  double dt;       /* time step, > 0 */
  double U0, V0;   /* uniform flow added to u (0 for the paper's test) */
  int32_t interp;  /* semi-Lagrangian gathers: LM_INTERP_BILINEAR or LM_INTERP_CUBIC */
} lm_e2d_config;

/* outputs of lm_e2d_end_interval, for lm_e2d_read */
typedef enum {
  LM_E2D_ZETA = 0,      /* vorticity at the end of the interval, zeta(x, tau + T)   */
  LM_E2D_PS_MEAN = 1,   /* pseudospectral zeta~^L = g~ / T                           */
  LM_E2D_PS_ETA_X = 2,  /* pseudospectral eta = x - Xi^{-1} = P / T (x component)    */
  LM_E2D_PS_ETA_Y = 3,
  LM_E2D_SL_MEAN = 4,   /* semi-Lagrangian zeta~^L                                   */
  LM_E2D_SL_ETA_X = 5,  /* semi-Lagrangian eta                                       */
  LM_E2D_SL_ETA_Y = 6
} lm_e2d_kind;

/* Allocate a flow (one device allocation).  LM_E_UNSUPPORTED for other n or
   interp, LM_E_ARG for a non-positive or non-finite dt or non-finite U0, V0. */
lm_status lm_e2d_create(const lm_e2d_config* cfg, void* hip_stream, lm_e2d** out);
/* Set the vorticity (N x N float64; truncated to the mask).  Resets the step
   counter; no interval is open.  Synchronous. */
lm_status lm_e2d_set_vorticity(lm_e2d* e, const double* zeta, int on_device);
/* Open an averaging interval at the current time (zeroes g~, P and the
   semi-Lagrangian fields).  LM_E_STATE before lm_e2d_set_vorticity. */
lm_status lm_e2d_begin_interval(lm_e2d* e);
/* Advance nsteps >= 0 steps (dynamics, both strategy-1 forms).  Asynchronous. */
lm_status lm_e2d_step(lm_e2d* e, int32_t nsteps);
/* As lm_e2d_step with events: *ms_step = average step, *ms_sl = average
   semi-Lagrangian kernel (milliseconds).  1 <= nsteps <= 4096.  Synchronous. */
lm_status lm_e2d_step_profiled(lm_e2d* e, int32_t nsteps, double* ms_step, double* ms_sl);
/* Close the interval (T = steps * dt) and compute the LM_E2D_* outputs.
   LM_E_STATE without an open interval holding a step.  Synchronous. */
lm_status lm_e2d_end_interval(lm_e2d* e, double* T_out);
/* Copy one output (N x N float64).  LM_E_STATE before the first end. */
lm_status lm_e2d_read(lm_e2d* e, int32_t kind, double* out, int on_device);
/* Release (waits for the stream).  Null is a no-op. */
lm_status lm_e2d_destroy(lm_e2d* e);

/* Device memory and copies of the HIP runtime the library is bound to, for
   callers that hold device arrays for the on_device = 1 paths without another
   GPU framework in the process (device 0, the null stream).
     lm_device_alloc: *ptr receives bytes of device memory (null for 0 bytes);
       LM_E_OOM when they cannot be allocated.
     lm_device_free: release it (null is a no-op).
     lm_memcpy: a blocking copy of bytes; kind is one of the LM_COPY_* below.
     lm_device_synchronize: wait for all work on the device.
     lm_copy_bandwidth: the bandwidth of a plain device-to-device copy of bytes,
       reps times (1..1000) after one untimed copy, timed with HIP events;
       *gbps = 2 * bytes * reps / time (bytes read plus bytes written) / 1e9.
       Allocates and releases two buffers of bytes.  For measurement. */
#define LM_COPY_HOST_TO_DEVICE 0
#define LM_COPY_DEVICE_TO_HOST 1
#define LM_COPY_DEVICE_TO_DEVICE 2
lm_status lm_device_alloc(size_t bytes, void** ptr);
lm_status lm_device_free(void* ptr);
lm_status lm_memcpy(void* dst, const void* src, size_t bytes, int32_t kind);
lm_status lm_device_synchronize(void);
lm_status lm_copy_bandwidth(size_t bytes, int32_t reps, double* gbps);

/* HIP versions, as major * 10^7 + minor * 10^5 + patch: *built receives that of
   the HIP headers the library was compiled with, *runtime that of the HIP
   runtime this process has bound (hipRuntimeGetVersion).  The library binds the
   HIP runtime already loaded in the process when there is one (PyTorch ships
   its own copy, with the same soname); otherwise the one it was built with.
   The two may differ; callers that care compare them.  Either pointer may be
   null.  LM_E_HIP if the runtime cannot report its version. */
lm_status lm_hip_versions(int32_t* built, int32_t* runtime);

/* Text of a status code (static storage). */
const char* lm_status_str(lm_status s);
/* Last error message of the calling thread ("" if none). */
const char* lm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LAGMEAN_H */
