/*
 * cbic.h -- C ABI of the MI355X batched trajectory-optimisation solver.
 *
 * The library solves many finite-horizon discrete-time optimal control
 * problems at once, one per initial state (paper Sec. II, eq. 1):
 *
 *     min_{X,U}  sum_{k=0}^{T-1} l(x_k, u_k) + l_T(x_T)
 *     s.t.       x_{k+1} = f(x_k, u_k),  x_0 = x_init,
 *
 * with x in R^n and u in R^m, by iLQR (paper Sec. II and IV): a forward
 * rollout, analytic linearisation and quadratisation, eigenvalue clipping of
 * the state- and control-cost Hessians (Sec. IV-B, eq. 7), a backward Riccati
 * sweep with a Cholesky factorisation of Q_uu, a backtracking line search, a
 * fixed iteration budget shared by the whole batch (Sec. IV-A), and at the end
 * the critic targets of Sec. II: the K-step partial cost-to-go V-bar of every
 * state, its gradient V-bar_x from the backward (costate) pass, and the state
 * K steps later.  The control bound |u| <= u_max of eq. 1 is an option
 * (cbic_solve_opts.u_max, unbounded by default).
 *
 * Conventions for every call
 *  - Return value: CBIC_OK (0) on success, CBIC_NOT_READY (1) for a pending
 *    result, a negative cbic_status on error.  No C++ exception crosses the
 *    ABI.  cbic_last_error() returns a message for the last failing call on
 *    the calling thread (valid until that thread's next failing call).
 *  - Invalid arguments are rejected with CBIC_E_INVALID before anything is
 *    launched.  Per-instance numerical outcomes are never errors; they are
 *    reported in the per-instance status word (CBIC_ST_* bits).
 *  - Pointers named d_* are device pointers (HIP device memory of the
 *    context's GPU); pointers named h_* are host pointers.  All arrays are
 *    C-contiguous, row-major, double precision unless stated otherwise, and
 *    8-byte aligned.  The caller owns every buffer it passes; the library
 *    never frees or retains caller memory beyond the call (device outputs are
 *    written by work enqueued on the caller's stream).
 *  - Stream ordering: cbic_solve_batch enqueues its kernels on the given HIP
 *    stream (hipStream_t passed as void*, NULL = the null stream) and returns
 *    without waiting; outputs are valid once that stream has completed the
 *    work.  A context's workspace serves one solve at a time: a solve on a
 *    different stream than the previous one first waits for the previous one.
 *
 * Parameter vectors (double, copied at cbic_system_create):
 *  CBIC_SYS_LQ          [n, m, A(n x n), B(n x m), Q(n x n), R(m x m), Q_T(n x n), x_ref(n)]
 *                       f = A x + B u, l = (x-x_ref)^T Q (x-x_ref) + u^T R u,
 *                       l_T = (x-x_ref)^T Q_T (x-x_ref).  (n,m) in {(2,1),(4,2),(6,3)}.
 *  CBIC_SYS_POINT_MASS  [dt, w_u, w_p, w_T, w_o, g_x, g_y, (c_x, c_y, r) x 3]   (n=4, m=2)
 *                       2-D double integrator, semi-implicit Euler v+ = v + dt u,
 *                       p+ = p + dt v+; l = w_u|u|^2 + w_p|p-g|^2
 *                       + w_o sum_i exp(-|p-c_i|^2/r_i^2); l_T = w_T(|p-g|^2 + |v|^2).
 *  CBIC_SYS_PLANAR3     [dt, m1, m2, m3, l1, l2, l3, w_u, w_ee, w_T, w_o, p_x, p_y, c_x, c_y, r]
 *                       (n=6, m=3) planar arm of uniform rods in a horizontal
 *                       plane, relative joint angles, semi-implicit Euler;
 *                       l = w_u|tau|^2 + w_ee|ee-p|^2 + w_o exp(-|ee-c|^2/r^2);
 *                       l_T = w_T|ee-p|^2.
 *  CBIC_SYS_QUAD_SYNTH  [dt, w_u, w_T, w_q, w_v, A(18x18), W1(18x18), W2(18x18), e(18), x_nom(37)]
 *                       (n=37 with q in R^19, v in R^18; m=12)
 *                       M(q) = A^T A + diag(1 + 0.1 sin q[0:18]),
 *                       b = W1 sin q[0:18] + (W2 cos q[0:18]) .* v,
 *                       v+ = v + dt M^-1 ([0_6; u] - b), q+ = q + dt [I_18; e^T] v+;
 *                       l = w_q|q-q_nom|^2 + w_v|v-v_nom|^2 + w_u|u|^2,
 *                       l_T = w_T (w_q|q-q_nom|^2 + w_v|v-v_nom|^2).
 */
#ifndef CBIC_H
#define CBIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cbic_status;
#define CBIC_OK 0
#define CBIC_NOT_READY 1
#define CBIC_E_INVALID (-1)     /* bad argument; nothing was launched          */
#define CBIC_E_OOM (-2)         /* workspace would exceed the context's cap     */
#define CBIC_E_HIP (-3)         /* a HIP runtime call failed                    */
#define CBIC_E_BUSY (-4)        /* server: the request can never be admitted    */
#define CBIC_E_UNSUPPORTED (-5) /* valid but not supported (e.g. LQ dimensions)  */

/* Per-instance status bits (cbic_outputs.status).  Exactly one of the first
 * three describes how the iteration ended; NONFINITE / CHOL_FAIL mark a
 * numerical stop.  The returned trajectory is always the last accepted one. */
#define CBIC_ST_CONVERGED 1u  /* tolerance mode: relative decrease <= rtol        */
#define CBIC_ST_MAX_ITER 2u   /* the iteration budget was used up                 */
#define CBIC_ST_LS_FAILED 4u  /* no trial step lowered the cost: frozen           */
#define CBIC_ST_NONFINITE 8u  /* non-finite cost or gains: frozen                 */
#define CBIC_ST_CHOL_FAIL 16u /* Q_uu not positive definite: frozen               */
#define CBIC_ST_BAD_INPUT 32u /* horizon outside 1..T_max: instance not solved,
                                 J = NaN and all its trajectory outputs zero       */

typedef enum {
  CBIC_SYS_LQ = 0,
  CBIC_SYS_POINT_MASS = 1,
  CBIC_SYS_PLANAR3 = 2,
  CBIC_SYS_QUAD_SYNTH = 3
} cbic_system_kind;

typedef enum { CBIC_FP64 = 0, CBIC_MIXED = 1 } cbic_precision;

typedef struct cbic_context cbic_context;
typedef struct cbic_system cbic_system;
typedef struct cbic_server cbic_server;

/* Solver options.  Fill with cbic_opts_default() and then change fields;
 * struct_size must equal sizeof(cbic_solve_opts). */
typedef struct {
  uint32_t struct_size;
  int32_t max_iter;      /* iteration budget for every instance (>= 0); default 50          */
  double psd_eps;        /* eigenvalue floor of the clipped Hessians (>= 0); default 1e-6   */
  int32_t ls_max_trials; /* line-search trials alpha = beta^j, j < trials (>= 0); default 16 */
  double ls_beta;        /* backtracking factor in (0,1); default 0.5                        */
  int32_t stop_mode;     /* 0: run the budget (freeze only on failure); 1: also stop when an
                            accepted step lowers J by at most rtol*|J|                       */
  double rtol;           /* default 1e-10                                                    */
  int32_t lookahead_K;   /* K of the K-step cost-to-go; <= 0 means the horizon (default 0)  */
  int32_t precision;     /* cbic_precision; default CBIC_FP64                                */
  int32_t schedule;      /* 0 = automatic (tuned table), else a schedule id (see below)      */
  int32_t iters_per_launch; /* G: iterations per kernel launch; <= 0 = all in one launch     */
  int32_t group_lanes;   /* lane schedule: lanes per instance (1,2,4,8,16; they split the
                            line-search trials); 0 = automatic                               */
  uint32_t flags;        /* CBIC_FLAG_* bits                                                 */
  int32_t regularization; /* CBIC_REG_CLIP (default) or CBIC_REG_LM, see below               */
  double lm_mu0;         /* CBIC_REG_LM: initial and smallest mu (> 0); default 1e-6          */
  double lm_factor;      /* CBIC_REG_LM: mu is multiplied or divided by it (> 1); default 10   */
  double lm_mu_max;      /* CBIC_REG_LM: largest mu tried (>= lm_mu0); default 1e10            */
  double u_max;          /* control bound |u_k,i| <= u_max of eq. 1 (> 0); default +infinity
                            (unbounded); see below                                            */
  int32_t wg_per_cu;     /* workgroup schedule: instances resident per compute unit, 1 or 2;
                            0 = automatic.  See below                                         */
} cbic_solve_opts;

/* regularization of the backward sweep (paper Sec. IV-B)
 * CBIC_REG_CLIP  the running and terminal state-cost Hessians and the
 *                control-cost Hessian are eigenvalue-clipped at psd_eps (eq. 7)
 * CBIC_REG_LM    Levenberg-Marquardt, the ablation the paper argues against
 *                for batches: the Hessians are only symmetrised and
 *                Q_uu + mu I is factored, mu per instance; when the Cholesky
 *                or the line search fails the instance multiplies mu by
 *                lm_factor and retries its backward sweep (frozen with the
 *                failure's status once mu would exceed lm_mu_max), after an
 *                accepted step it divides mu by lm_factor (not below lm_mu0);
 *                mu carries over between the launches of one solve.  Every
 *                system and schedule, and served requests. */
#define CBIC_REG_CLIP 0
#define CBIC_REG_LM 1

/* control bound (paper eq. 1): with a finite u_max every control component is
 * kept in [-u_max, u_max].  The warm start is clamped into the box; each step
 * of the backward sweep minimises the local model over the box (a bounded
 * quadratic program in the control step, solved exactly by an active-set
 * method in FP64), the feedback rows of the components held at a bound are
 * zero, and the line-search rollouts clamp their controls.  Every system and
 * schedule (the workgroup schedule solves the box QP with one wave, a lane
 * per control component), and served requests.  A bound that never binds
 * changes no bit of a result. */

/* schedule ids */
#define CBIC_SCHED_LANE 1  /* one lane per instance, registers + step-major HBM          */
#define CBIC_SCHED_GROUP 2 /* a workgroup per instance, matrices in LDS (37-dim system)   */

/* wg_per_cu (workgroup schedule only; the lane schedule ignores it)
 *   1  one instance per compute unit: the iteration kernel keeps all its
 *      values in registers (one wave per SIMD)
 *   2  two instances share a compute unit (two waves per SIMD): registers are
 *      capped at 256 per lane and some values spill, but the second instance
 *      hides the latency of the first one's serial chain; pays off once the
 *      batch has more instances than the device has compute units
 *   0  the autotuned choice for the problem class (cbic_autotune), else 1 for
 *      batches of at most one instance per compute unit and 2 above
 * FP64 solves always run one instance per compute unit (their shared-memory
 * block is half a compute unit's, and two per unit were slower at every
 * batch size measured).  No result depends on it. */

/* flags */
#define CBIC_FLAG_GRAPH 1u  /* launch the iteration chain through a captured HIP graph      */
#define CBIC_FLAG_TIMING 2u /* record HIP events around init / iterations / finalisation on
                               the solve's stream; read them with cbic_phase_times          */
#define CBIC_FLAG_INPUT_ORDER 4u /* iterate the instances in the horizon sort's order.  By
                               default the iteration launches take them longest horizon
                               first and, within a horizon, highest initial cost J^0 first
                               (quarter-octave levels; in a batch of one horizon, within a
                               level, highest non-convex share of J^0 first where the system
                               has one: the point mass's obstacle terms, half-octave
                               levels), so that instances of similar expected work share a
                               wave; a scheduling choice only: no result depends on it      */

/* Output buffers: caller-owned DEVICE pointers, AoS per instance, padded to
 * T_max; entries past an instance's horizon are written as zero.
 * Required: X[B][T_max+1][n], U[B][T_max][m], J[B] (double), iters[B] (int32),
 * status[B] (uint32).  Optional (NULL = not computed): Vbar[B][T_max+1],
 * Vx[B][T_max+1][n], xK[B][T_max+1][n], cost_trace[B][max_iter+1] (J after each
 * accepted iteration, then repeated), work[B][4] (int32: backward sweeps,
 * line-search rollout passes, rollout steps read, rollout steps written -- the
 * traffic that instance caused; lanes sharing an instance share its reads),
 * jtrace[B][max_iter] (int32: for each iteration the accepted line-search
 * index j, alpha = ls_beta^j; -1 for the iteration in which the instance was
 * frozen by a failure (no accepted step, Cholesky failure, non-finite gains);
 * -2 for iterations not run). */
typedef struct {
  double* X;
  double* U;
  double* J;
  int32_t* iters;
  uint32_t* status;
  double* Vbar;
  double* Vx;
  double* xK;
  double* cost_trace;
  int32_t* work;
  int32_t* jtrace;
} cbic_outputs;

/* Last error message of the calling thread ("" if none). */
const char* cbic_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t cbic_version(void);

/* Fill *opts with the defaults listed above. */
cbic_status cbic_opts_default(cbic_solve_opts* opts);

/* Create a context on HIP device `hip_device`.  workspace_cap_bytes bounds the
 * device memory the context may allocate for its workspace (0 = no bound).
 * The context owns its workspace and frees it in cbic_context_destroy. */
cbic_status cbic_context_create(int hip_device, size_t workspace_cap_bytes, cbic_context** out);
cbic_status cbic_context_destroy(cbic_context* ctx);

/* Create a system of the given kind from its parameter vector (host memory,
 * copied).  ctx may be NULL: the system is then only validated and usable for
 * cbic_system_dims / cbic_workspace_size; a solve needs a system created on
 * that solve's context (its device copy of the parameters lives there).
 * Errors: CBIC_E_INVALID for a wrong length or non-finite entry. */
cbic_status cbic_system_create(cbic_context* ctx, cbic_system_kind kind, const double* h_params,
                               size_t n_params, cbic_system** out);
cbic_status cbic_system_dims(const cbic_system* sys, int32_t* n, int32_t* m);
cbic_status cbic_system_destroy(cbic_system* sys);

/* Device workspace a solve of B instances with horizon capacity T_max needs. */
cbic_status cbic_workspace_size(const cbic_system* sys, int32_t B, int32_t T_max, const cbic_solve_opts* opts,
                                size_t* bytes);

/* Solve B instances (paper Sec. II, eq. 1; iLQR of Sec. IV).
 *  d_T   [B] int32 horizons in 1..T_max, or NULL for T_max everywhere;
 *  d_x0  [B][n] initial states (required);
 *  d_U0  [B][T_max][m] warm-start controls, or NULL for zeros (the initial
 *        states are the rollout of these controls).
 * Enqueues on `stream` and returns.  Errors: CBIC_E_INVALID (B < 1,
 * T_max < 1, NULL required pointer, misaligned pointer, bad opts),
 * CBIC_E_OOM, CBIC_E_HIP. */
cbic_status cbic_solve_batch(cbic_context* ctx, const cbic_system* sys, int32_t B, int32_t T_max,
                             const int32_t* d_T, const double* d_x0, const double* d_U0,
                             const cbic_solve_opts* opts, const cbic_outputs* out, void* stream);

/* Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, kernels and results as cbic_solve_batch, but
 * the workspace is not the context's: it is a device array of
 * CBIC_NOALLOC_SCRATCH_BYTES held by the library on every GPU it runs on from
 * load until the process ends, so the call allocates nothing (no hipMalloc,
 * no graph of its own) and only enqueues kernels on `stream`.
 * Limits and rules:
 *  - the solve's workspace (cbic_workspace_size) must fit the array, else
 *    CBIC_E_OOM before anything is launched (64 MiB: e.g. about 7000
 *    point-mass instances of horizon 100 in the mixed form, 3500 in FP64);
 *  - opts->flags must not hold CBIC_FLAG_GRAPH or CBIC_FLAG_TIMING, and an LQ
 *    system must already hold a parameter block for the solve's psd_eps (the
 *    one it was created with, 1e-6, or one an earlier cbic_solve_batch built)
 *    (CBIC_E_INVALID otherwise);
 *  - every call on one GPU uses that GPU's one array, whatever its context or
 *    stream: calls that overlap in time on a GPU race and give undefined
 *    results, so the caller orders them (one stream, or events).  No state
 *    carries over from one call to the next: each call initialises what it
 *    reads.
 * Errors: as cbic_solve_batch. */
#define CBIC_NOALLOC_SCRATCH_BYTES (64u << 20)
cbic_status cbic_solve_batch_noalloc(cbic_context* ctx, const cbic_system* sys, int32_t B, int32_t T_max,
                                     const int32_t* d_T, const double* d_x0, const double* d_U0,
                                     const cbic_solve_opts* opts, const cbic_outputs* out, void* stream);

/* Autotune the schedule for one problem class: solve the given batch (same
 * arguments as cbic_solve_batch) once per candidate, time each on `stream`,
 * and remember the fastest in the context for solves of the same system kind,
 * precision, stop rule, iteration budget, batch size (rounded up to a power of
 * two) and T_max.  The candidates are the lanes-per-instance widths 1, 2, 4,
 * 8, 16 on the lane schedule (used by solves whose group_lanes is 0), and one
 * or two instances per compute unit on the workgroup schedule in the mixed
 * precision (used by solves whose wg_per_cu is 0; an FP64 workgroup solve has
 * the one choice 1).  Blocks until done; allocates scratch outputs.  No
 * candidate changes results (the line-search rule picks the same step).
 * *best_group / *best_ms (may be NULL) receive the choice (the width, or the
 * instances per compute unit) and its time. */
cbic_status cbic_autotune(cbic_context* ctx, const cbic_system* sys, int32_t B, int32_t T_max, const int32_t* d_T,
                          const double* d_x0, const double* d_U0, const cbic_solve_opts* opts, void* stream,
                          int32_t* best_group, double* best_ms);

/* Iteration-budget calibration (paper Sec. IV-A).  Solves the batch (same
 * arguments as cbic_solve_batch, zero warm start) with the relative-decrease
 * stop (opts->rtol) and at most `cap` iterations (1..100000; the paper uses
 * 1000), then returns the nearest-rank 99th (*p99) and 50th (*p50) percentiles
 * of the per-instance accepted-iteration counts: the budget for batches
 * warm-started with zero controls and from a trained actor, respectively.  An instance
 * stopped by the cap counts as `cap`; instances with an invalid horizon are
 * left out.  opts supplies precision, eps and the line search; its stop_mode
 * and max_iter are replaced.  hist (optional, host, cap + 1 entries) receives
 * the histogram of the counts.  Blocks until done; allocates scratch outputs.
 * Errors: CBIC_E_INVALID (NULL required pointer, B or T_max < 1, cap out of
 * range, no valid instance), CBIC_E_OOM, CBIC_E_HIP. */
cbic_status cbic_calibrate_max_iter(cbic_context* ctx, const cbic_system* sys, int32_t B, int32_t T_max,
                                    const int32_t* d_T, const double* d_x0, const cbic_solve_opts* opts,
                                    int32_t cap, void* stream, int32_t* p99, int32_t* p50, int64_t* hist);

/* Milliseconds spent by the last solve on this context that was launched with
 * CBIC_FLAG_TIMING in its three phases: ms[0] warm start and initial rollout
 * (with the iteration order of CBIC_FLAG_INPUT_ORDER's default), ms[1] the
 * iteration kernels (backward sweeps and line searches), ms[2] finalisation
 * (status, critic targets, outputs).  A lane-schedule solve in one launch
 * (without CBIC_FLAG_GRAPH, iters_per_launch <= 0 or >= max_iter) finalises
 * each instance inside the iteration kernel as soon as it stops iterating:
 * ms[1] then holds both and ms[2] is 0.  Waits for that solve's stream work
 * to finish.  CBIC_E_INVALID if no timed solve was launched. */
cbic_status cbic_phase_times(cbic_context* ctx, double* ms3);

/* ---------------------------------------------------------------- serving
 * A continuous-batching request loop.  Requests (one TO instance each, any
 * system created on the server's context, any horizon up to the server's
 * t_max) are grouped into classes: the system, the precision and the options
 * that change a result (max_iter, psd_eps, the line search, the stop rule,
 * lookahead_K, the regularization and its parameters, u_max); requests of
 * different classes never share a pool, so each gets exactly its own options
 * (the lanes-per-instance width and launch split come from the class's first
 * request: they do not change results).  Each class has a device slot pool
 * with its own stream; admitted requests iterate G iterations per launch beside
 * the requests already resident, so work of requests that arrive while others
 * run overlaps on the GPU.  Their iterates stay in device memory until they
 * finish; finished slots are extracted, copied to host and freed for new
 * admissions.  Memory: the device memory of all pools together stays within
 * mem_cap_bytes.  A class's pool gets as many slots (up to slots_per_class)
 * as fit beside the others; when not even one fits, idle pools (nothing
 * resident or waiting) are released, and a class that still finds no room
 * waits until another pool goes idle. */
typedef struct {
  uint32_t struct_size;
  size_t mem_cap_bytes;    /* device memory for all slot pools; default 32 GiB              */
  int32_t slots_per_class; /* slots of each (system, precision) pool; default 4096           */
  int32_t t_max;           /* largest horizon a request may have; default 200               */
  int32_t iters_per_launch;/* G; default 4                                                  */
} cbic_server_opts;

/* Per-request result: host buffers the caller provides to cbic_server_poll.
 * X[(T+1) n], U[T m], Vbar[T+1], Vx[(T+1) n] (Vbar, Vx may be NULL). */
typedef struct {
  double* X;
  double* U;
  double* Vbar;
  double* Vx;
  double J;
  int32_t iters;
  uint32_t status;
  double t_submit;   /* seconds, server clock */
  double t_admit;
  double t_done;
} cbic_result;

cbic_status cbic_server_opts_default(cbic_server_opts* opts);
cbic_status cbic_server_create(cbic_context* ctx, const cbic_server_opts* opts, cbic_server** out);
/* Queue one request.  h_x0 [n]; h_U0 [T][m] or NULL; opts are checked as
 * cbic_solve_batch checks them.  Returns a ticket.  Errors: CBIC_E_INVALID (bad
 * argument or options; an LQ system whose clipped Hessians were built for
 * another psd_eps), CBIC_E_UNSUPPORTED (the Levenberg-Marquardt variant or a
 * control bound for a system on the workgroup schedule), CBIC_E_BUSY (a
 * one-slot pool of the request's class exceeds the cap: it can never run). */
cbic_status cbic_server_submit(cbic_server* srv, const cbic_system* sys, int32_t T, const double* h_x0,
                               const double* h_U0, const cbic_solve_opts* opts, uint64_t* ticket);
/* CBIC_OK with *out filled once the ticket is done (the ticket is then
 * released), CBIC_NOT_READY while pending, CBIC_E_INVALID for an unknown ticket. */
cbic_status cbic_server_poll(cbic_server* srv, uint64_t ticket, cbic_result* out);
/* Counters of a server (host-side bookkeeping; no device work). */
typedef struct {
  uint64_t submitted, completed, rounds;
  size_t inflight_bytes;      /* footprint of the requests resident now          */
  size_t peak_inflight_bytes; /* largest footprint resident at once so far        */
  size_t pool_bytes;          /* device memory held by the slot pools now         */
  int32_t classes;            /* request classes seen (see cbic_server_submit)    */
  int32_t max_resident;       /* most requests resident at once                   */
  size_t peak_pool_bytes;     /* most device memory the pools held at once (<= cap) */
  uint64_t evictions;         /* idle pools released to make room for another class */
  uint64_t launches;          /* iteration launches (G iterations of one class each) */
  uint64_t launched_slots;    /* resident requests summed over those launches      */
  double host_busy_s;         /* seconds the server's worker thread spent working (not
                                 sleeping): its share of wall time shows whether the host
                                 side limits the request rate                        */
} cbic_server_stats;
cbic_status cbic_server_get_stats(cbic_server* srv, cbic_server_stats* out);

/* Server clock in seconds (the time base of cbic_result's t_* fields). */
double cbic_server_clock(const cbic_server* srv);
/* Block until every submitted request is done. */
cbic_status cbic_server_drain(cbic_server* srv);
cbic_status cbic_server_destroy(cbic_server* srv);

/* ---- Biased initial states and the actor warm start (paper Sec. II, III) ----
 * CACTO-BIC ranks 10N candidate initial states by the std-critic's predicted
 * standard deviation V^std (eq. 6 trains it; Sec. III-C/D) and solves the N
 * most uncertain ones; from its second iteration the actor's rollouts
 * warm-start the TO batch (Sec. II).  These calls run those two steps on the
 * GPU with networks given as plain FP32 multilayer perceptrons.
 *
 * cbic_mlp describes a perceptron with `depth` hidden layers of `width` units
 * and activation `act`, then a linear output layer of out_dim units followed
 * by `out_act`.  Its parameters are one contiguous FP32 array in device memory
 * (row-major, y = x W + b):
 *   W_0 [in_dim][width], b_0 [width],
 *   then depth - 1 times W_l [width][width], b_l [width],
 *   then W_out [width][out_dim], b_out [out_dim]
 * (cbic_mlp_param_count gives the length).  Arithmetic is FP32, as the
 * paper's networks are.  Time enters the networks as an input feature
 * tau in [0, 1): the fraction of the episode already elapsed (paper Sec. II
 * appends time to the state). */
#define CBIC_ACT_TANH 0
#define CBIC_ACT_ELU 1
#define CBIC_ACT_RELU 2
#define CBIC_OUT_LINEAR 0
#define CBIC_OUT_TANH 1     /* out_scale * tanh(z): a bounded actor      */
#define CBIC_OUT_SOFTPLUS 2 /* log(1 + e^z): a positive std-critic output */
typedef struct {
  int32_t in_dim;      /* 1..64                                   */
  int32_t width;       /* 32 or 64                                */
  int32_t depth;       /* hidden layers, 1..4                     */
  int32_t out_dim;     /* 1..16                                   */
  int32_t act;         /* CBIC_ACT_*                              */
  int32_t out_act;     /* CBIC_OUT_*                              */
  double out_scale;    /* CBIC_OUT_TANH only; finite              */
  const float* params; /* device, cbic_mlp_param_count() floats  */
} cbic_mlp;

/* Number of FP32 parameters of the network (*count); CBIC_E_INVALID for a
 * description outside the ranges above. */
cbic_status cbic_mlp_param_count(const cbic_mlp* net, int64_t* count);

/* out[b][o] = net(in[b]) for B rows; d_in [B][in_dim] and d_out [B][out_dim]
 * are FP32 device arrays.  Asynchronous on `stream`. */
cbic_status cbic_mlp_forward(cbic_context* ctx, const cbic_mlp* net, int32_t B, const float* d_in, float* d_out,
                             void* stream);

/* Biased initial-state selection (Sec. III-D): score the Bc candidates
 * x~_i = (x_i, tau_i) with the std-critic, d_score[i] = V^std(x~_i), and write
 * to d_sel the indices of the N highest scores in ascending index order
 * (equal scores: lower index first; NaN scores rank lowest; -0 equals +0).
 * A candidate carries its remaining horizon T_i (1..T_max): it starts
 * T_max - T_i steps into the episode, tau_i = (T_max - T_i) / T_max (the time
 * convention of cbic_actor_rollout).  d_x [Bc][n] (FP64), d_T [Bc] (int32, or
 * NULL: the network then takes the state alone), d_score [Bc] (FP32,
 * written), d_sel [N] (int32); optional gathered outputs for the next TO
 * batch: d_x_sel [N][n] (the selected states, in d_sel's order) and d_T_sel
 * [N] (their horizons; requires d_T).  All device memory.  net->in_dim must
 * be n + 1 with d_T, n without; out_dim 1.  0 <= N <= Bc.  The selection runs
 * in one workgroup (it reads the scores a few times over).  Asynchronous on
 * `stream`.
 * Errors: CBIC_E_INVALID (bad sizes or network, NULL pointer), CBIC_E_HIP. */
cbic_status cbic_bic_select(cbic_context* ctx, const cbic_mlp* std_critic, int32_t Bc, int32_t n, const double* d_x,
                            const int32_t* d_T, int32_t T_max, int32_t N, float* d_score, int32_t* d_sel,
                            double* d_x_sel, int32_t* d_T_sel, void* stream);

/* Actor warm start (Sec. II): roll the system out from each initial state under
 * the actor, u_k = actor(x_k, tau_k) with tau_k = (T_max - T_b + k) / T_max
 * (an instance of horizon T_b starts T_max - T_b steps into the episode),
 * x_{k+1} = f(x_k, u_k) in FP64, for k < T_b.  Writes d_U [B][T_max][m] (the
 * warm start for cbic_solve_batch) and, if not NULL, d_X [B][T_max+1][n];
 * entries past T_b are zero.  d_T [B] (int32, or NULL: all T_max), d_x0
 * [B][n].  actor->in_dim must be n + 1, out_dim m.  Lane-schedule systems
 * only (CBIC_E_UNSUPPORTED for the quadruped).  Asynchronous on `stream`.
 * Errors: CBIC_E_INVALID, CBIC_E_UNSUPPORTED, CBIC_E_HIP. */
cbic_status cbic_actor_rollout(cbic_context* ctx, const cbic_system* sys, const cbic_mlp* actor, int32_t B,
                               int32_t T_max, const int32_t* d_T, const double* d_x0, double* d_U, double* d_X,
                               void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CBIC_H */
