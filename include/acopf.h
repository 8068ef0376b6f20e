/*
 * acopf.h -- C ABI of the MI355X (gfx950) two-level component ADMM for AC
 * optimal power flow (Kim & Kim, "Accelerated Computation and Tracking of AC
 * Optimal Power Flow Solutions Using GPUs", PSCC 2022).
 *
 * The problem is eq. (acopf) of Sec. II-A: minimize the sum of generator
 * costs subject to the bus power balances (eqs. pg, qg), line limits
 * (eqs. ij-limit, ji-limit), generator and voltage bounds, with branch flows
 * given by eqs. (pij)-(qji). It is decomposed by components (Sec. II-B/II-C)
 * and solved by Algorithm 1 (Sec. III): an inner ADMM over generators and
 * branches (x), buses (xbar), artificial variables (z) and multipliers (y),
 * inside an outer augmented-Lagrangian loop on z = 0 (lambda, beta).
 *
 * All per-element arrays are host pointers in structure-of-arrays form,
 * FP64 unless noted, per unit on base_mva. Every step of the iteration runs
 * in HIP kernels on the device given to acopf_create; host<->device copies
 * happen only in create/update_loads/get_state/set_state and a readback of a
 * few control words per chunk of iterations inside acopf_solve.
 *
 * Return codes: 0 on success, a negative ACOPF_E* value on error, with a
 * message available from acopf_last_error() (thread-local). Non-convergence
 * is not an error: it is reported in acopf_result.status.
 *
 * Threads: handles are independent, and different handles may be driven
 * from different host threads at once (each on its own stream). The calls
 * on one handle must not overlap; a handle has no lock of its own.
 */
#ifndef ACOPF_H
#define ACOPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ACOPF_OK = 0,
  ACOPF_EINVAL = -1,  /* invalid argument or grid data (NaN/Inf, bad index,
                         empty bound interval, r = x = 0, isolated bus)     */
  ACOPF_ENOMEM = -2,  /* device or host allocation failed                  */
  ACOPF_EDEVICE = -3, /* a HIP runtime call failed (text in last_error)     */
  ACOPF_ESTATE = -4,  /* call not valid in the handle's current state       */
  ACOPF_EBUDGET = -5  /* serving: the HBM budget cannot hold the resident
                         grids                                              */
};

enum { /* acopf_result.status */
  ACOPF_CONVERGED = 0, /* inner test and ||z||_inf <= eps_z both hold       */
  ACOPF_MAX_ITER = 1,  /* max_outer reached, or fixed-iteration mode ended   */
  ACOPF_NUMERICAL = 2  /* a residual became NaN or Inf                       */
};

enum { /* acopf_solve mode */
  ACOPF_COLD = 0,     /* cold start of Sec. IV-B, then Algorithm 1           */
  ACOPF_WARM = 1,     /* keep the primal/dual state (tracking, Sec. IV-C);
                         restart beta, the outer counter and ||z|| history  */
  ACOPF_CONTINUE = 2  /* keep everything, counters included                 */
};

enum { /* acopf_get_state / acopf_set_state: what */
  ACOPF_U = 0,         /* [m] generator/branch-side coupling values          */
  ACOPF_V = 1,         /* [m] bus-side copies                                */
  ACOPF_Z = 2,         /* [m] artificial variables                           */
  ACOPF_Y = 3,         /* [m] inner multipliers                              */
  ACOPF_LAMBDA = 4,    /* [m] outer multipliers                              */
  ACOPF_BRANCH_X = 5,  /* [6 n_branch] (v_i, v_j, th_i, th_j, s_ij, s_ji)    */
  ACOPF_BRANCH_LTIL = 6, /* [2 n_branch] line-limit AL multipliers           */
  ACOPF_BRANCH_RTIL = 7, /* [n_branch] line-limit AL penalties               */
  ACOPF_SCALARS = 8,   /* [9] beta, ||z|| at the last outer step, r_pri,
                          r_dual, r_z, outer, inner_total, inner_in_outer,
                          status                                             */
  ACOPF_PD = 9,        /* [n_bus] */
  ACOPF_QD = 10,       /* [n_bus] */
  ACOPF_HISTORY = 11,  /* get only: [6 inner_total] per inner iteration of
                          the last solve: r_pri, r_dual, r_z, 0, beta, outer */
  ACOPF_STATS = 12,    /* get only: [16] branch-solve counters summed over
                          the iterations run with acopf_set_counting on:
                          solves, algorithmic flops, sin/cos, TRON calls,
                          TRON iterations, f/g/H and f evaluations, Cauchy
                          trials, CG iterations, Cholesky attempts, search
                          trials, AL rounds, TRON converged / at the cap /
                          stalled, then 0; the same for every grid index    */
  ACOPF_BRANCH_ALPHA = 13, /* [n_branch] Cauchy step length each branch's last
                          trust-region solve ended with; the next solve of
                          that branch starts its projected search from it
                          (1 after a cold start)                            */
  ACOPF_SOLUTION = 14  /* get only: the ADMM solution of Sec. IV-A,
                          [2 n_gen + 2 n_bus + 4 n_branch] in input order:
                          p_g [n_gen] and q_g [n_gen] of the generator
                          problems; |V| = sqrt(w) [n_bus] and theta [n_bus]
                          of the bus problems (from each bus's first branch
                          end: from-ends, then to-ends, in input order);
                          p_ij, q_ij, p_ji, q_ji [n_branch each] recomputed
                          from those voltages by eqs. (pij)-(qji). Runs the
                          recovery kernels on the handle's stream; allocates
                          their scratch on first use                         */
};

/* Coupling order (m = 2 n_gen + 8 n_branch), the same in every vector:
 * generator g owns entries 2g (p_g) and 2g+1 (q_g); branch l owns
 * 2 n_gen + 8 l + k, k = 0..7: p_ij, q_ij, p_ji, q_ji, w_i(ij), th_i(ij),
 * w_j(ij), th_j(ij) (Sec. II-B). Each coupling reads u - v + z = 0.      */

typedef struct {
  int32_t n_bus, n_gen, n_branch, ref_bus;
  double base_mva;                            /* MVA, > 0                  */
  const double *pd, *qd;                      /* [n_bus] loads             */
  const double *gs, *bs;                      /* [n_bus] bus shunts        */
  const double *vmin, *vmax;                  /* [n_bus] |V| bounds        */
  const int32_t *gen_bus;                     /* [n_gen] 0-based bus       */
  const double *pmin, *pmax, *qmin, *qmax;    /* [n_gen] output bounds     */
  const double *c2, *c1, *c0;                 /* [n_gen] cost on MW: c2 P^2
                                                 + c1 P + c0, P = base_mva p */
  const int32_t *br_from, *br_to;             /* [n_branch] 0-based buses  */
  const double *r, *x, *b;                    /* [n_branch] series r + jx,
                                                 total line charging b      */
  const double *tap, *shift;                  /* [n_branch] a = tap e^{j shift}
                                                 (tap > 0, shift in rad)    */
  const double *rate;                         /* [n_branch] MVA/base limit;
                                                 <= 0 means unlimited       */
} acopf_grid;

typedef struct {
  double rho_pq, rho_va;     /* ADMM penalties on power / voltage couplings
                                (Table 1)                                   */
  double obj_scale;          /* objective scaling inside the ADMM (Sec. IV-A) */
  double rate_scale;         /* line-limit tightening (Sec. IV-A: 0.99)     */
  double beta0, beta_gamma, beta_omega, beta_max; /* outer penalty: beta *=
                                gamma when ||z|| > omega ||z||_prev, capped */
  double lambda_max;         /* projection bound of lambda                  */
  double eps_pri, eps_dual, eps_z; /* termination on inf-norms             */
  int32_t max_outer, max_inner;
  double tron_gtol, tron_ftol; /* branch TRON stopping tolerances           */
  int32_t tron_maxit;
  double al_rho0, al_rho_growth, al_rho_max, al_tol, al_shrink; /* branch
                                line-limit augmented Lagrangian            */
  int32_t al_maxit;
} acopf_params;

typedef struct {
  int32_t status;            /* ACOPF_CONVERGED / MAX_ITER / NUMERICAL      */
  int32_t inner_iters;       /* cumulative inner iterations of this solve   */
  int32_t outer_iters;
  int32_t branch_failures;   /* TRON exits by iteration cap or stall        */
  double objective;          /* sum of generator costs at the generator-side
                                p_g (Sec. IV-A), $/h, c0 included          */
  double r_pri, r_dual, r_z; /* final inf-norm residuals                    */
  double beta;
  double seconds;            /* wall time of the solve call                 */
} acopf_result;

/* Launch shape of the iteration (see acopf_set_tuning / acopf_autotune). */
typedef struct {
  int32_t xstep_block; /* threads per block of the branch/generator kernel:
                          64, 128 or 256 (one lane per branch)              */
  int32_t bus_block;   /* threads per block of the bus kernel: 64..1024,
                          a multiple of 64; a block takes a tile of up to
                          bus_block / 4 consecutive buses of one grid       */
  int32_t chunk;       /* inner iterations between control readbacks, 1..64 */
  int32_t use_graph;   /* 1: replay each chunk as one captured hipGraph     */
  int32_t xstep_waves; /* 0: the branch kernel above, one lane per branch;
                          1..4: persistent branch kernel instead, with this
                          many 64-lane wavefronts per SIMD of the device;
                          each lane takes branches from a shared counter and
                          advances one TRON iteration per loop trip, so lanes
                          that finish early take more work (same results) */
  int32_t xstep_per_lane; /* lane-per-branch kernel: unlimited branches
                          solved one after another by each lane, 1..8; 0:
                          automatic: 2 when that makes every branch
                          wavefront fit the device's SIMDs at once, else 1 */
  int32_t lanes;       /* launch lanes, 1..4 (at most the handle's grids;
                          more are reduced to that): the grids are split
                          into this many groups of about equal branch
                          count, each launched on a stream of its own, so
                          that one group's issue-bound branch step overlaps
                          another's memory-bound bus step (same results).
                          Default: 2 for a handle of several grids, else 1;
                          the persistent branch kernel runs as one lane   */
} acopf_tuning;

typedef struct acopf_s* acopf_handle;

/* Fill *p with the library defaults. */
void acopf_default_params(acopf_params* p);

/* Validate and lay out n_grids grids on device `device`, then cold-start
 * them. Grids are independent problems batched into the same launches and
 * share `params`. `hip_stream` is the hipStream_t to run on, or NULL for a
 * library-owned stream. Input arrays are borrowed for the call only; the
 * handle owns all device memory until acopf_destroy.
 * Errors: EINVAL (bad data, n_grids < 1), ENOMEM, EDEVICE. */
int acopf_create(const acopf_grid* grids, int32_t n_grids,
                 const acopf_params* params, int32_t device,
                 void* hip_stream, acopf_handle* out);

/* Run Algorithm 1 on every grid of the handle. mode: ACOPF_COLD, ACOPF_WARM
 * or ACOPF_CONTINUE. fixed_iters > 0 runs exactly that many inner
 * iterations (termination tests off; outer updates still happen when the
 * inner test passes). results: [n_grids], may be NULL; when given, every
 * grid's result is read at the end with one objective launch and one wait.
 * Errors: EINVAL (mode), ESTATE (WARM/CONTINUE before any solve), EDEVICE. */
int acopf_solve(acopf_handle h, int32_t mode, int32_t fixed_iters,
                acopf_result* results);

/* Replace the real-power bounds of grid `grid`'s generators (input order,
 * p.u.), e.g. the ramp-limited bounds max(pmin, p_t - r), min(pmax, p_t + r)
 * of a tracking horizon (Sec. IV-C); the generator step of the next
 * iterations projects onto them. Errors: EINVAL (index, NaN/Inf,
 * pmin > pmax), EDEVICE. */
int acopf_update_gen_bounds(acopf_handle h, int32_t grid, const double* pmin,
                            const double* pmax);

/* Replace the loads of grid `grid` (H2D copy of 2 n_bus doubles); the next
 * ACOPF_WARM solve tracks the new optimum from the resident state (Sec. IV-C).
 * Errors: EINVAL (index, NaN/Inf), EDEVICE. */
int acopf_update_loads(acopf_handle h, int32_t grid, const double* pd,
                       const double* qd);

/* Continuous batching. acopf_start begins a solve of one grid without
 * touching the others (mode and fixed_iters as in acopf_solve); acopf_run
 * iterates every running grid in the same launches until at least one of
 * them finishes or max_iters inner iterations have run, and reports how many
 * are still running; acopf_poll reads one grid's state and, once finished,
 * its result (seconds = host time from start to the readback that saw it
 * finish; with out non-NULL it waits for the handle's stream). Grids that
 * are not running cost nothing in the launches.
 * Errors: EINVAL, ESTATE (grid already running, or WARM/CONTINUE on a grid
 * never solved), EDEVICE. */
int acopf_start(acopf_handle h, int32_t grid, int32_t mode, int32_t fixed_iters);
int acopf_run(acopf_handle h, int32_t max_iters, int32_t* running);
int acopf_poll(acopf_handle h, int32_t grid, int32_t* is_running, acopf_result* out);

/* Device-side copy of the complete state of grid src into grid dst (ADMM
 * vectors, branch state, loads, control block). Both must hold the same grid
 * data (same arrays passed to acopf_create). Errors: EINVAL, ESTATE (dst
 * running), EDEVICE. */
int acopf_copy_grid(acopf_handle h, int32_t src, int32_t dst);

/* Device-side snapshot of the whole handle's state: what = 0 saves, 1
 * restores the last save (first save allocates a second copy of the state).
 * Errors: EINVAL, ESTATE (restore without save), ENOMEM, EDEVICE. */
int acopf_snapshot(acopf_handle h, int32_t what);

/* Launch shape: set explicitly, read back, or pick by timing `iters` inner
 * iterations of every candidate from the current state (the state is saved
 * before and restored after, so tuning leaves the solve unchanged).
 * Candidates: x-step {lane per branch at xstep_block 64, 128, 256 with
 * xstep_per_lane automatic or 1; persistent at xstep_waves 1, 2} x
 * bus_block {128, 256, 512, 1024} x
 * chunk {8, 16, 32}, graphs on, at the current lanes; then lanes {1, 2, 4}
 * (up to the number of grids) for the best of those. Errors: EINVAL,
 * ENOMEM, EDEVICE. */
int acopf_set_tuning(acopf_handle h, const acopf_tuning* t);
int acopf_get_tuning(acopf_handle h, acopf_tuning* t);
int acopf_autotune(acopf_handle h, int32_t iters, acopf_tuning* out);

/* Copy one state vector of grid `grid` to the host buffer out[n] (n must
 * equal the size listed with the ACOPF_* `what` codes, in canonical order):
 * the primal and dual iterates of Algorithm 1 (Sec. III: u = x side, v = xbar
 * side, z, y, lambda), the branch subproblem state of eq. (branch) (x,
 * ltil, rtil, Cauchy step length), the control scalars, loads, residual
 * history, counters, or the recovered solution (ACOPF_SOLUTION, Sec. IV-A).
 * The caller owns out. Synchronous on the handle's stream.
 * Errors: EINVAL (index, size, code), ENOMEM (solution scratch), EDEVICE. */
int acopf_get_state(acopf_handle h, int32_t grid, int32_t what, double* out,
                    int64_t n);

/* Overwrite one state vector (checkpoint/resume of Algorithm 1's iterates,
 * or warm-start data for the tracking use of Sec. IV-C); HISTORY, STATS and
 * SOLUTION are read-only. in[n] is borrowed for the call. Not allowed while
 * the grid is running. Errors: EINVAL (size, code, non-finite values,
 * non-positive step lengths), ESTATE (grid running), EDEVICE. */
int acopf_set_state(acopf_handle h, int32_t grid, int32_t what,
                    const double* in, int64_t n);

/* Number of grids, buses, generators, branches of grid `grid` (out[4]). */
int acopf_get_sizes(acopf_handle h, int32_t grid, int64_t* out4);

/* Turn per-kernel timing on or off. While on, every launch of a solve is
 * bracketed by HIP events on the handle's stream (a small overhead).
 * Errors: EINVAL, EDEVICE. */
int acopf_set_profiling(acopf_handle h, int32_t on);

/* Solution quality of grid `grid` at its current state (Sec. IV-A): the
 * ADMM solution is the generator outputs of the generator problems and w,
 * theta of the bus problems (from the bus's first branch end), with the flows
 * recomputed from them by eqs. (pij)-(qji). out6 (p.u.): [0] ||c(x)||_inf
 * over eq. (acopf), the largest of the rest; [1] max |residual of eq. (pg)|;
 * [2] of eq. (qg); [3] max excess sqrt(p^2 + q^2) - rate of eqs.
 * (ij-limit)-(ji-limit) on the unscaled rating; [4] max excess of v = sqrt(w)
 * over [vmin, vmax]; [5] max excess of |theta| over 2 pi. A NaN in the state
 * shows as NaN. Generator bounds hold by construction. Synchronous on the
 * handle's stream; allocates its scratch on the first call.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
int acopf_quality(acopf_handle h, int32_t grid, double* out6);

/* Turn counting on or off (default off): with it, the branch kernel also
 * counts the algorithmic flops of every branch solve (as the plain serial
 * algorithm performs them: + - * / sqrt one each, fused multiply-add two)
 * and its TRON events into ACOPF_STATS, at a few percent of its speed;
 * without it those counters are not touched. Results are the same either
 * way. Errors: EINVAL. */
int acopf_set_counting(acopf_handle h, int32_t on);

/* acopf_quality without any allocation, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same six values as acopf_quality, with the
 * recovery's scratch in a fixed device-resident array of the library
 * (2^20 eight-byte words, 8 MiB, per device, held until the process ends)
 * instead of memory it allocates. The handle must fit that array:
 * 2 n_bus + 4 n_branch + 6 n_grids, summed over the handle's grids, at most
 * 2^20; larger handles are rejected with EINVAL. Every call on one device
 * shares the array (each call clears what must start at zero), so calls
 * that overlap on one GPU, from several threads or on several streams, race.
 * Synchronous on the handle's stream. Errors: EINVAL, EDEVICE. */
int acopf_quality_noalloc(acopf_handle h, int32_t grid, double* out6);

/* Average device time (ms) per iteration over every iteration run with
 * profiling on since the handle was created: out[0] x-step launch
 * (generators, branches, and from a chunk's second iteration on the previous
 * iteration's control decision), out[1] bus/z/y/residual step (which also
 * applies an outer multiplier step that the previous iteration decided),
 * out[2] control kernel (it runs after a chunk's last iteration, or after
 * every iteration with counting on or the persistent x-step), out[3] = 0
 * (kept for layout: the outer step has no launch of its own); out[4] =
 * number of iterations timed. Errors: EINVAL. */
int acopf_get_timing(acopf_handle h, double* out5);

/* Free everything the handle owns. NULL is a no-op. */
void acopf_destroy(acopf_handle h);

/* Message of the last failing call on this thread ("" if none). */
const char* acopf_last_error(void);

/* Measurement helpers, not part of the method: the achievable rates of the
 * calling thread's current device, which a benchmark reports beside the
 * published peaks. Each allocates its own device buffers, stream and events,
 * synchronizes, and releases them before returning.
 * acopf_peak_hbm: a streaming copy of `bytes` bytes (>= 1 MiB, 16-byte
 *   vectors) into a second buffer, `iters` times after one warm-up copy;
 *   *gbs = bytes read plus bytes written, per second, in GB/s.
 * acopf_peak_fp64: eight wavefronts per SIMD, each lane running 8
 *   independent FP64 fused multiply-add chains for `iters` steps, timed
 *   after one untimed run of the same length;
 *   *tflops = 2 flops per fused multiply-add, per second, in TFLOP/s.
 * Return 0, ACOPF_EINVAL for invalid arguments, ACOPF_ENOMEM or
 * ACOPF_EDEVICE. */
int acopf_peak_hbm(int64_t bytes, int32_t iters, double* gbs);
int acopf_peak_fp64(int32_t iters, double* tflops);

/* Free and total device memory of device `device` in bytes (out2[0], out2[1])
 * for sizing a serving budget by HBM footprint (the tracking service's
 * admission). Errors: EINVAL (null output), EDEVICE. */
int acopf_device_memory(int32_t device, int64_t* out2);


/* ------------------------------------------------------------------------
 * Tracking service (Sec. I and Sec. IV-C: the ACOPF optimum followed as loads
 * change, each new load picture solved warm from the previous solution), with
 * continuous batching on one GPU. A server keeps n_grids grids resident in one
 * handle: per grid a home instance holding its committed ADMM state and k_j
 * slot instances within an HBM budget. A request (grid, new loads) is
 * admitted between iteration chunks as soon as one of its grid's slots is
 * free: the home state is copied into the slot on the device, the loads are
 * set, and a warm start joins the running launches. A finished slot becomes
 * its grid's home and the old home a free slot. A grid with no slot runs its
 * requests on its home, one at a time. Not thread-safe; one server per host
 * thread.
 * ---------------------------------------------------------------------- */
typedef struct acopf_server_s* acopf_server;

typedef struct {
  int64_t request_id;  /* as submitted                                      */
  int32_t grid;        /* resident grid                                     */
  int32_t instance;    /* handle instance that ran it (the grid's new home) */
  double submitted, admitted, finished; /* host steady-clock seconds        */
  acopf_result result; /* as acopf_poll reports it                          */
} acopf_served;

/* Slots per grid for a budget (no device needed): the footprint of an
 * instance is estimated from its sizes (coupling vectors, branch data, state
 * and records, generator and bus arrays, indices, residual history); the
 * homes must fit, then slots are added round robin over the grids, smallest
 * first, up to max_slots each, while the budget allows. slots_out[n_grids],
 * *bytes_used the planned footprint. Errors: EINVAL, EBUDGET (the homes
 * alone exceed budget_bytes). */
int acopf_serving_plan(const acopf_grid* grids, int32_t n_grids, double budget_bytes,
                       int32_t max_slots, int32_t* slots_out, double* bytes_used);

/* Create a server: plan the slots (budget_bytes <= 0: 90% of the device's
 * free memory), create the handle of homes and slots, set its chunk length
 * (iterations between admissions; 0: the default) and one launch lane (its
 * tuning can be changed through acopf_server_info's handle), and solve every
 * home cold to convergence. Grid arrays are borrowed for the call. Errors: EINVAL,
 * EBUDGET, ENOMEM, EDEVICE. */
int acopf_server_create(const acopf_grid* grids, int32_t n_grids, const acopf_params* params,
                        double budget_bytes, int32_t max_slots, int32_t chunk, int32_t device,
                        acopf_server* out);
/* Queue a request for `grid` with new loads pd, qd [that grid's n_bus],
 * copied. Errors: EINVAL (index, null or non-finite loads). */
int acopf_server_submit(acopf_server s, int32_t grid, const double* pd, const double* qd,
                        int64_t request_id);
/* Admit queued requests into free instances, run one chunk of iterations for
 * every request in flight, and retire the finished ones. *in_flight and
 * *queued (nullable) report the requests running and waiting afterwards.
 * Errors: as the handle calls it makes. */
int acopf_server_step(acopf_server s, int32_t* in_flight, int32_t* queued);
/* Move up to max finished requests, oldest first, into out[max]; *n = how
 * many. */
int acopf_server_poll(acopf_server s, acopf_served* out, int32_t max, int32_t* n);
/* Slots per grid and current home instance [n_grids each], the homes' cold
 * solves [n_grids], the planned footprint and the handle (whose state vectors
 * acopf_get_state reads; the server owns it). Every output is nullable. */
int acopf_server_info(acopf_server s, int32_t* slots_per_grid, int32_t* home_instance,
                      acopf_result* cold, double* bytes_used, acopf_handle* handle);
void acopf_server_destroy(acopf_server s);

#ifdef __cplusplus
}
#endif

#endif /* ACOPF_H */
