/*
 * pdlp.h - C ABI of the MI355X (gfx950) PDLP solver.
 *
 * The solver computes an approximate primal-dual solution of the linear program
 *
 *     minimize   c^T x
 *     subject to G x >= h   (the first m1 = m - n_eq rows of K)
 *                A x  = b   (the last n_eq rows of K)
 *                l <= x <= u
 *
 * with K = [G; A] and q = [h; b] (Section 2, problem (1), and its saddle-point form (2)),
 * by the PDHG iteration of Eq. (3) with the paper's enhancements: diagonal preconditioning
 * (Section 3.5), adaptive step sizes (Algorithm 2), adaptive restarts from the normalized
 * duality gap (Section 3.2), and primal-weight updates (Algorithm 3), driven by Algorithm 1.
 * Termination uses the relative KKT criteria of Section 4.1, Eq. (6a)-(6c).
 *
 * All arithmetic runs in IEEE float64 on the GPU.  The iteration needs no host round trip:
 * the host only enqueues work and reads back one small status record per block of
 * check_every accepted steps.
 *
 * Conventions shared by every entry point
 *  - Return value: a pdlp_status.  Negative values are API errors, non-negative values are
 *    solve outcomes.  No C++ exception crosses this boundary.  After an error,
 *    pdlp_last_error() describes it.
 *  - Pointers passed as inputs may be host or device (HIP) pointers; the library inspects
 *    each one.  Inputs are deep-copied: the caller may free them as soon as the call returns.
 *  - Output pointers may be host or device pointers to caller-owned memory of the stated
 *    length; NULL skips that output.
 *  - All device work of a solver is enqueued on the HIP stream given to pdlp_create (NULL =
 *    the default stream).  Every entry point has completed its device work when it returns.
 *  - A solver is not thread-safe: calls on one solver must not overlap.
 */
#ifndef PDLP_H
#define PDLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdlp_solver pdlp_solver;

typedef enum pdlp_status {
  PDLP_OPTIMAL = 0,              /* relative KKT error <= tol (Eq. (6a)-(6c))                 */
  PDLP_ITERATION_LIMIT = 1,      /* iter_limit accepted PDHG steps taken                       */
  PDLP_NUMERICAL_ERROR = 2,      /* non-finite value, or Algorithm 2 rejected max_retries times */
  PDLP_NOT_SOLVED = 3,           /* pdlp_solve has not run yet                                 */
  PDLP_ERR_INVALID_ARGUMENT = -1,
  PDLP_ERR_OUT_OF_MEMORY = -2,
  PDLP_ERR_DEVICE = -3,
  PDLP_ERR_INVALID_STATE = -4
} pdlp_status;

/* Solver options.  pdlp_default_options() fills in the paper's PDLP settings. */
typedef struct pdlp_options {
  int32_t ruiz_iters;            /* Ruiz passes before Pock-Chambolle (Section 3.5): 10       */
  int32_t pock_chambolle;        /* one Pock-Chambolle pass with alpha = 1: 1 (on)            */
  int32_t adaptive_restarts;     /* restart scheme of Section 3.2: 1 (on)                     */
  int32_t primal_weight_update;  /* Algorithm 3 at each restart: 1 (on)                       */
  int32_t check_every;           /* accepted steps between restart/termination checks: 40     */
  int32_t max_retries;           /* rejected attempts in a row that end the solve: 100        */
  int32_t trace_iters;           /* keep scaled (x, y) after each of the first trace_iters
                                    accepted steps (parity testing); 0 = off                  */
  int32_t trace_capacity;        /* ring capacity of the attempt / check logs: 4096           */
  int32_t time_kernels;          /* time every primal/dual step kernel with HIP events: 0    */
  int32_t xcd_panels;            /* XCD column panels for the products: -1 automatic (default:
                                    on for a copy whose gathered vector exceeds 4 MiB and whose
                                    panel rows stay below 0.4 of its nonzeros), 0 off,
                                    1 on whenever the copy has at least one nonzero            */
  double beta_sufficient;        /* restart criterion (i):  0.1 (see the design notes)        */
  double beta_necessary;         /* restart criterion (ii): 0.9                               */
  double beta_artificial;        /* restart criterion (iii): 0.5                              */
  double theta;                  /* primal-weight smoothing of Algorithm 3: 0.5               */
  double primal_importance;      /* multiplies the initial primal weight: 1                   */
  double eps_zero;               /* "small nonzero tolerance" of Section 3.3: 1e-10           */
  int32_t step_policy;           /* 0 adaptive (Algorithm 2, default); 1 constant
                                    eta = 0.9 / ||K~||_2 (the baseline PDHG of Section 2);
                                    2 the Malitsky-Pock line search of Appendix C             */
  int32_t restart_to_current;    /* 1 (default): candidate by GetRestartCandidate; 0: always
                                    the average (Appendix C "adaptive restart (theory)")      */
  int32_t power_iters;           /* power iterations for ||K~||_2 (constant policy): 200     */
  int32_t use_graphs;            /* replay each block of check_every attempts and its check as
                                    a captured HIP graph (one launch instead of one per
                                    kernel): 1 (default); ignored while time_kernels is set   */
  double mp_breaking_factor;     /* Malitsky-Pock (step_policy 2): a trial step eta^ is kept
                                    when eta^ ||K~^T (y^ - y)|| <= this * ||y^ - y||: 1       */
  double mp_downscaling;         /* factor applied to eta^ after a failed trial, in (0,1): 0.5 */
  double mp_interpolation;       /* first trial eta_k + this (sqrt(1+theta_k) - 1) eta_k,
                                    in [0,1]: 0.4 (the paper's best setting)                  */
  int32_t column_order;          /* internal order of the primal variables: -1 automatic (on
                                    exactly when the K~ copy may use XCD panels), 0 the user's
                                    order, 1 within each panel's column range the columns with
                                    the most nonzeros first.  Invisible at this interface:
                                    every n-vector in or out is in the user's order.           */
  int32_t pw_power_of_two;       /* with adaptive_restarts = 0: the "no restart" mode of
                                    Appendix C, which still updates the primal weight
                                    (Algorithm 3, from the current iterate and the previous
                                    update's) at k = 2, 4, 8, ...: 0 (off)                    */
  int32_t lds_gather;            /* operand of a product in panels staged in LDS (one
                                    workgroup of 1024 threads per CU): -1 automatic (default:
                                    the hot-first K~ copy stages each XCD panel's first
                                    lds_entries columns; a copy whose columns keep their order
                                    gets slices of lds_entries columns, one panel each, when
                                    its panel rows stay below 0.4 of its nonzeros, or below
                                    0.7 when it would otherwise be in XCD panels), 0 off,
                                    1 the slices whenever a copy is in panels, 2 XCD panels
                                    with each panel's first lds_entries columns staged.  A
                                    row's run of 513 .. 16384 nonzeros inside one panel is cut
                                    into pieces of 512; never for a copy with a longer run.    */
  int32_t lds_entries;           /* operand entries staged per panel: 0 = 19456 (the most;
                                    152 KiB of LDS), else 1 .. 19456                           */
  int32_t xcd_subpanels;         /* a copy in XCD panels without an LDS stage: each panel's
                                    column range cut into this many equal ranges, which the
                                    XCD's workgroups take one after another, so that fewer
                                    lines of the gathered operand are in use at a time): -1
                                    automatic (default: none while each panel's range of the
                                    operand fits in 1 MiB, else the fewest that keep each
                                    within it, rounded up to an even count, at most 8; used
                                    while the panel rows stay below 0.4 of the nonzeros),
                                    0 or 1 none, 2 .. 8 that many                             */
} pdlp_options;

/* Counters and scalars of a solver (pdlp_get_info). */
typedef struct pdlp_info {
  int32_t status;                /* last pdlp_status of pdlp_solve                            */
  int32_t output_is_average;     /* 1 if the returned point is the restart candidate average  */
  int64_t m, n, n_eq, nnz;
  int64_t iterations;            /* accepted PDHG steps k                                     */
  int64_t attempts;              /* PDHG attempts (accepted + rejected)                       */
  int64_t restarts;              /* outer-loop restarts n                                     */
  int64_t checks;                /* restart/termination checks evaluated                      */
  int64_t spmv_K, spmv_KT;       /* products with K~ and K~^T (2 of them = 1 KKT pass)        */
  double omega;                  /* current primal weight                                     */
  double eta_hat;                /* step size proposed for the next step                      */
  double kkt[4];                 /* relative gap, primal, dual residual and their max at the
                                    returned point (unscaled problem)                         */
  double create_seconds;         /* host wall time of pdlp_create (copy, transpose, scaling)  */
  double solve_seconds;          /* host wall time of the last pdlp_solve                     */
  double step_bytes;             /* algorithmic HBM bytes of one accepted PDHG step           */
  int32_t layout_K, layout_KT;   /* layout of the K~ and K~^T copies: 0 plain rows, 1 XCD column
                                    panels, 2 LDS slices (every gather from LDS), 3 XCD panels
                                    with each panel's first columns staged in LDS              */
  int32_t panels_K, panels_KT;   /* column panels of each copy (1 in the plain layout)         */
} pdlp_info;

/* Scalars of a checkpoint (pdlp_get_state / pdlp_set_state). */
typedef struct pdlp_state {
  int64_t k;                     /* accepted steps                                            */
  int64_t t;                     /* accepted steps since the last restart                     */
  int64_t n_outer;               /* restarts so far                                           */
  double eta_hat;                /* step size the next step starts from                       */
  double omega;                  /* primal weight                                             */
  double s_eta;                  /* sum of the steps of the iterates in the average           */
  double mu_prev;                /* candidate gap at the previous check (+inf after a restart)*/
  double mu_anchor;              /* gap of the anchor vs the previous anchor (+inf before the
                                    first restart)                                            */
} pdlp_state;

/* One Algorithm-2 attempt, as logged by the solver. */
typedef struct pdlp_attempt_rec {
  int64_t k;                     /* accepted steps before this attempt                        */
  double eta;                    /* step size tried                                           */
  double eta_bar;                /* the largest step Eq. (5) allows (+inf if dy^T K dx = 0)   */
  int32_t accepted;
  int32_t pad;
} pdlp_attempt_rec;

/* One restart/termination check (Algorithm 1 at k = multiple of check_every). */
typedef struct pdlp_check_rec {
  int64_t k;
  double mu_cur;                 /* normalized gap of the current iterate vs the anchor       */
  double mu_avg;                 /* normalized gap of the average vs the anchor               */
  double kkt;                    /* relative KKT error of the candidate                       */
  double omega_after;            /* primal weight after this check                            */
  double mu_anchor;              /* gap of the new anchor vs the old one (after a restart)    */
  int32_t use_avg;               /* candidate = average (1) or current iterate (0)            */
  int32_t mask;                  /* restart criteria met: 1 = (i), 2 = (ii), 4 = (iii)        */
  int32_t terminated;
  int32_t pad;
} pdlp_check_rec;

/* Fills *opts with the defaults listed in pdlp_options. */
void pdlp_default_options(pdlp_options *opts);

/*
 * pdlp_create - validate and copy an LP onto the GPU and precondition it.
 *   out        receives the new solver (NULL on failure).
 *   m, n, n_eq K is m x n; its last n_eq rows are equalities, the first m - n_eq ">=" rows.
 *              Requires n >= 1, m >= 0, 0 <= n_eq <= m, m and n below 2^31.
 *   c          n costs;  q  m right-hand sides [h; b];  l, u  n bounds, +-INFINITY allowed.
 *   row_ptr    m + 1 row offsets of K (int64, row_ptr[0] = 0, non-decreasing).
 *   col_idx    row_ptr[m] column indices (int32), strictly increasing within each row.
 *   val        row_ptr[m] finite values.
 *   opts       NULL = pdlp_default_options().
 *   hip_stream hipStream_t for all work of this solver, NULL = default stream.
 * Errors: PDLP_ERR_INVALID_ARGUMENT for bad sizes, non-finite c, q or values, NaN bounds,
 * l > u, l = +inf or u = -inf, column indices out of range, unsorted or duplicated within a
 * row; PDLP_ERR_OUT_OF_MEMORY; PDLP_ERR_DEVICE for HIP failures.
 * The LP is stored twice in CSR (K~ and a transposed copy K~^T, both preconditioned), so the
 * device holds about 24 * nnz + 8 * (m + n) * 30 bytes.
 */
int pdlp_create(pdlp_solver **out, int64_t m, int64_t n, int64_t n_eq, const double *c,
                const int64_t *row_ptr, const int32_t *col_idx, const double *val,
                const double *q, const double *l, const double *u,
                const pdlp_options *opts, void *hip_stream);

/*
 * pdlp_solve - run Algorithm 1 until the relative KKT error of a checked point is <= tol,
 * iter_limit accepted steps have been taken (counted from creation), or a numerical error.
 * A later call continues from the current state with the new tol and iter_limit.
 * Returns the pdlp_status of the solve (or an API error).
 */
int pdlp_solve(pdlp_solver *s, double tol, int64_t iter_limit);

/*
 * pdlp_get - the returned point of the last solve, in the user's (unscaled) variables:
 * x (n values), y (m values) and kkt (4 values: relative gap, primal residual, dual
 * residual, max).  PDLP_ERR_INVALID_STATE before the first pdlp_solve.
 */
int pdlp_get(const pdlp_solver *s, double *x, double *y, double *kkt);

/* pdlp_get_info - counters and scalars; see pdlp_info. */
int pdlp_get_info(const pdlp_solver *s, pdlp_info *info);

/* pdlp_destroy - free a solver and all its device memory.  NULL is allowed. */
void pdlp_destroy(pdlp_solver *s);

/* pdlp_last_error - text of the last error of s (or of the last failed pdlp_create when s is
 * NULL).  Owned by the library, valid until the next call on s. */
const char *pdlp_last_error(const pdlp_solver *s);

/* pdlp_set_host_threads - host threads of the preparation work of the next pdlp_create calls
 * in this process (transpose, column order, panel layouts, interleaved entries): n >= 1, or 0
 * for the default (the hardware threads, at most 16).  The prepared data, and so every result,
 * are the same for any n.  Returns the count now in effect.  Not for calls that overlap a
 * pdlp_create on another thread. */
int pdlp_set_host_threads(int n);

/* ---- batched solve: many independent LPs in one launch ----------------------------------- */

typedef struct pdlp_batch pdlp_batch;

/*
 * pdlp_batch_create - a batch of `count` independent LPs of the form above, solved later in one
 * persistent launch with one GPU workgroup per LP; every LP has its own preconditioning, step
 * size, primal weight, restart state and termination (the method of Section 3 applied to each).
 *   m, n, n_eq   count sizes each (as in pdlp_create, per member).
 *   c, l, u      members' n-vectors concatenated in member order (sum of n values).
 *   q            members' m-vectors concatenated (sum of m values).
 *   row_ptr      members' CSR row offsets concatenated (sum of m + 1 values; each member's
 *                offsets start at 0 and index that member's nonzeros).
 *   col_idx, val members' nonzeros concatenated (member-local column indices).
 *   opts         as in pdlp_create (the same ranges are checked), with step_policy 0 (adaptive)
 *                and pw_power_of_two 0 (the "no restart" weight events are not implemented
 *                here); traces, kernel timing, panels and graphs do not apply.
 * Inputs are deep-copied; host or device pointers.  Errors as pdlp_create (the message names
 * the first invalid member).
 */
int pdlp_batch_create(pdlp_batch **out, int64_t count, const int64_t *m, const int64_t *n,
                      const int64_t *n_eq, const double *c, const int64_t *row_ptr,
                      const int32_t *col_idx, const double *val, const double *q,
                      const double *l, const double *u, const pdlp_options *opts,
                      void *hip_stream);

/* pdlp_batch_solve - solve every member to relative KKT error tol or iter_limit accepted
 * steps (each member separately).  Every call starts from the members' data as created (a
 * later call repeats the solve, with its own tol and iter_limit).
 * The members fall into PDLP_BATCH_CLASSES size classes by nonzeros ([0, 2^11), [2^11, 2^13),
 * [2^13, 2^15), [2^15, ...)); each class runs as one persistent launch, members largest first,
 * classes concurrently, with the schedule set for that class: the threads per member (64, 128,
 * 256, 512 or 1024) and the rows per thread whose products are in flight together (1 or 2;
 * 2 only with 128, 256 or 512 threads).  Until pdlp_batch_tune or pdlp_batch_set_schedule,
 * every class runs 256 threads x 1 row. */
#define PDLP_BATCH_CLASSES 4
int pdlp_batch_solve(pdlp_batch *b, double tol, int64_t iter_limit);

/* pdlp_batch_tune - pick each class's schedule: every candidate (64x1, 128x1, 128x2, 256x1,
 * 256x2, 512x1, 512x2, 1024x1 threads x rows) runs the class's members for `steps` accepted
 * steps (tol 0, so none stops early; timed with HIP events after one untimed run) and the
 * fastest is kept.  threads, rows (may be NULL) receive the PDLP_BATCH_CLASSES choices.  The
 * timing runs leave no solve behind (pdlp_batch_get needs a pdlp_batch_solve after it).
 * Errors: PDLP_ERR_INVALID_ARGUMENT for steps < 1. */
int pdlp_batch_tune(pdlp_batch *b, int64_t steps, int32_t *threads, int32_t *rows);

/* pdlp_batch_set_schedule - set the PDLP_BATCH_CLASSES schedules (threads[c] x rows[c], one
 * of the candidates of pdlp_batch_tune; else PDLP_ERR_INVALID_ARGUMENT). */
int pdlp_batch_set_schedule(pdlp_batch *b, const int32_t *threads, const int32_t *rows);

/* pdlp_batch_schedule - the current schedule and the member count of each class
 * (PDLP_BATCH_CLASSES values each; any pointer may be NULL). */
int pdlp_batch_schedule(const pdlp_batch *b, int32_t *threads, int32_t *rows, int64_t *members);

/* pdlp_batch_tune_seconds - host wall time of the last pdlp_batch_tune. */
double pdlp_batch_tune_seconds(const pdlp_batch *b);

/* pdlp_batch_get - returned points, unscaled and concatenated like the inputs (x: sum of n,
 * y: sum of m), and per member the pdlp_status, accepted steps and kkt[4] (4 * count values).
 * Any pointer may be NULL. */
int pdlp_batch_get(const pdlp_batch *b, double *x, double *y, int32_t *status,
                   int64_t *iterations, double *kkt);

/* pdlp_batch_solve_seconds - host wall time of pdlp_batch_solve (launch to completion). */
double pdlp_batch_solve_seconds(const pdlp_batch *b);

void pdlp_batch_destroy(pdlp_batch *b);
const char *pdlp_batch_last_error(const pdlp_batch *b);

/* ---- unrolled PDHG and its adjoint (differentiating through a fixed number of steps) ------- */

/* Scalars of the last unrolled forward / backward pass (pdlp_unroll_get_info). */
typedef struct pdlp_unroll_info {
  int64_t steps;                 /* T of the last pdlp_unroll_forward                          */
  int64_t segment;               /* steps per checkpoint segment                               */
  int64_t checkpoints;           /* ceil(T / segment) stored iterates                          */
  int64_t recomputed_steps;      /* forward steps the last backward pass recomputed            */
  double eta;                    /* frozen step size used (preconditioned problem)             */
  double omega;                  /* frozen primal weight used                                  */
  double forward_seconds;        /* host wall time of the last forward / backward call         */
  double backward_seconds;
  double device_bytes;           /* device memory the solver allocated for its own unroll buffers
                                    (0 while only pdlp_unroll_forward_noalloc has run)          */
  int32_t ready;                 /* 1 if a forward pass can be differentiated                  */
  int32_t pad;
} pdlp_unroll_info;

/*
 * pdlp_unroll_forward - T = steps iterations of Eq. (3) on the solver's preconditioned LP with
 * new objective c and right-hand side q, a fixed step eta and primal weight omega
 * (tau = eta / omega, sigma = eta * omega) and the solver's frozen D1, D2: no restarts, no
 * step-size rule, no rejections.  Starts at x0 = proj_[l,u](0), y0 = 0 (Section 4.1's start).
 * This is the map that a network with an LP "optimization layer" differentiates, the use of
 * GPU PDLP that the introduction (Section 1) mentions; the paper itself gives no derivative.
 *   c, q      n and m values in the user's units (c~ = D2 c, q~ = D1 q); NULL = the LP's own.
 *   steps     T >= 0.
 *   segment   steps between stored checkpoints of (x, y, K~ x): 0 = one segment (no
 *             recomputation in the backward pass, most memory), else at most ceil(T/segment)
 *             checkpoints of n + 2m values plus segment * (n + m) bytes of projection masks.
 *   eta       <= 0: 0.9 / ||K~||_2 from power iteration (the baseline step of Section 2).
 *   omega     <= 0: the initial primal weight of Section 3.3 from the LP's own c~, q~.
 *   x_T, y_T  outputs (n, m values, user's units x = D2 x~, y = D1 y~); NULL skips.
 * The solver keeps what pdlp_unroll_backward needs until the next forward call.  The unroll
 * uses its own buffers: it neither reads nor changes the state of pdlp_solve.
 * Errors: PDLP_ERR_INVALID_ARGUMENT (negative steps or segment, non-finite eta or omega),
 * PDLP_ERR_OUT_OF_MEMORY, PDLP_ERR_DEVICE.
 */
int pdlp_unroll_forward(pdlp_solver *s, const double *c, const double *q, int64_t steps,
                        int64_t segment, double eta, double omega, double *x_T, double *y_T);

/*
 * pdlp_unroll_backward - reverse mode of the last pdlp_unroll_forward: given gx_T = dL/dx_T
 * (n values) and gy_T = dL/dy_T (m values; either may be NULL = 0), writes gc = dL/dc (n) and
 * gq = dL/dq (m) in the user's units.  eta, omega, D1, D2, l and u are held constant.  Where a
 * projection is active the derivative of the clamp is taken as 0 (strictly inside the bounds,
 * and y > 0 on ">=" rows, it is 1).  Segments other than the last are recomputed from their
 * checkpoints; the result is identical to storing every step.  May be called several times.
 * Errors: PDLP_ERR_INVALID_STATE without a forward pass; as pdlp_unroll_forward otherwise.
 */
int pdlp_unroll_backward(pdlp_solver *s, const double *gx_T, const double *gy_T, double *gc,
                         double *gq);

/*
 * pdlp_unroll_forward_noalloc - pdlp_unroll_forward for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc).  Same arguments, result and
 * errors as pdlp_unroll_forward, and the same kernels; it calls no hipMalloc, hipFree or other
 * allocating routine.  The unroll's buffers (staging of c and q, the running iterate, the
 * ceil(T/segment) checkpoints of n + 2m values, segment * (n + m) bytes of projection masks,
 * the adjoints) are carved from a per-GPU scratch array of 64 MiB that the library holds from
 * its load until the process ends, instead of the solver's own buffers.  Requests whose
 * buffers exceed 64 MiB (about 8 (7 (n + m) + nseg (n + 2m)) + segment (n + m) bytes) fail with
 * PDLP_ERR_INVALID_ARGUMENT before any device work.  The solver itself must exist (its
 * pdlp_create allocates, once).
 * Sharing: every no-alloc call on one GPU uses the same array and leaves its contents there.
 * pdlp_unroll_backward after this call reads them, and fails with PDLP_ERR_INVALID_STATE if
 * another no-alloc forward on that GPU (on any solver) has claimed the array since.  Calls
 * that overlap in time on one GPU (from several host threads) race and must be serialized by
 * the caller.
 */
int pdlp_unroll_forward_noalloc(pdlp_solver *s, const double *c, const double *q, int64_t steps,
                                int64_t segment, double eta, double omega, double *x_T,
                                double *y_T);

/* pdlp_unroll_get_info - see pdlp_unroll_info. */
int pdlp_unroll_get_info(const pdlp_solver *s, pdlp_unroll_info *info);

/* ---- inspection entry points (parity tests and measurement) ---------------------------- */

/*
 * pdlp_get_state - checkpoint of Algorithm 1 before its next step, in the preconditioned
 * variables: the iterate x~ (n values), y~ (m), the anchor z^{n,0} xa (n), ya (m), the
 * step-weighted sums of the iterates since the last restart sx (n), sy (m) (the average is
 * sx / s_eta), and the scalars in *st.  Any pointer may be NULL.
 */
int pdlp_get_state(const pdlp_solver *s, double *x, double *y, double *xa, double *ya,
                   double *sx, double *sy, pdlp_state *st);

/*
 * pdlp_set_state - resume Algorithm 1 from a checkpoint with the layout of pdlp_get_state
 * (all six vectors and st are required).  The next pdlp_solve continues from it without a
 * new termination check at its start.  Used for warm starts and for replaying single steps.
 * Under the Malitsky-Pock policy the line search resumes with theta = 1 and eta_hat as its
 * last accepted step.
 */
int pdlp_set_state(pdlp_solver *s, const double *x, const double *y, const double *xa,
                   const double *ya, const double *sx, const double *sy, const pdlp_state *st);

/* pdlp_get_scaling - the diagonal preconditioners: D1 (m values) and D2 (n values), with
 * K~ = D1 K D2 (Section 3.5). */
int pdlp_get_scaling(const pdlp_solver *s, double *D1, double *D2);

/* pdlp_get_iterate - the current iterate z^{n,t} in the preconditioned variables
 * (x~ = x / D2: n values, y~ = y / D1: m values). */
int pdlp_get_iterate(const pdlp_solver *s, double *x_scaled, double *y_scaled);

/*
 * pdlp_get_trace - the solver's logs since creation.
 *   att / att_cap / n_att   attempt records (the last att_cap are kept in the ring);
 *   chk / chk_cap / n_chk   check records;
 *   xs, ys                  scaled iterates after accepted steps 1..n_iter (n_iter <= trace_iters),
 *                           stored row-wise: xs[(k-1)*n + j], ys[(k-1)*m + i].
 * Any pointer may be NULL.  n_att / n_chk receive the total number logged (may exceed the cap).
 */
int pdlp_get_trace(const pdlp_solver *s, pdlp_attempt_rec *att, int64_t att_cap, int64_t *n_att,
                   pdlp_check_rec *chk, int64_t chk_cap, int64_t *n_chk,
                   double *xs, double *ys, int64_t *n_iter);

/* pdlp_spmv - out = K~ x (transpose = 0; x: n values, out: m values) or out = K~^T x
 * (transpose = 1; x: m values, out: n values) with the solver's preconditioned matrix and
 * the same kernels the iteration uses.  x and out are device pointers. */
int pdlp_spmv(pdlp_solver *s, int transpose, const double *x, double *out);

/* pdlp_kernel_times - with options.time_kernels set, the summed HIP-event time in ms and
 * the count of the attempt slots that ran, for the primal step (K~^T product fused with the
 * primal update: times[0], counts[0]) and the dual step (K~ product fused with the dual update
 * and the step-size rule: times[1], counts[1]) over all solves since the last reset.  A slot
 * runs when its attempt does; slots left idle by a pending check, the end of the solve or
 * the iteration limit are not counted.  With time_kernels the solver runs one block at a
 * time and without graphs, and a block stops at the iteration limit instead of idling. */
int pdlp_kernel_times(const pdlp_solver *s, double *times_ms, int64_t *counts);

/* pdlp_set_kernel_timing - turn kernel timing (options.time_kernels) on (1) or off (0) for
 * the next solves of s.  The arithmetic is the same either way; with it off, whole blocks
 * replay as captured graphs again (options.use_graphs). */
int pdlp_set_kernel_timing(pdlp_solver *s, int on);

/* pdlp_pass_times - the same split into four passes (times_ms[4], counts[4]): the primal
 * first pass (the K~^T product, or its panel pass), the primal combine (the panel partials
 * added and the primal update; 0 in the plain layout, where one kernel does both), the dual
 * first pass and the dual combine (with the step-size tail). */
int pdlp_pass_times(const pdlp_solver *s, double *times_ms, int64_t *counts);

/* pdlp_reset_kernel_times - zero the counters of pdlp_kernel_times. */
int pdlp_reset_kernel_times(pdlp_solver *s);

/*
 * pdlp_build_schedule - host-only (no GPU needed): the work schedule the CSR products use
 * for a matrix with nrows rows and offsets row_ptr.  Rows of at most 512 nonzeros are
 * grouped by the lane count L = 2^p (the smallest with length <= 8 L), ordered by length
 * within a group, and listed in *perm (nrows entries at most, may be NULL); a wavefront task
 * {a, b, 0 | p << 8, E} covers rows perm[a .. a + b), E (1..8) entries per lane, E L >= the
 * longest of those rows.  Longer rows get workgroup tasks {row, 0, 1, 0}; rows above 16384
 * nonzeros are cut into chunks {row, chunk, 2, split id}.  Writes up to cap tasks of four
 * int32 (wavefront tasks first) to desc and sets *ndesc (all tasks) and *nsplit.
 */
int pdlp_build_schedule(const int64_t *row_ptr, int64_t nrows, int32_t *desc, int64_t cap,
                        int64_t *ndesc, int64_t *nsplit, int32_t *perm);

/* The column-panel form of a CSR copy as the products read it (pdlp_build_panel_layout).
 * Counts are set by a call with prow_ptr NULL; a second call with every array allocated by
 * the caller (the counts below give their lengths; any array may be NULL to skip it) fills
 * them, and fails if the counts no longer match. */
typedef struct pdlp_panel_layout {
  int64_t nprow;        /* panel rows (row r restricted to panel p, nonempty)                */
  int64_t nwave;        /* wavefront tasks                                                     */
  int64_t nblock;       /* workgroup tasks (panel rows longer than 512 nonzeros)               */
  int64_t nslots;       /* interleaved slots of the wavefront tasks                            */
  int64_t nseg;         /* LDS segments                                                        */
  int32_t *cut;         /* npanel + 1: column offsets of the panels                            */
  int64_t *prow_ptr;    /* nprow + 1: offsets of each panel row's nonzeros (panel order)       */
  int32_t *prow_row;    /* nprow: original row of each panel row                               */
  int64_t *src;         /* nnz: index in the input CSR of each panel-ordered nonzero           */
  int64_t *slot_ptr;    /* nrows + 1: panel rows of row r at slot_idx[slot_ptr[r] ..]          */
  int32_t *slot_idx;    /* nprow: panel rows of each row, in panel order                       */
  int32_t *wave;        /* 4 nwave: {first panel row, rows, log2(lanes) << 8, entries per lane} */
  int32_t *wave_begin;  /* npanel + 1: first wavefront task of each panel                      */
  int64_t *task_off;    /* nwave + 1: first interleaved slot of each wavefront task            */
  int32_t *cis;         /* nslots: interleaved columns (round i of task t from task_off[t] +
                           64 E i; entry k of lane j at 64 k + j)                             */
  double *vs;           /* nslots: interleaved values (0 in padding slots)                     */
  int32_t *seg_ptr;     /* groups + 1: segments of each LDS workgroup                          */
  int32_t *seg;         /* 4 nseg: {panel, first task, end task, 0}                             */
} pdlp_panel_layout;

/*
 * pdlp_build_panel_layout - host-only (no GPU needed): the panel layout the products use for
 * the nrows x ncols CSR matrix (row_ptr, col_idx, val): npanel panels cut at `cuts` (npanel
 * + 1 column offsets) or, if cuts is NULL, at about equal nonzero counts; wavefront tasks of
 * at most emax entries per lane (8, or 16 as in the layouts of the LDS-staged products); its
 * interleaved entries (with emax 16, the layouts of the LDS-staged kernel, a row's run of 513 to
 * 16384 entries inside one panel is cut into consecutive panel rows of at most 512 entries);
 * and the split of its wavefront tasks among `groups` LDS workgroups
 * (aligned: group b stays on panel b mod npanel, which needs groups to be a multiple of
 * npanel).  Returns 0, or -1 on invalid arguments (including a matrix that is not CSR with
 * in-range, increasing columns per row, or cuts that are not non-decreasing from 0 to ncols)
 * or mismatched counts.
 */
int pdlp_build_panel_layout(const int64_t *row_ptr, const int32_t *col_idx, const double *val,
                            int64_t nrows, int64_t ncols, int32_t npanel, const int32_t *cuts,
                            int32_t emax, int32_t groups, int32_t aligned, pdlp_panel_layout *out);

#ifdef __cplusplus
}
#endif

#endif /* PDLP_H */
