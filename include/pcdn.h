/*
 * pcdn.h -- C ABI of the MI355X (gfx950) PCDN library.
 *
 * Parallel Coordinate Descent Newton (Bian, Li, Liu, Yang, arXiv:1306.4080)
 * for L1-regularised loss minimisation (Sec. 2, eq. (1)):
 *
 *     min_w  F(w) = C * sum_{i<n} phi(w; x_i, y_i) + ||w||_1,   w in R^p,
 *
 * with the logistic loss phi = log(1 + exp(-y w^T x)) (eq. (2)) or the L2 hinge
 * loss phi = max(0, 1 - y w^T x)^2 (eq. (3)).  The paper writes s samples and
 * n features; this interface writes n samples and p features.
 *
 * Conventions shared by every entry point:
 *  - Return codes: PCDN_OK (0) on success, PCDN_NOT_CONVERGED (1) when a solve
 *    stopped at max_outer, a negative PCDN_E_* code on error.  After an error
 *    pcdn_last_error() describes it; the context stays usable unless the code
 *    is PCDN_E_DEVICE.
 *  - No exception crosses the ABI.  A context is not thread-safe: use one per
 *    host thread.  Work runs on the context's HIP stream, except that the
 *    multi-problem drivers (and pcdn_solve / pcdn_iterate on the heavy-bundle
 *    path of the automatic schedule) also launch on streams of their own,
 *    ordered after the context stream's earlier work; every entry point that
 *    returns host data synchronises all of them before returning.
 *  - Host arrays are borrowed for the duration of the call only.  The library
 *    owns every device buffer it allocates and frees them in pcdn_destroy().
 *  - Layouts: X is compressed sparse column (CSC).  Column j holds rows
 *    row_idx[col_ptr[j] .. col_ptr[j+1]) in strictly increasing order with
 *    values val[...]; labels y[i] are +1 or -1.
 */
#ifndef PCDN_H
#define PCDN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcdn_ctx pcdn_ctx;

/* Loss selector: eq. (2) or eq. (3). */
typedef enum { PCDN_LOSS_LOGISTIC = 0, PCDN_LOSS_L2SVM = 1 } pcdn_loss;

enum {
  PCDN_OK = 0,
  PCDN_NOT_CONVERGED = 1,
  PCDN_E_ARG = -1,     /* invalid argument (sizes, C, P, eps, loss, bundle) */
  PCDN_E_CSC = -2,     /* malformed CSC, non-finite value or label not +-1  */
  PCDN_E_OOM = -3,     /* device allocation failed                          */
  PCDN_E_DEVICE = -4,  /* HIP runtime error                                 */
  PCDN_E_STATE = -5,   /* call out of order (no data loaded, no state set)  */
  PCDN_E_NUMERIC = -6  /* NaN reached the objective, or a retained quantity
                          left its range (e^{w^T x_i} not a positive normal
                          double, |w^T x_i| above about 708; b_i not finite) */
};

/* Options.  A zero-filled struct (or NULL) selects the paper's settings:
 * sigma = 0.01, beta = 0.5, gamma = 0 (Sec. 5.1), nu = 1e-12 (Hessian floor,
 * proof of Lemma 1(b)), max_outer = 1000, max_ls = 30, seed = 0, w0 = 0
 * (Algorithm 3 starts from zero). */
typedef struct {
  uint64_t seed;        /* seeds the per-outer-iteration feature partition  */
  int32_t max_outer;    /* outer iterations at most (0: 1000)               */
  int32_t max_ls;       /* backtracking steps q = 0..max_ls-1 (0: 30; <=32) */
  double sigma;         /* Armijo sigma in (0,1) (0: 0.01)                  */
  double beta;          /* backtracking factor in (0,1) (0: 0.5)            */
  double gamma;         /* Delta's Hessian weight in [0,1) (0 is valid)     */
  double nu;            /* floor added to a Hessian entry <= 0 (0: 1e-12)   */
  const double* w0;     /* host, p entries, warm start; NULL: zeros         */
  int32_t schedule;     /* PCDN_SCHED_*: how bundles map onto the GPU       */
  int32_t shrink;       /* 1: outer-iteration shrinking (below); 0: off     */
  int32_t penalty;      /* PCDN_PENALTY_*: the regulariser (below)          */
  int32_t chunk;        /* nonzeros per wavefront range of the WIDE
                           schedule's bundle sweep: a bundle's nonzeros in
                           partition order are cut into ranges of `chunk`
                           (a column of L nonzeros spans about L / chunk
                           wavefronts; 0: 256; 64, 128, 256 or 512).  It
                           fixes the order of the g_j, h_j sums            */
  double l2;            /* ridge weight b of ELASTIC and L2 (> 0); 0 for L1 */
} pcdn_opts;

/* Regulariser.  Eq. (1) is F(w) = ||w||_1 + C sum_i phi_i; the paper's
 * conclusion extends PCDN to any separable regulariser.  With
 * R(w) = sum_j a |w_j| + (b/2) w_j^2 in place of ||w||_1 in F, in the
 * one-dimensional subproblem (eq. (4)), in Delta (eq. (7)) and in the Armijo
 * test (eq. (6)):
 *   PCDN_PENALTY_L1       a = 1, b = 0   (eq. (1); default)
 *   PCDN_PENALTY_ELASTIC  a = 1, b = l2  (elastic net)
 *   PCDN_PENALTY_L2       a = 0, b = l2  (ridge).
 * The direction keeps eq. (5)'s form: d = -(g + a + b w)/(h + b) if
 * g + a <= h w, -(g - a + b w)/(h + b) if g - a >= h w, else -w (g, h are
 * the loss term's, as pcdn_step reports them).  The stopping rule uses the
 * minimum-norm subgradient of this F, and shrinking's threshold is a - M/n
 * (nothing is left out for ridge).  Other values of penalty, l2 != 0 with L1,
 * or l2 <= 0 otherwise: PCDN_E_ARG. */
enum { PCDN_PENALTY_L1 = 0, PCDN_PENALTY_ELASTIC = 1, PCDN_PENALTY_L2 = 2 };

/* Shrinking (opt-in; the paper shrinks between outer iterations, not inside
 * the parallel loop, and gives no rule): after outer iteration k, feature j
 * stays active for iteration k+1 iff w_j != 0 or |g_j| >= 1 - M_{k-1}/n,
 * where M_{k-1} is the largest minimum-norm subgradient after iteration k-1
 * (infinite before the first, so the first two iterations use every
 * feature).  Iteration k+1 partitions only the active features: the seeded
 * permutation restricted to them (inactive features sort last), bundles of P.
 * The stopping rule still uses every feature; a feature is only left out
 * while its minimum-norm subgradient is 0.  pcdn_reset and pcdn_solve start
 * with every feature active; pcdn_iterate continues the current active set.
 * pcdn_step ignores it. */

/* Bundle schedules (same arithmetic, different launch structure):
 *  WIDE:   every bundle is four kernels over the whole GPU (many nonzeros);
 *  NARROW: one workgroup runs all bundles of an outer iteration (small
 *          bundles, where kernel-boundary latency would dominate);
 *  AUTO:   NARROW when the average bundle holds few nonzeros, else WIDE;
 *          under NARROW, when a bundle can hold 4,096 nonzeros or more
 *          (long columns), pcdn_solve, pcdn_iterate and each solve of
 *          pcdn_solve_path run in the rounds of the batch engine
 *          (pcdn_solve_batch), which reads each partition's list of such
 *          bundles and runs them as WIDE between single-workgroup segments
 *          (with kernel profiling on, direct launches that do the same). */
enum { PCDN_SCHED_AUTO = 0, PCDN_SCHED_WIDE = 1, PCDN_SCHED_NARROW = 2 };

/* Per-solve report. */
typedef struct {
  int32_t outer_iters;  /* outer iterations run                             */
  int32_t converged;    /* 1 if the stopping rule held                      */
  int64_t bundles;      /* inner iterations (bundles) run                   */
  int64_t ls_steps;     /* line-search candidates tested, q+1 per bundle    */
  int64_t ls_fail;      /* bundles whose search found no step (w unchanged) */
  int64_t nnz_swept;    /* sum over bundles of the bundle's nonzeros        */
  double objective;     /* F(w) at exit, from the retained quantities       */
  double subgrad;       /* ||grad^S F(w)||_1 at exit                        */
  double subgrad0;      /* ||grad^S F(0)||_1, the stopping reference        */
  double alg_bytes;     /* algorithmic HBM bytes of the kernels run         */
  double seconds;       /* wall time of the solve (stream-synchronised)     */
  /* How close the solve's decisions came to their thresholds (a decision at
   * the rounding floor can fall either way between two summation orders):
   * the smallest |dF - sigma Delta_q| / S of any Armijo test (eq. (6)),
   * S = |sigma Delta_q| plus the rounding scales of the terms dF is summed
   * from (for R_j(w + s) - R_j(w) the magnitudes it is the difference of;
   * for a logistic loss change its size plus |its argument|; for a squared-
   * hinge change the two squares plus 2 max(0, b') |argument|), and the
   * smallest |G_k - eps G0| / (eps G0) of any stopping test; +inf when
   * there was none. */
  double min_armijo_margin;
  double min_stop_margin;
  /* The schedule and chunk the solve ran with (PCDN_SCHED_*; nonzeros per
   * wavefront range of the bundle sweep): the options' values, or the autotuner's for a batch job
   * with P = 0.  Passing them back reproduces the solve bit for bit. */
  int32_t schedule;
  int32_t chunk;
} pcdn_info;

/* Per-inner-iteration report of pcdn_step(). */
typedef struct {
  double alpha;   /* accepted step beta^q, 0 when no q < max_ls passed      */
  double delta;   /* Delta of the Armijo rule (eq. (7))                     */
  double dF;      /* F(w + alpha d) - F(w) from retained quantities, eq. (10) */
  int32_t q;      /* accepted backtracking index, -1 if none                */
  int32_t pad;
} pcdn_step_info;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * run on (borrowed; it must outlive the context) or NULL for a stream the
 * library creates.  *out receives the context, or NULL on error. */
int pcdn_create(pcdn_ctx** out, int device, void* hip_stream);

/* Load (copy) the design matrix and labels, replacing any previous data.
 * n, p >= 1 and < 2^31; nnz >= 0.  ptr_kind 0: the four arrays are host
 * pointers; 1: device pointers on the context's device.  The CSC is validated
 * (col_ptr[0] = 0, non-decreasing, col_ptr[p] = nnz, rows in range and
 * strictly increasing per column, finite values, y in {-1,+1}); on failure
 * nothing is replaced and PCDN_E_CSC is returned. */
int pcdn_load_csc(pcdn_ctx* ctx, int64_t n, int64_t p, int64_t nnz,
                  const int64_t* col_ptr, const int32_t* row_idx,
                  const float* val, const int8_t* y, int ptr_kind);

/* pcdn_load_csc of X with a bias feature appended: column p (the last of
 * p + 1) holds the value `bias` (finite, non-zero) in every row, and its
 * weight is regularised like every other coordinate (the bias term of the
 * paper's logistic-regression experiments, Sec. 5.2).  w then has p + 1
 * entries, the bias weight last.  Same checks and ownership as
 * pcdn_load_csc. */
int pcdn_load_csc_bias(pcdn_ctx* ctx, int64_t n, int64_t p, int64_t nnz,
                       const int64_t* col_ptr, const int32_t* row_idx,
                       const float* val, const int8_t* y, int ptr_kind, float bias);

/* Algorithm 3 (PCDN) with Algorithm 4's line search on the loaded data:
 * for outer iteration k the features are split by a seeded uniform random
 * permutation into ceil(p/P) bundles of P (the last may be smaller), each
 * bundle takes one P-dimensional approximate Newton step with Armijo
 * backtracking.  Stops after the outer iteration at which
 * ||grad^S F(w)||_1 <= eps * ||grad^S F(0)||_1 (the paper fixes only that its
 * rule resembles newGLMNET's outer test) or at max_outer.  C > 0,
 * 1 <= P <= p, eps >= 0.  w_out (host, p doubles, nullable) receives w;
 * info (nullable) the report.  Returns PCDN_OK or PCDN_NOT_CONVERGED.  The
 * final state stays on the device for pcdn_get_w() and pcdn_step(). */
int pcdn_solve(pcdn_ctx* ctx, double C, int64_t P, double eps, int loss,
               const pcdn_opts* opts, double* w_out, pcdn_info* info);

/* One solve of a batch: the arguments of pcdn_solve for one context. */
typedef struct {
  pcdn_ctx* ctx;          /* loaded context; at most one job per context       */
  double C;               /* as pcdn_solve                                     */
  int64_t P;              /* as pcdn_solve; 0: chosen by pcdn_autotune first
                             (and written back)                                */
  double eps;
  int32_t loss;
  int32_t status;         /* out: what pcdn_solve would have returned          */
  const pcdn_opts* opts;  /* nullable: defaults                                */
  double* w_out;          /* nullable: host, p doubles                         */
  pcdn_info* info;        /* nullable                                          */
} pcdn_job;

/* Independent solves together on one device (the contexts must share it).
 * Each job follows the trajectory pcdn_solve would (same partitions, same
 * arithmetic; Algorithm 3 per problem).  The jobs advance in rounds of one
 * outer iteration each: the bundles of every job on the single-workgroup
 * schedule run in one launch, one workgroup per job (their partition and
 * stopping sweeps are replayed graphs on each context's stream); a job whose
 * bundles include heavy ones (automatic schedule) runs its segments and
 * heavy bundles as a chain of launches on a stream of the batch; jobs on the
 * multi-kernel schedule run their whole outer iteration (partition included)
 * as tasks of lock-step multi-problem launches, launch s running task s of
 * every such job with the grid of its own launch.  A job leaves the batch when its
 * stopping rule holds or at its max_outer.  Arguments are checked for every
 * job before any work: an invalid job makes the call return that job's error
 * code (its context holds the message) with nothing run.  Otherwise returns
 * PCDN_OK, with each job's PCDN_OK / PCDN_NOT_CONVERGED in jobs[i].status, or
 * the first device error.  count = 0 is allowed.  Kernel profiling
 * (pcdn_profile) does not bracket batch launches. */
int pcdn_solve_batch(pcdn_job* jobs, int32_t count);

/* ---- solve server: continuous batching of independent requests ---------- */

/* A request: a problem as host CSC arrays (the layout and checks of
 * pcdn_load_csc; the arrays, and opts->w0 if set, must stay valid and
 * unchanged until the request has finished) and the arguments of pcdn_solve
 * (P = 0: about 5% of the features, the paper's starting point). */
typedef struct {
  int64_t n, p, nnz;
  const int64_t* col_ptr;
  const int32_t* row_idx;
  const float* val;
  const int8_t* y;
  double C;
  int64_t P;
  double eps;
  int32_t loss;
  int32_t reserved;       /* must be 0                                         */
  const pcdn_opts* opts;  /* nullable; copied at submission                    */
} pcdn_request;

typedef struct pcdn_server pcdn_server;

/* A server on HIP device `device` that keeps at most hbm_budget_bytes of
 * problem state (data, w, retained quantities, work arrays) resident. */
int pcdn_server_create(pcdn_server** out, int device, int64_t hbm_budget_bytes);

/* Queue a request (first in, first out); *id identifies it.  Cheap argument
 * checks only (the CSC is checked at admission).  PCDN_E_OOM if its state
 * could never fit the budget.  Does not touch the GPU. */
int pcdn_server_submit(pcdn_server* s, const pcdn_request* r, int64_t* id);

/* One scheduling step: admit queued requests in order while their state fits
 * the budget (the data is uploaded and the solve set up on the device), run
 * one outer iteration of every admitted solve (the rounds of
 * pcdn_solve_batch), and finish the solves that stopped, releasing their
 * device memory.  *finished (nullable) receives how many requests finished
 * in this step (a request whose data fails the checks finishes with that
 * error).  Each solve follows the trajectory pcdn_solve would take for it. */
int pcdn_server_step(pcdn_server* s, int32_t* finished);

/* Queue length, admitted solves and the device bytes they hold. */
int pcdn_server_status(const pcdn_server* s, int32_t* waiting, int32_t* running,
                       int64_t* bytes_in_use);

/* Result of a finished request (then forgotten): w_out (nullable, p
 * doubles), info (nullable), *status (what pcdn_solve would have returned,
 * or the admission error).  PCDN_E_STATE if the request has not finished,
 * PCDN_E_ARG for an unknown id. */
int pcdn_server_take(pcdn_server* s, int64_t id, double* w_out, pcdn_info* info,
                     int32_t* status);

const char* pcdn_server_last_error(const pcdn_server* s);

/* Release the server, its queue and every admitted solve.  NULL is accepted. */
int pcdn_server_destroy(pcdn_server* s);

/* Continue the current states of several contexts on one device together:
 * for each context j, what pcdn_iterate(ctxs[j], P[j], k_first, iters, opts,
 * &subgrads[j]) does (outer iterations k_first .. k_first+iters-1 of
 * Algorithm 3 from the state left by pcdn_reset, pcdn_solve or earlier
 * iterations, no stopping test), advanced in the rounds of pcdn_solve_batch.
 * iters >= 1; subgrads (nullable, count entries) receives each context's
 * ||grad^S F(w)||_1 after its last iteration. */
int pcdn_iterate_batch(pcdn_ctx* const* ctxs, const int64_t* P, int32_t count, int64_t k_first,
                       int64_t iters, const pcdn_opts* opts, double* subgrads);

/* Regularisation path: pcdn_solve for C = Cs[0], Cs[1], ... in order, each
 * warm-started from the previous solution (the first from opts->w0, or 0),
 * with the reference norm of the stopping rule at w = 0 for every C.  W_out
 * (nullable, host, count x p doubles, row k = the solution for Cs[k]) and
 * infos (nullable, count entries) receive the results.  Returns PCDN_OK if
 * every solve converged, PCDN_NOT_CONVERGED if one stopped at max_outer, or
 * the first error. */
int pcdn_solve_path(pcdn_ctx* ctx, const double* Cs, int32_t count, int64_t P, double eps,
                    int loss, const pcdn_opts* opts, double* W_out, pcdn_info* infos);

/* The regularisation path over `lanes` contexts that hold the same X and y
 * (same n, p, nnz and contents; else PCDN_E_ARG): Cs is cut into
 * min(lanes, count) contiguous runs of equal length (+-1), run i =
 * Cs[floor(i count / L)] .. Cs[floor((i + 1) count / L) - 1] is solved on
 * ctxs[i] as pcdn_solve_path solves it (the first C from opts->w0 or 0, each
 * next one warm-started from the previous solution), and the runs advance
 * together, one outer iteration of every unfinished run per round of the
 * batch engine (as pcdn_solve_batch).  Each solve meets the same stopping
 * rule as in pcdn_solve_path, and a run's solves are those pcdn_solve_path
 * gives for that run alone; only the first C of each run starts cold.  The
 * contexts' states are overwritten; ctxs[i] is left with the last solution
 * of run i.  W_out (nullable, host, count x p) and infos (nullable, count)
 * are indexed like Cs.  Returns as pcdn_solve_path. */
int pcdn_solve_path_lanes(pcdn_ctx* const* ctxs, int32_t lanes, const double* Cs, int32_t count,
                          int64_t P, double eps, int loss, const pcdn_opts* opts, double* W_out,
                          pcdn_info* infos);

/* Bundle-size autotuning (pcdn_autotune). */
typedef struct {
  int64_t P;                /* candidate bundle size                             */
  int32_t schedule;         /* pcdn_opts.schedule it ran with                    */
  int32_t outer;            /* pilot outer iterations run                        */
  double sec_per_outer;     /* measured seconds per outer iteration              */
  double rate;              /* measured decay of log ||grad^S F||_1 per iteration */
  double predicted_seconds; /* predicted time to reach eps (INFINITY: no progress) */
  int32_t chunk;            /* pcdn_opts.chunk it ran with (resolved)            */
  int32_t narrow;           /* 1 if it ran on the single-workgroup schedule      */
} pcdn_tune_point;

typedef struct {
  int64_t P;                /* chosen bundle size                                */
  int32_t schedule;         /* chosen pcdn_opts.schedule                         */
  int32_t n_tried;          /* entries of tried[]                                */
  double predicted_seconds; /* prediction for the chosen P                       */
  int32_t chunk;            /* chosen pcdn_opts.chunk                            */
  int32_t pad;
  pcdn_tune_point tried[12];
} pcdn_tune;

/* Choose the bundle size P, the schedule and the sweep's range width for
 * solving the loaded problem with (loss, C, eps), by the pilot procedure of
 * Sec. 5.1 ("Bundle Size Choice"): the paper starts at about 5% of the
 * features, P0 = 0.05 p, and adjusts P by measured runtime.
 *  1. P: candidates P0 * 4^k for k = 0, -1, 1, -2, 2, -3 (clipped to [1, p])
 *     in that order, with opts->schedule and opts->chunk;
 *  2. schedule (only if opts->schedule is PCDN_SCHED_AUTO): at the best P,
 *     the schedule the automatic choice did not take (WIDE after a
 *     single-workgroup run; NARROW after a WIDE run when P <= 1024);
 *  3. the bundle sweep's range width (only if opts->chunk is 0, and the
 *     best pilot so far ran WIDE bundles): 64, 128 and 512 nonzeros per
 *     wavefront (256 ran in steps 1 and 2).
 * Each pilot is the solve itself through the batch engine (the path
 * pcdn_solve_batch takes), from the start pcdn_solve would use, to the
 * target eps (graphs and task lists built before the clock starts), abandoned as soon as
 * it has run longer than the fastest finished one.  The fastest finished
 * pilot wins (if none finishes within max_outer, the one with the largest
 * decrease of the stopping norm per second); P, schedule and chunk are the
 * values to pass to pcdn_solve (pcdn_solve_batch applies them to a job
 * with P = 0).  tried[] reports every pilot (predicted_seconds: its measured
 * time, INFINITY if it did not finish).  The context's device state
 * afterwards is the last pilot's.  Returns PCDN_OK or an error. */
int pcdn_autotune(pcdn_ctx* ctx, int loss, double C, double eps, const pcdn_opts* opts,
                  pcdn_tune* out);

/* Set the device state to (loss, C, w): w (host, p doubles) or zeros if NULL;
 * the retained e^{w^T x_i} (logistic) or b_i = 1 - y_i w^T x_i (SVM) are
 * recomputed from w in FP64 (Sec. 3.1).  PCDN_E_NUMERIC if a retained
 * quantity falls outside its range (see PCDN_E_NUMERIC); pcdn_step and the
 * solves report a step that takes one there the same way. */
int pcdn_reset(pcdn_ctx* ctx, int loss, double C, const double* w);

/* One inner iteration of Algorithm 3 on an explicit bundle (host array of P
 * distinct feature indices in [0, p)), from the current device state; updates
 * w and the retained quantities.  opts supplies sigma, beta, gamma, nu and
 * max_ls (NULL: defaults).  Optional host outputs (NULL to skip): g, h, d
 * (P doubles each, bundle order): gradient, Hessian diagonal (eq. (11); SVM:
 * generalised Hessian) and the direction (eq. (5)); dtx (n doubles): d^T x_i
 * before any backtracking scaling. */
int pcdn_step(pcdn_ctx* ctx, const int32_t* bundle, int64_t P, const pcdn_opts* opts,
              pcdn_step_info* out, double* g, double* h, double* d, double* dtx);

/* Run `count` outer iterations of Algorithm 3, iterations k_first ..
 * k_first+count-1 of the partition sequence of opts->seed, from the current
 * device state (left by pcdn_reset, pcdn_solve or an earlier call) with that
 * state's loss and C.  Each outer iteration draws its partition, runs every
 * bundle, then the full-gradient stopping sweep.  subgrad (nullable)
 * receives ||grad^S F(w)||_1 after the last iteration.  1 <= P <= p,
 * k_first >= 0, count >= 0. */
int pcdn_iterate(pcdn_ctx* ctx, int64_t P, int64_t k_first, int64_t count,
                 const pcdn_opts* opts, double* subgrad);

/* The feature permutation of outer iteration k for `seed` (host, p int32):
 * features sorted by the upper 32 bits of output j of the SplitMix64 stream
 * whose seed is output k of the SplitMix64 stream seeded with `seed`, ties by
 * index.  Bundle t of that iteration is perm[tP, min((t+1)P, p)). */
int pcdn_permutation(pcdn_ctx* ctx, uint64_t seed, int64_t k, int32_t* perm_out);

/* Copy the current w (host, p doubles). */
int pcdn_get_w(pcdn_ctx* ctx, double* w_out);

/* Copy the retained per-sample quantities (host, n doubles). */
int pcdn_get_cache(pcdn_ctx* ctx, double* cache_out);

/* F(w) (eq. (1)) and ||grad^S F(w)||_1 at the current state (either pointer
 * may be NULL), with the regulariser of the last pcdn_solve, pcdn_iterate,
 * pcdn_step or batched call that advanced this state (eq. (1)'s after
 * pcdn_reset). */
int pcdn_evaluate(pcdn_ctx* ctx, double* objective, double* subgrad);

/* Kernel timing.  Kernel classes: 0 bundle sweep (g, h and, for the slots
 * inside one range, d), 1 its finish (the slots across ranges, the empty
 * ones), 2 d^T x with the first line-search candidates, 3 Armijo decision
 * and apply, 4 stopping sweep, 5 single-workgroup kernel (every step of
 * every bundle of an outer iteration, PCDN_SCHED_NARROW).
 * pcdn_profile(ctx, mask) brackets every launch of each class whose bit
 * (1 << class) is set in mask with HIP events on the context's stream (mask
 * 0: off) and restarts the accumulators;
 * pcdn_profile_read() returns for class `which` the summed event time in ms
 * and the launch count since then (bracketed classes only), and the
 * algorithmic bytes all launches of that class moved since then. */
int pcdn_profile(pcdn_ctx* ctx, int mask);
int pcdn_profile_read(pcdn_ctx* ctx, int which, double* ms, int64_t* launches,
                      double* alg_bytes);

/* Description of the last error on ctx (or, when ctx is NULL, of this
 * thread's last failed pcdn_create or pcdn_solve_static); valid until the
 * next call on ctx (or on this thread). */
const char* pcdn_last_error(const pcdn_ctx* ctx);

/* pcdn_solve without any device allocation, for callers that cannot
 * allocate: code that runs while a HIP graph is captured around it, tight
 * serving loops, harnesses that forbid hipMalloc.  One call loads and solves
 * one problem as pcdn_load_csc then pcdn_solve would (the same partitions,
 * kernels and arithmetic; the automatic schedule keeps bundles of many
 * nonzeros in the single workgroup instead of moving them to the
 * multi-kernel path, and no launch is captured as a graph), with no context.
 *  device, hip_stream: the GPU and the stream to run on (NULL: the null
 *    stream); the call returns when its work on the stream is done.
 *  n, p, nnz, col_ptr (int64, p + 1), row_idx (int32, nnz), val (fp32, nnz),
 *    y (int8, n): X in CSC and the labels, in DEVICE memory, read only,
 *    checked on the device as pcdn_load_csc checks them (PCDN_E_CSC).
 *  C, P, eps, loss, opts, info: as pcdn_solve (opts->w0, if given, is host
 *    memory).
 *  w_out: DEVICE, p doubles, written with the solution; it also holds w
 *    while the solve runs.
 * Every other buffer lives in a workspace of 64 MiB per device compiled into
 * the library (each device the library runs on holds it until the process
 * ends); a problem whose buffers do not fit (roughly 70 bytes per nonzero,
 * 110 per feature and 50 per sample) is rejected with PCDN_E_ARG before any
 * work.  Every call on one device shares that workspace: calls that overlap
 * on one device (two host threads, or two streams) race and must not be
 * made.  Errors are described by pcdn_last_error(NULL). */
int pcdn_solve_static(int device, void* hip_stream, int64_t n, int64_t p, int64_t nnz,
                      const int64_t* col_ptr, const int32_t* row_idx, const float* val,
                      const int8_t* y, double C, int64_t P, double eps, int loss,
                      const pcdn_opts* opts, double* w_out, pcdn_info* info);

/* Release the context and its device memory.  NULL is accepted. */
int pcdn_destroy(pcdn_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* PCDN_H */
