/*
 * libsccs -- cyclic coordinate descent (CCD) for the MAP fit of the Bayesian
 * self-controlled case series (BSCCS) model on one AMD Instinct MI355X
 * (gfx950), after Suchard, Simpson, Zorych, Ryan and Madigan, "Massive
 * parallelization of serial inference algorithms for a complex generalized
 * linear model".
 *
 * Model (Section 2.1).  Patient i = 0..N-1 has eras k (rows of X, grouped by
 * patient) with length l_k >= 0 days, event count y_k >= 0 and a binary
 * exposure row x_k over J drugs.  With n_i = sum_k y_ik the conditional
 * log-likelihood is Eq. 2,
 *     L(beta) = sum_i omega_i [ sum_k y_ik x_ik'beta - n_i log sum_k l_ik exp(x_ik'beta) ],
 * where omega_i >= 0 is an optional integer patient weight (1 by default;
 * cross-validation folds use 0/1, the bootstrap uses resample counts).
 * The prior (Eq. 3) is Normal(0, var) or Laplace(0, var) on every beta_j,
 * var being the variance (Laplace rate lambda = sqrt(2/var)).  The library
 * maximises P(beta) = L(beta) + log p(beta) by Algorithm 1: coordinates
 * j = 0..J-1 are visited in order each sweep; each visit computes the
 * one-dimensional gradient and Hessian g_j, h_j (Eqs. 7-9), takes one
 * prior-regularised Newton step (Eq. 4) bounded by an adaptable trust region
 * (after Genkin et al. 2007: step clipped to +-trust_j, then
 * trust_j <- max(2|step|, trust_j/2), trust_j = 1 at the start of a fit), and
 * if the step is nonzero updates exp(X beta) on the column's rows and the
 * per-patient sums M[L x exp(X beta)] (Section 2.4, Steps 1-4).
 *
 * Laplace step rules at a kink (the paper leaves them open): beta_j > 0 uses
 * the branch with -lambda and stops at zero if the step would cross it;
 * beta_j < 0 symmetrically; beta_j = 0 moves only if |g_j| > lambda
 * (strict).  Without curvature (h_j = 0) no step is taken.
 *
 * Conventions.
 *  - Status: 0 = SCCS_OK; positive = informational; negative = error.  No
 *    C++ exception crosses this interface.  On error, sccs_last_error()
 *    describes it.  Validation finishes before any state changes.
 *  - Host pointers unless stated.  Input arrays are borrowed for the duration
 *    of the call only; the library copies what it needs.
 *  - A handle is not thread-safe; separate handles are independent.  All
 *    device work of a handle is ordered on its stream (options.stream, a
 *    hipStream_t; NULL = the null stream).  Calls that return host data
 *    synchronise that stream.
 *  - Device memory comes from a caller-owned workspace (sccs_query_workspace
 *    gives its size; the caller allocates it, for example as a torch uint8
 *    tensor, and keeps it alive until sccs_destroy) or, if the workspace
 *    pointer is NULL, from hipMalloc inside sccs_create (freed by
 *    sccs_destroy).
 */
#ifndef SCCS_H
#define SCCS_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sccs_status;
#define SCCS_OK 0
#define SCCS_NOT_CONVERGED 1       /* sccs_fit stopped at max_sweeps */
#define SCCS_ERR_INVALID_ARG (-1)  /* bad argument or malformed problem */
#define SCCS_ERR_WORKSPACE (-2)    /* workspace too small or misaligned */
#define SCCS_ERR_HIP (-3)          /* a HIP runtime call failed */
#define SCCS_ERR_STATE (-4)        /* call not valid in the current state */
#define SCCS_ERR_NUMERIC (-5)      /* non-finite g, h or beta; last finite beta kept */
#define SCCS_ERR_SYNC (-6)         /* the device-wide reduction did not complete */

enum { SCCS_PRIOR_NONE = 0, SCCS_PRIOR_NORMAL = 1, SCCS_PRIOR_LAPLACE = 2, SCCS_PRIOR_GROUPED = 3 };
enum { SCCS_PREC_FP64 = 0, SCCS_PREC_MIXED = 1 };
enum { SCCS_CRIT_FIXED = 0, SCCS_CRIT_REL_LOGPOST = 1, SCCS_CRIT_ABS_DXBETA = 2 };
enum { SCCS_ORDER_GIVEN = 0, SCCS_ORDER_INDEPENDENT = 1 };

typedef struct sccs_handle sccs_handle;

/*
 * One SCCS problem in the matrix form of Section 2.3 (Eq. 5-6), host memory.
 *   patient_ptr [N+1] int64: rows of patient i are [ptr[i], ptr[i+1]);
 *                 ptr[0] = 0, non-decreasing, ptr[N] = n_rows.
 *   offset      [K] int32: era length l_k >= 0.
 *   count       [K] int32: events y_k >= 0; y_k > 0 requires l_k > 0.
 *   col_ptr     [J+1] int64: X in compressed column storage.
 *   row_idx     [nnz] int32: rows of each column, strictly increasing.
 *   patient_weight [N] int32 >= 0, or NULL for all ones.
 *   value       [nnz] double, finite: covariate values x_kj in the order of
 *                 row_idx, or NULL for binary exposures (all stored entries
 *                 1, the paper's drug eras).  Non-binary and dense covariates
 *                 (Section 4: baseline measurements, doses) take the general
 *                 form of Eqs. 7-9: g_j = sum omega y x - sum omega n A_i and
 *                 h_j = -sum omega n (B_i - A_i^2), with A_i = M[w x X_j]_i/den_i
 *                 and B_i = M[w x X_j^2]_i/den_i, and a step multiplies
 *                 exp(X beta) by exp(delta x_kj) entry by entry.  A dense
 *                 column is a column that stores every row.  The batched form
 *                 takes binary problems only.
 * Limits: N, K, J >= 1; N < 2^28; K < 2^31; nnz < 2^31.  Patients without events
 * (n_i = 0) are accepted and carry no information (cases-only design).
 */
typedef struct sccs_problem {
  int32_t n_patients;
  int64_t n_rows;
  int32_t n_cols;
  int64_t nnz;
  const int64_t* patient_ptr;
  const int32_t* offset;
  const int32_t* count;
  const int64_t* col_ptr;
  const int32_t* row_idx;
  const int32_t* patient_weight;
  const double* value;
} sccs_problem;

typedef struct sccs_options {
  int32_t precision;       /* SCCS_PREC_FP64 or SCCS_PREC_MIXED (FP32 exp(X beta) and row products) */
  int32_t n_workgroups;    /* persistent workgroups; 0 = one per compute unit */
  int32_t refresh_period;  /* sweeps between exact recomputation of w and den from beta;
                              0 = never, -1 = default (0 for FP64, 1 for mixed) */
  int32_t tile_nnz;        /* nonzeros per tile (one wavefront each): 0 = 64, else 8..64;
                              a patient with more nonzeros in a column gets a tile of its own */
  int32_t max_group;       /* single fit: consecutive columns that share no patient have
                              independent Newton steps and are visited with one device-wide
                              reduction, up to max_group columns at a time (results equal
                              those of visiting them one by one, up to summation order);
                              0 = 4, else 1..4 (1 = one column per reduction).  The lockstep
                              batched engine groups columns only when all its fits share one
                              problem, with at most 64 / n_fits columns per group. */
  int32_t merge_passes;    /* single fit: 1 = let up to 3 consecutive column groups (5 columns
                              at most) share one reduction when every earlier column of the
                              pass that shares a patient with a later group took a zero step
                              in its previous visit; the prediction is checked after the step
                              and, where it fails, the first group it fails for and the groups
                              after it are visited again, so g_j, h_j and beta are those of
                              the plain cyclic order (bit for bit); used for launches that
                              follow one where most steps were zero (see sccs_pass_stats);
                              0 = off.  Default 1. */
  void* stream;            /* hipStream_t */
  int32_t batch_engine;    /* batched form: 0 = partitioned (default): each fit runs the single-fit
                              sweep (with column groups up to max_group) on its own range of the
                              launch's workgroups; up to 32 fits per launch, taken in decreasing
                              order of nonzeros, the workgroups shared out in multiples of 8 in
                              proportion to nonzeros; one launch per prior link and per 32 fits.
                              1 = lockstep: all fits on all workgroups in one launch, one
                              device-wide reduction per coordinate (or column group) for all */
  int32_t column_order;    /* order in which a sweep visits the coordinates (Algorithm 1 cycles
                              over the drugs in a fixed order; how the drugs are numbered is
                              free).  SCCS_ORDER_GIVEN (default): the problem's column order.
                              SCCS_ORDER_INDEPENDENT: the order of sccs_column_order with width
                              max_group, under which consecutive columns share no patient far
                              more often, so that more of them share a device-wide reduction.
                              Betas, trust bounds, class_of and grad_hess's j stay in the
                              problem's numbering at the ABI.  The lockstep batched engine
                              takes SCCS_ORDER_GIVEN only. */
} sccs_options;

typedef struct sccs_fit_opts {
  int32_t criterion;   /* SCCS_CRIT_* */
  int32_t max_sweeps;  /* >= 1 */
  double tol;          /* REL_LOGPOST: |P_t - P_{t-1}| < tol |P_t|;
                          ABS_DXBETA: sum_k |eta_k^t - eta_k^{t-1}| < tol (Section 2.2 uses 5e-4) */
} sccs_fit_opts;

typedef struct sccs_fit_result {
  int32_t sweeps;      /* sweeps run by this call */
  int32_t converged;   /* 1 if the criterion was met */
  double loglik;       /* L(beta) at exit (Eq. 2, from the maintained state) */
  double logpost;      /* L + log p(beta), constants dropped */
} sccs_fit_result;

/* Options with defaults: FP64, one workgroup per CU, default refresh, 64-nonzero tiles,
 * groups of up to 4 columns, merged passes on, NULL stream. */
void sccs_default_options(sccs_options* opts);

/* Device bytes sccs_create needs for this problem and these options.
 * Validates the problem (same checks as sccs_create). */
sccs_status sccs_query_workspace(const sccs_problem* prob, const sccs_options* opts, size_t* bytes);

/* Validate and repack the problem into device memory and set beta = 0,
 * trust = 1, no prior.  workspace: device pointer of >= the queried bytes,
 * 256-byte aligned, owned by the caller; NULL makes the library allocate.
 * Setup (Algorithm 1, initialisation): n_i, Y'X_j and the initial
 * w = L, den = M L are computed on the device. */
sccs_status sccs_create(const sccs_problem* prob, const sccs_options* opts, void* workspace,
                        size_t workspace_bytes, sccs_handle** out);

/* Release host-side memory (and the workspace if the library allocated it).
 * NULL-safe.  Synchronises the stream first. */
sccs_status sccs_destroy(sccs_handle* h);

/* Prior of Eq. 3: kind SCCS_PRIOR_NONE / _NORMAL / _LAPLACE; variance > 0
 * (ignored for NONE).  Changes nothing else (beta and trust are kept).
 * (SCCS_PRIOR_GROUPED is set by sccs_set_prior_grouped.) */
sccs_status sccs_set_prior(sccs_handle* h, int32_t kind, double variance);

/* Grouped Normal prior, a hierarchical prior of the kind Section 4 proposes
 * (drugs grouped a priori into classes borrow strength from each other):
 * drug j of class c = class_of[j] has beta_j = mu_c + b_j with
 * b_j ~ N(0, variance) and the class mean mu_c ~ N(0, class_variance).
 * Integrating mu_c out, a class of m drugs has covariance
 * variance I + class_variance 1 1', so Eq. 4 takes
 *   d log p / d beta_j = -(beta_j - kappa_c S_c) / variance,
 *   d2 log p / d beta_j^2 = -(1 - kappa_c) / variance,
 * with kappa_c = class_variance / (variance + m class_variance) and S_c the
 * sum of the class's coefficients (kept on the device as steps are taken;
 * columns of one class are stepped in column order, also inside a column
 * group).  class_variance = 0 is the Normal prior; a class of one drug is
 * a Normal prior of variance variance + class_variance.  class_of: [J] host
 * int32 in [0, n_classes), 1 <= n_classes <= J; variance > 0;
 * class_variance >= 0.  Single fits only; the merged-pass form is not used
 * under this prior.  Changes nothing else (beta and trust are kept). */
sccs_status sccs_set_prior_grouped(sccs_handle* h, double variance, double class_variance, int32_t n_classes,
                                   const int32_t* class_of);

/* Warm start: copy beta [J] (host) and trust [J] (host, or NULL for all
 * ones), then recompute w = L x exp(X beta) and den = M w exactly. */
sccs_status sccs_set_beta(sccs_handle* h, const double* beta, const double* trust);

/* Copy the current beta [J] and, if trust is not NULL, the trust bounds [J]
 * to host memory.  Synchronises. */
sccs_status sccs_get_beta(sccs_handle* h, double* beta, double* trust);

/* Run exactly n_sweeps cycles over j = 0..J-1 (Algorithm 1 without the stop
 * test) in one device launch.  If logpost is not NULL, the log posterior
 * after the last sweep is written there (synchronises).  Needs a prior. */
sccs_status sccs_sweep(sccs_handle* h, int32_t n_sweeps, double* logpost);

/* Allocation-free variant of sccs_sweep, for callers that cannot allocate
 * device memory or call allocating routines (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  It runs the same
 * sweeps with the same kernels and results, but the device-wide reduction
 * slots and the control block of the launch live in a static device array
 * inside the library (480 KiB per device, slots for up to 256 workgroups,
 * held until the process ends) instead of the handle's workspace; the
 * handle's state (beta, trust, exp(X beta), den) is in its workspace as
 * always.  Needs n_sweeps >= 1 and the handle's device current
 * (SCCS_ERR_STATE otherwise); a handle with more workgroups than the array
 * holds gets SCCS_ERR_INVALID_ARG.  All handles on one device share the
 * array and each call re-initialises it: calls that overlap on one device
 * (other streams, other threads) race and must be serialised by the
 * caller.  Synchronises the stream; sccs_pass_stats and
 * sccs_last_kernel_ms report on it as on sccs_sweep. */
sccs_status sccs_sweep_static(sccs_handle* h, int32_t n_sweeps, double* logpost);

/* Run cycles until the criterion holds or max_sweeps cycles ran, in one
 * device launch; the stop test is evaluated on the device after every
 * sweep.  Returns SCCS_OK if converged, SCCS_NOT_CONVERGED otherwise (or an
 * error).  Synchronises. */
sccs_status sccs_fit(sccs_handle* h, const sccs_fit_opts* fo, sccs_fit_result* res);

/* Likelihood-only g_j and h_j (Eqs. 7-9) at the current beta, from the
 * maintained state (diagnostic; no step is taken).  Synchronises. */
sccs_status sccs_grad_hess(sccs_handle* h, int32_t j, double* g, double* hess);

/* L(beta) and L + log p(beta) at the current beta from the maintained
 * state.  Synchronises. */
sccs_status sccs_objective(sccs_handle* h, double* loglik, double* logpost);

/* Device-side timing of the most recent sccs_sweep / sccs_fit launch in
 * milliseconds (HIP events on the handle's stream around the persistent
 * kernel alone).  Synchronises. */
sccs_status sccs_last_kernel_ms(sccs_handle* h, double* ms);

/* Schedule statistics of the most recent sccs_sweep / sccs_fit launch:
 * passes = device-wide coordinate reductions run (one per column group, or
 * per run of groups merged as options.merge_passes describes), rejects =
 * merged passes whose later groups had to be visited again, zero_steps =
 * coordinate visits whose step was exactly zero.  Merged passes are used
 * for a launch when at least half of the previous launch's visits took
 * zero steps (until that share falls below 35 %).  ERR_STATE before any
 * sweep. */
sccs_status sccs_pass_stats(sccs_handle* h, int32_t* passes, int32_t* rejects, int32_t* zero_steps);

/* Per-coordinate timing on or off (on = 1, off = 0; off when a handle is
 * created) for the handle's later sccs_sweep / sccs_fit launches: with it
 * on, workgroup 0 stores the device wall clock once per column group, a
 * store its next barrier waits for, so the sweep runs slightly slower.
 * SCCS_ERR_INVALID_ARG for another value. */
sccs_status sccs_group_timing(sccs_handle* h, int32_t on);

/* Per-coordinate timing (for achieved bandwidth against column size): after
 * an sccs_sweep / sccs_fit launch in the one-pass-per-group form (a launch
 * that did not use merged passes; binary covariates) made with
 * sccs_group_timing on, t_us[g] is the time
 * from the start of that launch's last sweep to the moment column group g's
 * steps were taken, in microseconds of the device wall clock, for the
 * n_groups groups; group g holds the columns visited at positions
 * [first_col[g], first_col[g+1]) of the sweep (sccs_get_column_order maps
 * positions to columns).
 * t_us: [max_groups]; first_col: [max_groups + 1].  SCCS_ERR_STATE if no
 * such launch preceded; SCCS_ERR_INVALID_ARG if max_groups < n_groups
 * (n_groups is still written).  Synchronises. */
sccs_status sccs_group_times(sccs_handle* h, int32_t max_groups, double* t_us, int32_t* first_col, int32_t* n_groups);

/* Autotuner: times candidate schedules -- workgroup counts (all compute
 * units, 3/4, 1/2, 1/4 of them) x tile sizes (16, 32, 64 nonzeros) -- on
 * this problem with this prior, each for n_sweeps sweeps after one warm-up
 * sweep from beta = 0, on temporary library-allocated handles; returns the
 * fastest as options (opts with n_workgroups and tile_nnz filled in) and the
 * per-candidate timings.  Synchronises; allocates and frees device memory. */
#define SCCS_TUNE_MAX 16
typedef struct sccs_tune_result {
  int32_t n_candidates;
  int32_t best;                               /* index of the fastest */
  int32_t n_workgroups[SCCS_TUNE_MAX];
  int32_t tile_nnz[SCCS_TUNE_MAX];
  double ms_per_sweep[SCCS_TUNE_MAX];
} sccs_tune_result;

sccs_status sccs_tune(const sccs_problem* prob, const sccs_options* base, int32_t prior_kind, double variance,
                      int32_t n_sweeps, sccs_options* best, sccs_tune_result* result);

/* The independence relabelling of a problem's columns (host only, no GPU
 * needed): columns are visited in decreasing order of nonzeros (ties:
 * smaller index first); each joins the first group, in creation order, that
 * has fewer than width columns (1..4) and shares no patient with it, or opens
 * a new group at the end.  order[k] ([n_cols], caller-owned) is the column
 * visited k-th: the groups in creation order, each group's columns in the
 * order they joined.  SCCS_ERR_INVALID_ARG for a malformed problem or
 * width outside [1, 4]; sccs_last_error(NULL) describes it. */
sccs_status sccs_column_order(const sccs_problem* prob, int32_t width, int32_t* order);

/* The order in which h's sweeps visit the columns (order[k], k < n_cols):
 * the identity under SCCS_ORDER_GIVEN. */
sccs_status sccs_get_column_order(sccs_handle* h, int32_t* order);

/* Human-readable description of the last error on this handle (or of the
 * last failed create when h is NULL).  Never NULL. */
const char* sccs_last_error(const sccs_handle* h);

/* ------------------------------------------------------------ batched form
 *
 * F <= 64 independent fits on one device (Section 2.5: cross-validation
 * over a prior grid and bootstrap replicates need many fits; different
 * outcomes over one drug vocabulary likewise).  All problems of a batch
 * share n_cols.  Two engines (sccs_options.batch_engine): partitioned, where
 * each fit runs the single-fit sweep on its own range of workgroups and
 * stops on its own, one launch per prior link; or lockstep, where one
 * persistent launch runs every chain and, per coordinate, one device-wide
 * reduction carries the partial sums of all fits.  Each fit walks a chain
 * of priors in order: link l starts from the beta where link l-1 ended
 * (warm start, Section 2.5), with every trust bound reset to 1, and ends
 * when the stopping rule holds or after max_sweeps sweeps; its beta and
 * result are recorded.  Per fit, patient weights (for example the training
 * indicator of a cross-validation fold) override the problem's own.
 */
typedef struct sccs_batch sccs_batch;

typedef struct sccs_fit_spec {
  int32_t problem;               /* index into the problem array */
  int32_t n_links;               /* >= 1 priors visited in order */
  const int32_t* prior_kind;     /* [n_links] SCCS_PRIOR_* */
  const double* variance;        /* [n_links] > 0 (ignored for NONE) */
  const int32_t* patient_weight; /* [N of its problem] >= 0, or NULL */
} sccs_fit_spec;

/* Device bytes for sccs_batch_create (validates as sccs_batch_create). */
sccs_status sccs_batch_query_workspace(const sccs_problem* probs, int32_t n_probs, const sccs_fit_spec* fits,
                                       int32_t n_fits, const sccs_options* opts, size_t* bytes);

/* Validate, repack every problem once (fits of one problem share its index
 * data), set up every fit at beta = 0.  workspace as for sccs_create.
 * Errors as for sccs_create; n_fits in [1, 64]. */
sccs_status sccs_batch_create(const sccs_problem* probs, int32_t n_probs, const sccs_fit_spec* fits,
                              int32_t n_fits, const sccs_options* opts, void* workspace, size_t workspace_bytes,
                              sccs_batch** out);

/* Run every fit's chain to its end in one launch.  fo->criterion is
 * SCCS_CRIT_FIXED (each link runs exactly max_sweeps sweeps) or
 * SCCS_CRIT_REL_LOGPOST (per link, until |P_t - P_{t-1}| < tol |P_t| or
 * max_sweeps).  Synchronises. */
sccs_status sccs_batch_run(sccs_batch* b, const sccs_fit_opts* fo);

/* beta [J] (host, nullable) and the result of link `link` of fit `fit`. */
sccs_status sccs_batch_get(sccs_batch* b, int32_t fit, int32_t link, double* beta, sccs_fit_result* res);

/* Held-out log-likelihood of link `link` of fit `fit`: Eq. 2 at the link's
 * beta, summed over the patients whose weight in this fit is 0 (for a
 * cross-validation fold, the patients left out of training; Section 2.5).
 * Evaluated on the device when the link ends, from the maintained den_i.
 * SCCS_ERR_STATE if the fit has no patient weights or the link has not run. */
sccs_status sccs_batch_heldout(sccs_batch* b, int32_t fit, int32_t link, double* loglik);

/* Device time of the last sccs_batch_run (ms): its launch (lockstep), or
 * the sum of its sweep launches (partitioned). */
sccs_status sccs_batch_last_kernel_ms(sccs_batch* b, double* ms);

/* NULL-safe. */
sccs_status sccs_batch_destroy(sccs_batch* b);

/* Description of the last error on b, or of the last failed create. */
const char* sccs_batch_last_error(const sccs_batch* b);

/* Autotuner of the batched form: times the same candidate launch shapes as
 * sccs_tune -- workgroup counts (all compute units, 3/4, 1/2, 1/4) x tile
 * sizes (16, 32, 64 nonzeros) -- on this batch of problems and fits, each
 * for n_sweeps sweeps (every fit's first link, FIXED) after one warm-up
 * sweep, on temporary library-allocated batches of base's engine; returns
 * the fastest as options and the per-candidate timings (ms per sweep of the
 * whole batch).
 * Synchronises; allocates and frees device memory. */
sccs_status sccs_batch_tune(const sccs_problem* probs, int32_t n_probs, const sccs_fit_spec* fits, int32_t n_fits,
                            const sccs_options* base, int32_t n_sweeps, sccs_options* best, sccs_tune_result* result);

/* ------------------------------------------------------------ bootstrap
 *
 * Non-parametric bootstrap over patients (Section 2.5): each replicate r
 * refits the MAP beta with patient weights omega_i = replicate_weight[r][i]
 * (the number of times patient i was drawn when N patients are resampled
 * with replacement; the caller draws them, so results are reproducible from
 * the caller's generator).  The replicates run as batched fits, up to 64 per
 * launch, one launch after another in the same workspace, each from
 * beta = 0 with trust 1 under one prior.  Per coefficient the result is the
 * percentile interval -- the (1 - level)/2 and (1 + level)/2 quantiles of
 * the R estimates, by linear interpolation between order statistics
 * (position (R - 1) q) -- and p_nonzero, the share of replicates whose MAP
 * estimate is not exactly 0 (under the Laplace prior, the paper's estimate
 * of the probability that beta_j != 0).  The paper reports level 0.95 over
 * 200 replicates. */
typedef struct sccs_bootstrap_out {
  double* beta;        /* [R][J] each replicate's beta, or NULL */
  double* ci_lo;       /* [J] lower percentile bound */
  double* ci_hi;       /* [J] upper percentile bound */
  double* p_nonzero;   /* [J] share of replicates with beta_j != 0 */
  int32_t* sweeps;     /* [R] sweeps run per replicate, or NULL */
  int32_t* converged;  /* [R] 1 if the replicate met the criterion, or NULL */
} sccs_bootstrap_out;

/* Device bytes sccs_bootstrap needs (a batch of min(R, 64) fits). */
sccs_status sccs_bootstrap_query_workspace(const sccs_problem* prob, const sccs_options* opts, int32_t n_replicates,
                                           size_t* bytes);

/* Run R = n_replicates bootstrap fits and summarise them.  replicate_weight:
 * [R][N] host int32 >= 0.  fo: criterion FIXED or REL_LOGPOST, per
 * replicate.  level in (0, 1).  workspace as for sccs_batch_create (NULL:
 * library-allocated for the call).  Errors as for sccs_batch_create and
 * sccs_batch_run; sccs_batch_last_error(NULL) describes them.
 * Synchronises. */
sccs_status sccs_bootstrap(const sccs_problem* prob, const sccs_options* opts, void* workspace, size_t workspace_bytes,
                           int32_t prior_kind, double variance, int32_t n_replicates, const int32_t* replicate_weight,
                           const sccs_fit_opts* fo, double level, sccs_bootstrap_out* out);

/* ------------------------------------------------------------ prior-variance search
 *
 * Cross-validated choice of the prior variance (Section 2.5): the patients
 * are split into folds; for a variance, each fold is fitted on the other
 * folds' patients (one batched run, one fit per fold) and the held-out
 * Eq. 2 of its own patients is summed over folds (the predictive
 * log-likelihood).  Instead of a fixed grid, the search brackets the
 * maximum and then narrows it, the refinement the paper suggests:
 *   1. evaluate t0 = log10(var_start) and t0 + s, s = log10(bracket_step);
 *      walk on in steps of s in the rising direction until a point is
 *      lower than its predecessor (the bracket lo < t_best < hi);
 *   2. golden-section search inside the bracket (the new point in the
 *      larger part, at 0.381966 of it from the current best) until
 *      hi - lo <= log10_tol.
 * Each evaluation may start every fold from that fold's fit at the nearest
 * variance evaluated so far (warm_start), with trust bounds reset to 1.
 * The search stops early when max_evals evaluations ran (then bracketed may
 * be 0: the maximum lies beyond the walked range). */
#define SCCS_CV_MAX_EVALS 64
typedef struct sccs_cv_opts {
  int32_t prior_kind;     /* SCCS_PRIOR_NORMAL or SCCS_PRIOR_LAPLACE */
  int32_t n_folds;        /* 2..64 */
  const int32_t* fold;    /* [N] fold of each patient, in [0, n_folds) */
  double var_start;       /* > 0 */
  double bracket_step;    /* > 1, factor between bracketing evaluations */
  double log10_tol;       /* > 0, final bracket width in log10(variance) */
  int32_t max_evals;      /* 3..SCCS_CV_MAX_EVALS */
  int32_t warm_start;     /* 1 = start folds from the nearest evaluated variance */
  sccs_fit_opts fit;      /* per fold fit: FIXED or REL_LOGPOST */
} sccs_cv_opts;

typedef struct sccs_cv_result {
  int32_t n_evals;                          /* evaluations run */
  int32_t best;                             /* index of the largest predictive log-likelihood */
  int32_t bracketed;                        /* 1 if an interior maximum was bracketed */
  double variance[SCCS_CV_MAX_EVALS];       /* evaluated variances, in order */
  double pred_loglik[SCCS_CV_MAX_EVALS];    /* their predictive log-likelihoods */
} sccs_cv_result;

/* Device bytes sccs_cv_search needs (a batch of n_folds fits). */
sccs_status sccs_cv_query_workspace(const sccs_problem* prob, const sccs_options* opts, int32_t n_folds, size_t* bytes);

/* Run the search; workspace as for sccs_batch_create (NULL:
 * library-allocated for the call).  Errors as for the batched form;
 * sccs_batch_last_error(NULL) describes them.  Synchronises. */
sccs_status sccs_cv_search(const sccs_problem* prob, const sccs_options* opts, void* workspace, size_t workspace_bytes,
                           const sccs_cv_opts* co, sccs_cv_result* out);

#ifdef __cplusplus
}
#endif
#endif
