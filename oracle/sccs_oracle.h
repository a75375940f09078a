/*
 * Plain FP64 CPU oracle for cyclic coordinate descent (CCD) on the Bayesian
 * self-controlled case series (BSCCS) model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP library.
 *
 * Everything here is single-threaded double precision, written for a reader
 * to check against the paper by eye: Eq. 2 (log-likelihood), Eqs. 7-9 (one-
 * dimensional gradient and Hessian), Eq. 4 (single Newton step with the prior)
 * and Algorithm 1 (the CCD cycle).  Readings of points the paper leaves open
 * (the Laplace step rules, the trust-region update, the convergence tests) are
 * documented in oracle/sccs_oracle.c next to the code that applies them.
 */
#ifndef SCCS_ORACLE_H
#define SCCS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Raw problem, host memory, borrowed for the duration of each call. */
typedef struct ora_problem {
  int32_t n_patients;          /* N */
  int64_t n_rows;              /* K = total eras */
  int32_t n_cols;              /* J */
  const int64_t* patient_ptr;  /* [N+1] eras of patient i: [ptr[i], ptr[i+1]) */
  const int32_t* offset;       /* [K] era length l_ik (days) */
  const int32_t* count;        /* [K] event count y_ik */
  const int64_t* col_ptr;      /* [J+1] CSC column pointers */
  const int32_t* row_idx;      /* [nnz] CSC rows, ascending within a column */
  const int32_t* weight;       /* [N] patient weight (CV / bootstrap), NULL = 1 */
  const double* value;         /* [nnz] covariate values x_kj in CSC order, NULL = all 1 (binary) */
} ora_problem;

enum { ORA_PRIOR_NONE = 0, ORA_PRIOR_NORMAL = 1, ORA_PRIOR_LAPLACE = 2 };
enum { ORA_CRIT_FIXED = 0, ORA_CRIT_REL_LOGPOST = 1, ORA_CRIT_ABS_DXBETA = 2 };

typedef struct ora_result {
  int32_t sweeps;      /* sweeps performed */
  int32_t converged;   /* 1 if the criterion was met */
  double loglik;       /* L(beta) at exit, Eq. 2 */
  double logpost;      /* L(beta) + log p(beta) at exit (constants dropped) */
} ora_result;

/* Eq. 2 evaluated from its definition at beta.  Returns 0 on success. */
int ora_loglik(const ora_problem* p, const double* beta, double* loglik);

/* log p(beta) without constants: Normal -sum b^2/(2 var), Laplace
 * -sqrt(2/var) sum |b|, none 0. */
double ora_log_prior(int32_t kind, double var, int32_t J, const double* beta);

/* g_j and h_j of Eqs. 7-9 at beta (likelihood only, no prior).  With
 * covariate values the Hessian takes its general form (see the .c file). */
int ora_grad_hess(const ora_problem* p, const double* beta, int32_t j, double* g, double* h);

/* Unbounded single-coordinate step of Eq. 4 under the prior (see the .c
 * file for the Laplace rules), then the trust-region bound.  trust_io holds
 * the coordinate's current bound on entry and its updated bound on exit. */
double ora_newton_step(int32_t kind, double var, double beta_j, double g, double h);
double ora_trust_clamp(double dv, double* trust_io);

/* Grouped ("hierarchical") Normal prior, one of the richer priors Section 4
 * proposes to borrow strength across drugs of one class: drug j of class
 * c = class_of[j] has beta_j = mu_c + b_j with b_j ~ N(0, var) and the class
 * mean mu_c ~ N(0, class_var).  Integrating mu_c out, a class of m drugs
 * has covariance var I + class_var 1 1', whose inverse is
 * (I - kappa_c 1 1') / var with kappa_c = class_var / (var + m class_var). */
typedef struct ora_groups {
  int32_t n_classes;
  const int32_t* class_of;  /* [J] in [0, n_classes) */
  double class_var;         /* >= 0; 0 gives the independent Normal prior */
} ora_groups;

/* log p(beta) of the grouped prior, constants dropped:
 * -sum_c (sum_{j in c} beta_j^2 - kappa_c S_c^2) / (2 var), S_c = sum_{j in c} beta_j. */
double ora_log_prior_grouped(double var, const ora_groups* gr, int32_t J, const double* beta);

/* Eq. 4 under the grouped prior: d log p / d beta_j = -(beta_j - kappa S)/var,
 * d2 log p / d beta_j^2 = -(1 - kappa)/var, with S the class sum at beta. */
double ora_newton_step_grouped(double var, double kappa, double beta_j, double class_sum, double g, double h);

/* Algorithm 1 under the grouped prior (arguments as ora_ccd). */
int ora_ccd_grouped(const ora_problem* p, double var, const ora_groups* gr, double* beta_io, double* trust_io,
                    int32_t max_sweeps, int32_t criterion, double tol, ora_result* res, double* trace,
                    double* logpost_trace);

/* Algorithm 1.  beta_io/trust_io ([J]) hold the start point (warm start) and
 * receive the result.  criterion/tol select the stopping rule; at most
 * max_sweeps cycles run.  trace (nullable) receives g, h, delta-beta of every
 * visit as [sweep][j][3]; logpost_trace (nullable) the log posterior after
 * each sweep.  Returns 0 on success, negative on invalid input. */
int ora_ccd(const ora_problem* p, int32_t prior_kind, double var, double* beta_io,
            double* trust_io, int32_t max_sweeps, int32_t criterion, double tol,
            ora_result* res, double* trace, double* logpost_trace);

#ifdef __cplusplus
}
#endif
#endif
