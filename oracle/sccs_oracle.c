/*
 * Plain FP64 CPU oracle for cyclic coordinate descent on the Bayesian
 * self-controlled case series model.  TEST INFRASTRUCTURE ONLY (see the
 * header): the product path never includes, links or calls it.
 *
 * Notation follows the paper (Sections 2.1-2.3):
 *   i = 1..N patients, k = eras (rows of X), j = 1..J drugs (columns of X),
 *   l_k era length, y_k event count, n_i = sum_k y_ik,
 *   eta = X beta, w = L x exp(X beta), den_i = M[w]_i, num_ij = M[w x X_j]_i,
 *   W = num/den (Eq. 8).
 * Patient weights omega_i (1 by default) multiply patient i's whole
 * log-likelihood term; they express cross-validation folds (0/1) and
 * bootstrap resamples (counts).
 *
 * Covariates are binary drug exposures unless the problem carries values
 * x_kj (Section 4 names dense, non-binary covariates such as baseline
 * measurements).  Then eta_k = sum_j x_kj beta_j, and differentiating Eq. 2
 * twice along beta_j gives, with A_i = M[w x X_j]_i / den_i and
 * B_i = M[w x X_j^2]_i / den_i,
 *   g_j = sum_i omega_i (sum_k y_ik x_kj) - sum_i omega_i n_i A_i,
 *   h_j = -sum_i omega_i n_i (B_i - A_i^2);
 * for binary x, B = A = W and this is Eq. 9's W(1 - W).  The binary case
 * keeps the formulas of Eqs. 7-9 as written.
 */
#include "sccs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static double weight_of(const ora_problem* p, int64_t i) {
  return p->weight ? (double)p->weight[i] : 1.0;
}

/* x of the CSC entry e (1 for a binary problem) */
static double value_of(const ora_problem* p, int64_t e) {
  return p->value ? p->value[e] : 1.0;
}

static int check_problem(const ora_problem* p) {
  if (!p || p->n_patients < 0 || p->n_rows < 0 || p->n_cols < 0) return -1;
  if (!p->patient_ptr || !p->col_ptr) return -1;
  if (p->patient_ptr[0] != 0 || p->patient_ptr[p->n_patients] != p->n_rows) return -1;
  if (p->col_ptr[0] != 0) return -1;
  return 0;
}

/* eta = X beta, accumulated column by column from the CSC storage. */
static void linear_predictor(const ora_problem* p, const double* beta, double* eta) {
  for (int64_t k = 0; k < p->n_rows; ++k) eta[k] = 0.0;
  for (int32_t j = 0; j < p->n_cols; ++j)
    for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
      if (p->value) eta[p->row_idx[e]] += p->value[e] * beta[j];
      else eta[p->row_idx[e]] += beta[j];
    }
}

/* Eq. 2: L(beta) = sum_i omega_i [ sum_k y_ik x_ik'beta - n_i log sum_k l_ik exp(x_ik'beta) ]. */
int ora_loglik(const ora_problem* p, const double* beta, double* loglik) {
  if (check_problem(p) || !beta || !loglik) return -1;
  double* eta = (double*)malloc(sizeof(double) * (size_t)(p->n_rows > 0 ? p->n_rows : 1));
  if (!eta) return -2;
  linear_predictor(p, beta, eta);
  double total = 0.0;
  for (int64_t i = 0; i < p->n_patients; ++i) {
    double lin = 0.0, s = 0.0, n = 0.0;
    for (int64_t k = p->patient_ptr[i]; k < p->patient_ptr[i + 1]; ++k) {
      lin += (double)p->count[k] * eta[k];
      s += (double)p->offset[k] * exp(eta[k]);
      n += (double)p->count[k];
    }
    if (n > 0.0) total += weight_of(p, i) * (lin - n * log(s));
  }
  free(eta);
  *loglik = total;
  return 0;
}

/* log of the Eq. 3 priors, constants dropped.  Laplace(0, var) is read with
 * var as its variance: density (lambda/2) exp(-lambda |b|), lambda = sqrt(2/var). */
double ora_log_prior(int32_t kind, double var, int32_t J, const double* beta) {
  double s = 0.0;
  if (kind == ORA_PRIOR_NORMAL) {
    for (int32_t j = 0; j < J; ++j) s -= beta[j] * beta[j] / (2.0 * var);
  } else if (kind == ORA_PRIOR_LAPLACE) {
    double lambda = sqrt(2.0 / var);
    for (int32_t j = 0; j < J; ++j) s -= lambda * fabs(beta[j]);
  }
  return s;
}

/* Eqs. 7-9 at beta, written out from the definitions:
 *   g_j = Y'X_j - N'W,   h_j = -N'[W x (1 - W)],   W = M[w x X_j] / M[w]. */
int ora_grad_hess(const ora_problem* p, const double* beta, int32_t j, double* g, double* h) {
  if (check_problem(p) || !beta || !g || !h || j < 0 || j >= p->n_cols) return -1;
  int64_t K = p->n_rows, N = p->n_patients;
  double* eta = (double*)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
  double* num = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
  double* num2 = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
  double* den = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
  double* nn = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
  int32_t* pid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
  if (!eta || !num || !num2 || !den || !nn || !pid) {
    free(eta); free(num); free(num2); free(den); free(nn); free(pid);
    return -2;
  }
  linear_predictor(p, beta, eta);
  double yx = 0.0;
  for (int64_t i = 0; i < N; ++i)
    for (int64_t k = p->patient_ptr[i]; k < p->patient_ptr[i + 1]; ++k) {
      pid[k] = (int32_t)i;
      den[i] += (double)p->offset[k] * exp(eta[k]);
      nn[i] += (double)p->count[k];
    }
  for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
    int64_t k = p->row_idx[e];
    int32_t i = pid[k];
    double x = value_of(p, e);
    num[i] += (double)p->offset[k] * exp(eta[k]) * x;
    num2[i] += (double)p->offset[k] * exp(eta[k]) * x * x;
    yx += weight_of(p, i) * (double)p->count[k] * x;
  }
  double G = 0.0, H = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    if (num[i] == 0.0 && num2[i] == 0.0) continue;
    double wn = weight_of(p, i) * nn[i];
    if (p->value) {
      double A = num[i] / den[i], B = num2[i] / den[i];
      G += wn * A;
      H += wn * (B - A * A);
    } else {
      double W = num[i] / den[i];
      G += wn * W;
      H += wn * W * (1.0 - W);
    }
  }
  *g = yx - G;
  *h = -H;
  free(eta); free(num); free(num2); free(den); free(nn); free(pid);
  return 0;
}

/* Eq. 4: delta = -(g + d/db log p) / (h + d2/db2 log p), maximising P.
 *
 * Normal prior: d log p = -beta_j/var, d2 log p = -1/var.
 * Laplace prior (lambda = sqrt(2/var)) is not differentiable at zero; the
 * step follows the coordinate rules of Genkin et al. (2007), the method the
 * paper cites for its update:
 *   beta_j > 0: step on the smooth branch -lambda; if it crosses zero, stop at 0.
 *   beta_j < 0: step on the smooth branch +lambda; if it crosses zero, stop at 0.
 *   beta_j = 0: move only if |g| > lambda (strict), toward the side of g.
 * Without curvature (h >= 0, possible only when every W is 0 or 1) the
 * likelihood is flat in beta_j and no step is taken (prior none / Laplace). */
double ora_newton_step(int32_t kind, double var, double beta_j, double g, double h) {
  if (kind == ORA_PRIOR_NORMAL) {
    return -(g - beta_j / var) / (h - 1.0 / var);
  }
  double lambda = (kind == ORA_PRIOR_LAPLACE) ? sqrt(2.0 / var) : 0.0;
  if (!(h < 0.0)) return 0.0;
  double dv;
  if (beta_j > 0.0) {
    dv = -(g - lambda) / h;
    if (beta_j + dv < 0.0) dv = -beta_j;
  } else if (beta_j < 0.0) {
    dv = -(g + lambda) / h;
    if (beta_j + dv > 0.0) dv = -beta_j;
  } else {
    if (g > lambda) dv = -(g - lambda) / h;
    else if (g < -lambda) dv = -(g + lambda) / h;
    else dv = 0.0;
  }
  return dv;
}

/* Adaptable trust region (Genkin et al. 2007): the step is clipped to
 * [-trust_j, trust_j]; afterwards trust_j <- max(2 |step|, trust_j / 2).
 * The bound is updated on every visit, including visits with a zero step. */
double ora_trust_clamp(double dv, double* trust_io) {
  double t = *trust_io;
  double d = dv;
  if (d > t) d = t;
  if (d < -t) d = -t;
  double a = 2.0 * fabs(d), b = 0.5 * t;
  *trust_io = a > b ? a : b;
  return d;
}

/* Members of class c and kappa_c = class_var / (var + m_c class_var). */
static double group_kappa(double var, const ora_groups* gr, int32_t J, int32_t c) {
  int32_t m = 0;
  for (int32_t j = 0; j < J; ++j) m += gr->class_of[j] == c;
  return gr->class_var / (var + (double)m * gr->class_var);
}

static double group_sum(const ora_groups* gr, int32_t J, int32_t c, const double* beta) {
  double s = 0.0;
  for (int32_t j = 0; j < J; ++j)
    if (gr->class_of[j] == c) s += beta[j];
  return s;
}

double ora_log_prior_grouped(double var, const ora_groups* gr, int32_t J, const double* beta) {
  double q = 0.0;
  for (int32_t j = 0; j < J; ++j) q += beta[j] * beta[j];
  for (int32_t c = 0; c < gr->n_classes; ++c) {
    double S = group_sum(gr, J, c, beta);
    q -= group_kappa(var, gr, J, c) * S * S;
  }
  return -q / (2.0 * var);
}

double ora_newton_step_grouped(double var, double kappa, double beta_j, double class_sum, double g, double h) {
  return -(g - (beta_j - kappa * class_sum) / var) / (h - (1.0 - kappa) / var);
}

static int ccd_run(const ora_problem* p, int32_t prior_kind, double var, const ora_groups* gr, double* beta,
                   double* trust, int32_t max_sweeps, int32_t criterion, double tol, ora_result* res, double* trace,
                   double* logpost_trace);

int ora_ccd(const ora_problem* p, int32_t prior_kind, double var, double* beta, double* trust, int32_t max_sweeps,
            int32_t criterion, double tol, ora_result* res, double* trace, double* logpost_trace) {
  return ccd_run(p, prior_kind, var, NULL, beta, trust, max_sweeps, criterion, tol, res, trace, logpost_trace);
}

int ora_ccd_grouped(const ora_problem* p, double var, const ora_groups* gr, double* beta, double* trust,
                    int32_t max_sweeps, int32_t criterion, double tol, ora_result* res, double* trace,
                    double* logpost_trace) {
  if (!gr || !gr->class_of || gr->n_classes < 1 || !(gr->class_var >= 0.0)) return -1;
  for (int32_t j = 0; j < p->n_cols; ++j)
    if (gr->class_of[j] < 0 || gr->class_of[j] >= gr->n_classes) return -1;
  return ccd_run(p, ORA_PRIOR_NORMAL, var, gr, beta, trust, max_sweeps, criterion, tol, res, trace, logpost_trace);
}

/* log prior of either kind */
static double log_prior_of(int32_t kind, double var, const ora_groups* gr, int32_t J, const double* beta) {
  return gr ? ora_log_prior_grouped(var, gr, J, beta) : ora_log_prior(kind, var, J, beta);
}

/* Algorithm 1 (cyclic coordinate descent), coordinates visited j = 0..J-1 in
 * order every sweep.  State: eta = X beta, w = L x exp(eta) per era and
 * den = M[w] per patient.  After a nonzero step on column j the three are
 * brought up to date (Steps 1-3 of Section 2.4): eta and w on the column's
 * rows, and den recomputed from all eras of every patient the column touches
 * (an exact recomputation rather than an increment). */
static int ccd_run(const ora_problem* p, int32_t prior_kind, double var, const ora_groups* gr, double* beta,
                   double* trust, int32_t max_sweeps, int32_t criterion, double tol, ora_result* res, double* trace,
                   double* logpost_trace) {
  if (check_problem(p) || !beta || !trust || !res || max_sweeps < 0) return -1;
  if ((prior_kind == ORA_PRIOR_NORMAL || prior_kind == ORA_PRIOR_LAPLACE) && !(var > 0.0)) return -1;
  int64_t K = p->n_rows, N = p->n_patients;
  int32_t J = p->n_cols;
  size_t KK = (size_t)(K > 0 ? K : 1), NN = (size_t)(N > 0 ? N : 1);
  double* eta = (double*)malloc(sizeof(double) * KK);
  double* eta_prev = (double*)malloc(sizeof(double) * KK);
  double* w = (double*)malloc(sizeof(double) * KK);
  int32_t* pid = (int32_t*)malloc(sizeof(int32_t) * KK);
  double* den = (double*)malloc(sizeof(double) * NN);
  double* num = (double*)calloc(NN, sizeof(double));
  double* num2 = (double*)calloc(NN, sizeof(double));    /* M[w x X_j^2], covariate values only */
  double* wn = (double*)malloc(sizeof(double) * NN);     /* omega_i n_i */
  double* ytx = (double*)malloc(sizeof(double) * (size_t)(J > 0 ? J : 1));
  int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * NN);
  if (!eta || !eta_prev || !w || !pid || !den || !num || !num2 || !wn || !ytx || !touched) {
    free(eta); free(eta_prev); free(w); free(pid); free(den); free(num); free(num2); free(wn); free(ytx);
    free(touched);
    return -2;
  }

  /* problem-derived constants: pid(k), omega_i n_i, Y'X_j (weighted) */
  for (int64_t i = 0; i < N; ++i) {
    double n = 0.0;
    for (int64_t k = p->patient_ptr[i]; k < p->patient_ptr[i + 1]; ++k) {
      pid[k] = (int32_t)i;
      n += (double)p->count[k];
    }
    wn[i] = weight_of(p, i) * n;
  }
  for (int32_t j = 0; j < J; ++j) {
    double s = 0.0;
    for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
      int64_t k = p->row_idx[e];
      s += weight_of(p, pid[k]) * (double)p->count[k] * value_of(p, e);
    }
    ytx[j] = s;
  }

  /* initial state from the start point (beta = 0 gives eta = 0, w = L, den = M L) */
  linear_predictor(p, beta, eta);
  for (int64_t k = 0; k < K; ++k) w[k] = (double)p->offset[k] * exp(eta[k]);
  for (int64_t i = 0; i < N; ++i) {
    double s = 0.0;
    for (int64_t k = p->patient_ptr[i]; k < p->patient_ptr[i + 1]; ++k) s += w[k];
    den[i] = s;
  }

  double lp_prev = 0.0;
  if (criterion == ORA_CRIT_REL_LOGPOST) {
    double L;
    ora_loglik(p, beta, &L);
    lp_prev = L + log_prior_of(prior_kind, var, gr, J, beta);
  }
  int32_t sweep = 0, converged = 0;
  while (sweep < max_sweeps) {
    if (criterion == ORA_CRIT_ABS_DXBETA) memcpy(eta_prev, eta, sizeof(double) * KK);
    for (int32_t j = 0; j < J; ++j) {
      /* Step 4: num_i = M[w x X_j]_i over the patients of column j */
      int32_t nt = 0;
      for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
        int64_t k = p->row_idx[e];
        int32_t i = pid[k];
        if (nt == 0 || touched[nt - 1] != i) touched[nt++] = i;
        if (p->value) {
          num[i] += w[k] * p->value[e];
          num2[i] += w[k] * p->value[e] * p->value[e];
        } else {
          num[i] += w[k];
        }
      }
      /* fused transform and the two inner products N'W and N'[W(1-W)]
       * (general form with covariate values: N'A and N'(B - A^2)) */
      double G = 0.0, H = 0.0;
      for (int32_t t = 0; t < nt; ++t) {
        int32_t i = touched[t];
        /* W_i = 0 adds nothing (also when all of the patient's eras have
         * length 0, where den_i = 0 too and such a patient has n_i = 0) */
        if (num[i] == 0.0 && num2[i] == 0.0) continue;
        if (p->value) {
          double A = num[i] / den[i], B = num2[i] / den[i];
          G += wn[i] * A;
          H += wn[i] * (B - A * A);
        } else {
          double W = num[i] / den[i];
          G += wn[i] * W;
          H += wn[i] * W * (1.0 - W);
        }
      }
      double g = ytx[j] - G, h = -H;
      double dv;
      if (gr) {   /* the class sum at the current beta, recomputed at every visit */
        int32_t c = gr->class_of[j];
        dv = ora_newton_step_grouped(var, group_kappa(var, gr, J, c), beta[j], group_sum(gr, J, c, beta), g, h);
      } else {
        dv = ora_newton_step(prior_kind, var, beta[j], g, h);
      }
      double db = ora_trust_clamp(dv, &trust[j]);
      if (trace) {
        double* tr = trace + ((size_t)sweep * (size_t)J + (size_t)j) * 3;
        tr[0] = g; tr[1] = h; tr[2] = db;
      }
      if (db != 0.0) {
        beta[j] += db;
        for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
          int64_t k = p->row_idx[e];
          if (p->value) eta[k] += db * p->value[e];
          else eta[k] += db;
          w[k] = (double)p->offset[k] * exp(eta[k]);
        }
        for (int32_t t = 0; t < nt; ++t) {
          int32_t i = touched[t];
          double s = 0.0;
          for (int64_t k = p->patient_ptr[i]; k < p->patient_ptr[i + 1]; ++k) s += w[k];
          den[i] = s;
        }
      }
      for (int32_t t = 0; t < nt; ++t) num[touched[t]] = num2[touched[t]] = 0.0;
    }
    ++sweep;
    double L;
    ora_loglik(p, beta, &L);
    double lp = L + log_prior_of(prior_kind, var, gr, J, beta);
    if (logpost_trace) logpost_trace[sweep - 1] = lp;
    if (criterion == ORA_CRIT_REL_LOGPOST) {
      if (fabs(lp - lp_prev) < tol * fabs(lp)) { converged = 1; }
      lp_prev = lp;
    } else if (criterion == ORA_CRIT_ABS_DXBETA) {
      double s = 0.0;
      for (int64_t k = 0; k < K; ++k) s += fabs(eta[k] - eta_prev[k]);
      if (s < tol) converged = 1;
    }
    if (converged) break;
  }
  double L;
  ora_loglik(p, beta, &L);
  res->sweeps = sweep;
  res->converged = converged;
  res->loglik = L;
  res->logpost = L + log_prior_of(prior_kind, var, gr, J, beta);
  free(eta); free(eta_prev); free(w); free(pid); free(den); free(num); free(num2); free(wn); free(ytx);
  free(touched);
  return 0;
}
