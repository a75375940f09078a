"""Python access to the plain FP64 CPU oracle (oracle/sccs_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path
(``paper_1208_0945_amd``) never does.  It shares no code with the HIP
library; only the seeded input generator feeds both.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsccs_oracle.so")
SRC_PATH = os.path.join(HERE, "sccs_oracle.c")

PRIOR_NONE, PRIOR_NORMAL, PRIOR_LAPLACE = 0, 1, 2
CRIT_FIXED, CRIT_REL_LOGPOST, CRIT_ABS_DXBETA = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-o", LIB_PATH, SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [("n_patients", ctypes.c_int32), ("n_rows", ctypes.c_int64),
                ("n_cols", ctypes.c_int32), ("patient_ptr", ctypes.c_void_p),
                ("offset", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("col_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p),
                ("weight", ctypes.c_void_p), ("value", ctypes.c_void_p)]


class _Groups(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("class_of", ctypes.c_void_p), ("class_var", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("loglik", ctypes.c_double), ("logpost", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        L.ora_loglik.argtypes = [P, ctypes.c_void_p, dp]
        L.ora_loglik.restype = ctypes.c_int
        L.ora_log_prior.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p]
        L.ora_log_prior.restype = ctypes.c_double
        L.ora_grad_hess.argtypes = [P, ctypes.c_void_p, ctypes.c_int32, dp, dp]
        L.ora_grad_hess.restype = ctypes.c_int
        L.ora_newton_step.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double]
        L.ora_newton_step.restype = ctypes.c_double
        L.ora_trust_clamp.argtypes = [ctypes.c_double, dp]
        L.ora_trust_clamp.restype = ctypes.c_double
        L.ora_ccd.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                              ctypes.POINTER(_Result), ctypes.c_void_p, ctypes.c_void_p]
        L.ora_ccd.restype = ctypes.c_int
        G = ctypes.POINTER(_Groups)
        L.ora_log_prior_grouped.argtypes = [ctypes.c_double, G, ctypes.c_int32, ctypes.c_void_p]
        L.ora_log_prior_grouped.restype = ctypes.c_double
        L.ora_newton_step_grouped.argtypes = [ctypes.c_double] * 6
        L.ora_newton_step_grouped.restype = ctypes.c_double
        L.ora_ccd_grouped.argtypes = [P, ctypes.c_double, G, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      ctypes.POINTER(_Result), ctypes.c_void_p, ctypes.c_void_p]
        L.ora_ccd_grouped.restype = ctypes.c_int
        _lib = L
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class OracleProblem:
    """Keeps contiguous copies of the arrays alive for the C structure."""

    def __init__(self, prob, weight: Optional[np.ndarray] = None):
        self.patient_ptr = _c(prob.patient_ptr, np.int64)
        self.offset = _c(prob.offset, np.int32)
        self.count = _c(prob.count, np.int32)
        self.col_ptr = _c(prob.col_ptr, np.int64)
        self.row_idx = _c(prob.row_idx, np.int32)
        self.weight = None if weight is None else _c(weight, np.int32)
        v = getattr(prob, "value", None)
        self.value = None if v is None else _c(v, np.float64)
        self.J = int(prob.n_cols)
        self.s = _Problem(int(prob.n_patients), int(self.patient_ptr[-1]), self.J,
                          self.patient_ptr.ctypes.data, self.offset.ctypes.data,
                          self.count.ctypes.data, self.col_ptr.ctypes.data,
                          self.row_idx.ctypes.data,
                          None if self.weight is None else self.weight.ctypes.data,
                          None if self.value is None else self.value.ctypes.data)


def _prob(prob, weight=None) -> OracleProblem:
    return prob if isinstance(prob, OracleProblem) else OracleProblem(prob, weight)


def loglik(prob, beta, weight=None) -> float:
    P = _prob(prob, weight)
    b = _c(beta, np.float64)
    out = ctypes.c_double()
    rc = lib().ora_loglik(ctypes.byref(P.s), b.ctypes.data, ctypes.byref(out))
    if rc:
        raise ValueError(f"ora_loglik failed ({rc})")
    return out.value


def log_prior(kind: int, var: float, beta) -> float:
    b = _c(beta, np.float64)
    return lib().ora_log_prior(kind, var, len(b), b.ctypes.data)


def grad_hess(prob, beta, j: int, weight=None) -> Tuple[float, float]:
    P = _prob(prob, weight)
    b = _c(beta, np.float64)
    g, h = ctypes.c_double(), ctypes.c_double()
    rc = lib().ora_grad_hess(ctypes.byref(P.s), b.ctypes.data, int(j), ctypes.byref(g), ctypes.byref(h))
    if rc:
        raise ValueError(f"ora_grad_hess failed ({rc})")
    return g.value, h.value


def newton_step(kind: int, var: float, beta_j: float, g: float, h: float) -> float:
    return lib().ora_newton_step(kind, var, beta_j, g, h)


def trust_clamp(dv: float, trust: float) -> Tuple[float, float]:
    t = ctypes.c_double(trust)
    d = lib().ora_trust_clamp(dv, ctypes.byref(t))
    return d, t.value


def ccd(prob, prior_kind: int, var: float, max_sweeps: int, criterion: int = CRIT_FIXED,
        tol: float = 0.0, beta0=None, trust0=None, weight=None, want_trace: bool = False):
    """Run Algorithm 1.  Returns dict(beta, trust, sweeps, converged, loglik,
    logpost, trace[sweeps, J, 3] or None, logpost_trace[sweeps])."""
    P = _prob(prob, weight)
    J = P.J
    beta = np.zeros(J) if beta0 is None else _c(beta0, np.float64).copy()
    trust = np.ones(J) if trust0 is None else _c(trust0, np.float64).copy()
    res = _Result()
    trace = np.zeros((max(max_sweeps, 1), J, 3)) if want_trace else None
    lpt = np.zeros(max(max_sweeps, 1))
    rc = lib().ora_ccd(ctypes.byref(P.s), int(prior_kind), float(var), beta.ctypes.data,
                       trust.ctypes.data, int(max_sweeps), int(criterion), float(tol),
                       ctypes.byref(res), None if trace is None else trace.ctypes.data,
                       lpt.ctypes.data)
    if rc:
        raise ValueError(f"ora_ccd failed ({rc})")
    n = res.sweeps
    return {"beta": beta, "trust": trust, "sweeps": n, "converged": bool(res.converged),
            "loglik": res.loglik, "logpost": res.logpost,
            "trace": None if trace is None else trace[:n], "logpost_trace": lpt[:n]}


def _quantile_sorted(x, q: float) -> float:
    """Quantile of an ascending list at probability q by linear interpolation
    between order statistics at position (R - 1) q (the paper names no
    quantile rule; this is the common default, Hyndman and Fan's type 7)."""
    pos = (len(x) - 1) * q
    k = int(np.floor(pos))
    k1 = min(k + 1, len(x) - 1)
    return x[k] + (pos - k) * (x[k1] - x[k])


def bootstrap_summary(betas, level: float = 0.95):
    """Section 2.5, non-parametric bootstrap: per coefficient j, the interval
    from the (1 - level)/2 and (1 + level)/2 quantiles of the replicate
    estimates, and p_hat_j, the share of replicates whose MAP estimate of
    beta_j is not zero.  betas: [R, J].  Returns (lo, hi, p_hat)."""
    B = np.asarray(betas, dtype=np.float64)
    R, J = B.shape
    lo, hi, p_hat = np.zeros(J), np.zeros(J), np.zeros(J)
    for j in range(J):
        x = sorted(float(v) for v in B[:, j])
        lo[j] = _quantile_sorted(x, 0.5 * (1.0 - level))
        hi[j] = _quantile_sorted(x, 0.5 * (1.0 + level))
        p_hat[j] = sum(1 for v in x if v != 0.0) / R
    return lo, hi, p_hat


def bootstrap(prob, prior_kind: int, var: float, weights, max_sweeps: int, criterion: int = CRIT_FIXED,
              tol: float = 0.0, level: float = 0.95):
    """One Algorithm 1 fit per replicate, from beta = 0, with the replicate's
    patient weights (weights: [R, N]); then bootstrap_summary.  Returns
    dict(beta [R, J], sweeps [R], lo, hi, p_hat)."""
    W = np.asarray(weights)
    fits = [ccd(prob, prior_kind, var, max_sweeps, criterion, tol, weight=W[r]) for r in range(W.shape[0])]
    betas = np.array([f["beta"] for f in fits])
    lo, hi, p_hat = bootstrap_summary(betas, level)
    return {"beta": betas, "sweeps": np.array([f["sweeps"] for f in fits]), "lo": lo, "hi": hi, "p_hat": p_hat}


def cv_predictive_loglik(prob, folds, n_folds: int, prior_kind: int, var: float, max_sweeps: int,
                         criterion: int = CRIT_REL_LOGPOST, tol: float = 1e-10, beta0=None):
    """Section 2.5: sum over folds of Eq. 2 over the fold's patients at the
    MAP fitted on the other folds.  beta0: optional [n_folds, J] start points.
    Returns (predictive log-likelihood, [n_folds, J] fold betas)."""
    folds = np.asarray(folds)
    total, betas = 0.0, []
    for f in range(n_folds):
        train = (folds != f).astype(np.int32)
        held = (folds == f).astype(np.int32)
        r = ccd(prob, prior_kind, var, max_sweeps, criterion, tol, weight=train,
                beta0=None if beta0 is None else beta0[f])
        total += loglik(prob, r["beta"], weight=held)
        betas.append(r["beta"])
    return total, np.array(betas)


def cv_search(prob, folds, n_folds: int, prior_kind: int, var_start: float, bracket_step: float, log10_tol: float,
              max_evals: int, max_sweeps: int, criterion: int = CRIT_REL_LOGPOST, tol: float = 1e-10,
              warm_start: bool = True):
    """Bracketing and golden-section search of the predictive log-likelihood
    over t = log10(variance) (Section 2.5 suggests an initial bracketing and
    an intervaled line search in place of a fixed grid):
    evaluate t0 and t0 + s; walk on by s in the rising direction until a
    value falls (the bracket); then golden-section steps inside the bracket,
    each new point in the larger part at (3 - sqrt 5)/2 of it from the best
    point, until the bracket is narrower than log10_tol.  Each evaluation
    starts every fold from its fit at the nearest evaluated variance (in
    log) when warm_start is set.  Returns dict(variance, pred_loglik [per
    evaluation], best, bracketed)."""
    evals_t, evals_f, evals_beta = [], [], []

    def f_at(t):
        if len(evals_t) >= max_evals:
            raise StopIteration
        b0 = None
        if warm_start and evals_t:
            near = min(range(len(evals_t)), key=lambda e: abs(evals_t[e] - t))
            b0 = evals_beta[near]
        v, B = cv_predictive_loglik(prob, folds, n_folds, prior_kind, 10.0 ** t, max_sweeps, criterion, tol, b0)
        evals_t.append(t)
        evals_f.append(v)
        evals_beta.append(B)
        return v

    s = math.log10(bracket_step)
    bracketed = False
    try:
        a = math.log10(var_start)
        b = a + s
        fa, fb = f_at(a), f_at(b)
        step = s
        if fb < fa:
            a, b, fa, fb = b, a, fb, fa
            step = -s
        while True:
            c = b + step
            fc = f_at(c)
            if fc < fb:
                bracketed = True
                break
            a, fa, b, fb = b, fb, c, fc
        lo, hi = min(a, c), max(a, c)
        g = 0.5 * (3.0 - math.sqrt(5.0))
        while hi - lo > log10_tol:
            x = b + g * (hi - b) if hi - b > b - lo else b - g * (b - lo)
            fx = f_at(x)
            if fx > fb:
                if x > b:
                    lo = b
                else:
                    hi = b
                b, fb = x, fx
            else:
                if x > b:
                    hi = x
                else:
                    lo = x
    except StopIteration:
        pass
    var = [10.0 ** t for t in evals_t]
    return {"variance": np.array(var), "pred_loglik": np.array(evals_f),
            "best": int(np.argmax(evals_f)), "bracketed": bracketed}


def _groups(class_of, class_var):
    c = _c(class_of, np.int32)
    return _Groups(int(c.max()) + 1 if c.size else 1, c.ctypes.data, float(class_var)), c


def log_prior_grouped(var: float, class_of, class_var: float, beta) -> float:
    gr, keep = _groups(class_of, class_var)
    b = _c(beta, np.float64)
    return lib().ora_log_prior_grouped(float(var), ctypes.byref(gr), len(b), b.ctypes.data)


def newton_step_grouped(var, kappa, beta_j, class_sum, g, h) -> float:
    return lib().ora_newton_step_grouped(float(var), float(kappa), float(beta_j), float(class_sum), float(g), float(h))


def ccd_grouped(prob, var: float, class_of, class_var: float, max_sweeps: int, criterion: int = CRIT_FIXED,
                tol: float = 0.0, beta0=None, weight=None, want_trace: bool = False):
    """Algorithm 1 under the grouped Normal prior (see sccs_oracle.h)."""
    P = _prob(prob, weight)
    gr, keep = _groups(class_of, class_var)
    J = P.J
    beta = np.zeros(J) if beta0 is None else _c(beta0, np.float64).copy()
    trust = np.ones(J)
    res = _Result()
    trace = np.zeros((max(max_sweeps, 1), J, 3)) if want_trace else None
    lpt = np.zeros(max(max_sweeps, 1))
    rc = lib().ora_ccd_grouped(ctypes.byref(P.s), float(var), ctypes.byref(gr), beta.ctypes.data, trust.ctypes.data,
                               int(max_sweeps), int(criterion), float(tol), ctypes.byref(res),
                               None if trace is None else trace.ctypes.data, lpt.ctypes.data)
    if rc:
        raise ValueError(f"ora_ccd_grouped failed ({rc})")
    n = res.sweeps
    return {"beta": beta, "trust": trust, "sweeps": n, "converged": bool(res.converged),
            "loglik": res.loglik, "logpost": res.logpost,
            "trace": None if trace is None else trace[:n], "logpost_trace": lpt[:n]}


def independent_groups(prob, width: int = 4):
    """Column groups of the independence relabelling, as lists of columns.

    Coordinate descent visits the coordinates in a fixed cyclic order
    (Algorithm 1); the numbering of the drugs is the caller's.  This
    numbering is built greedily: columns are taken by decreasing number of
    nonzeros (ties: smaller index first) and each joins the earliest-opened
    group that still has fewer than `width` columns and shares no patient
    with any of them; if there is none it opens a new group.  Reading the
    groups in the order they were opened, each in joining order, gives the
    relabelling (independent_order).  Plain restatement for the tests: per
    patient, the groups holding one of its columns are kept in a table."""
    N, J = int(prob.n_patients), int(prob.n_cols)
    patient_of_row = np.repeat(np.arange(N), np.diff(np.asarray(prob.patient_ptr)))
    col_ptr = np.asarray(prob.col_ptr)
    pats = [np.unique(patient_of_row[prob.row_idx[col_ptr[j]:col_ptr[j + 1]]]) for j in range(J)]
    per_patient = np.zeros(N, dtype=np.int64)
    for p in pats:
        per_patient[p] += 1
    table = np.full((N, max(1, int(per_patient.max(initial=0)))), -1, dtype=np.int64)
    used = np.zeros(N, dtype=np.int64)
    sizes = np.diff(col_ptr)
    groups = []
    for j in sorted(range(J), key=lambda c: (-int(sizes[c]), c)):
        p = pats[j]
        taken = set(np.unique(table[p]).tolist()) if len(p) else set()
        home = None
        for g, members in enumerate(groups):
            if len(members) < width and g not in taken:
                home = g
                break
        if home is None:
            home = len(groups)
            groups.append([])
        groups[home].append(j)
        table[p, used[p]] = home
        used[p] += 1
    return groups


def independent_order(prob, width: int = 4) -> np.ndarray:
    """The relabelling: order[k] is the column visited k-th."""
    return np.array([j for g in independent_groups(prob, width) for j in g], dtype=np.int64)
