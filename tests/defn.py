"""Independent NumPy definitions used to pin the oracle (test helper).

Nothing here is derived from the oracle's code.  The log-likelihood is Eq. 2
written over complex numbers so that derivatives can be taken by the complex
step; the full gradient and Hessian use the textbook multinomial (conditional
logit) form of each patient's term,

    grad L_i = sum_k y_ik x_ik - n_i mu_i,
    Hess L_i = -n_i ( sum_k pi_ik x_ik x_ik' - mu_i mu_i' ),

with pi_ik = l_ik exp(x_ik'beta) / sum_k' l_ik' exp(x_ik''beta) and
mu_i = sum_k pi_ik x_ik, which is a different route to the quantities that
the paper's Eqs. 7-9 give one coordinate at a time.
"""
from __future__ import annotations

import numpy as np


def dense_x(prob) -> np.ndarray:
    """X as a dense [K, J] matrix: ones at the stored entries of a binary
    problem, the stored covariate values otherwise."""
    X = np.zeros((prob.n_rows, prob.n_cols))
    v = getattr(prob, "value", None)
    for j in range(prob.n_cols):
        sl = slice(prob.col_ptr[j], prob.col_ptr[j + 1])
        X[prob.row_idx[sl], j] = 1.0 if v is None else v[sl]
    return X


def patient_of_row(prob) -> np.ndarray:
    return np.repeat(np.arange(prob.n_patients), np.diff(prob.patient_ptr))


def weights(prob, weight=None) -> np.ndarray:
    return np.ones(prob.n_patients) if weight is None else np.asarray(weight, dtype=np.float64)


def loglik(prob, beta, weight=None, X=None) -> complex:
    """Eq. 2 in complex arithmetic (analytic in beta)."""
    X = dense_x(prob) if X is None else X
    pid = patient_of_row(prob)
    om = weights(prob, weight)
    eta = X @ np.asarray(beta)
    y = prob.count.astype(np.float64)
    l = prob.offset.astype(np.float64)
    N = prob.n_patients
    lin = np.zeros(N, dtype=complex)
    s = np.zeros(N, dtype=complex)
    n = np.zeros(N)
    np.add.at(lin, pid, y * eta)
    np.add.at(s, pid, l * np.exp(eta))
    np.add.at(n, pid, y)
    keep = n > 0
    return np.sum(om[keep] * (lin[keep] - n[keep] * np.log(s[keep])))


def grad_cs(prob, beta, j, weight=None, X=None, step=1e-30) -> float:
    """dL/dbeta_j by the complex step: Im L(beta + i h e_j) / h."""
    b = np.asarray(beta, dtype=complex).copy()
    b[j] += 1j * step
    return float(np.imag(loglik(prob, b, weight, X)) / step)


def hess_fd(prob, beta, j, weight=None, X=None, eps=1e-3) -> float:
    """d2L/dbeta_j^2: Richardson-extrapolated central difference of the
    complex-step gradient (error O(eps^4))."""
    def d(e):
        bp = np.array(beta, dtype=np.float64); bp[j] += e
        bm = np.array(beta, dtype=np.float64); bm[j] -= e
        return (grad_cs(prob, bp, j, weight, X) - grad_cs(prob, bm, j, weight, X)) / (2 * e)
    return (4.0 * d(eps / 2) - d(eps)) / 3.0


def grad_hess_full(prob, beta, weight=None, X=None):
    """Full gradient and Hessian of L, multinomial form (see module doc)."""
    X = dense_x(prob) if X is None else X
    pid = patient_of_row(prob)
    om = weights(prob, weight)
    y = prob.count.astype(np.float64)
    l = prob.offset.astype(np.float64)
    eta = X @ np.asarray(beta, dtype=np.float64)
    J = prob.n_cols
    g = np.zeros(J)
    H = np.zeros((J, J))
    for i in range(prob.n_patients):
        lo, hi = prob.patient_ptr[i], prob.patient_ptr[i + 1]
        yi = y[lo:hi]
        ni = yi.sum()
        if ni == 0 or om[i] == 0:
            continue
        a = l[lo:hi] * np.exp(eta[lo:hi] - eta[lo:hi].max())
        pi = a / a.sum()
        Xi = X[lo:hi]
        mu = pi @ Xi
        g += om[i] * (yi @ Xi - ni * mu)
        H -= om[i] * ni * ((Xi * pi[:, None]).T @ Xi - np.outer(mu, mu))
    return g, H


def log_prior(kind, var, beta):
    beta = np.asarray(beta)
    if kind == 1:
        return -np.sum(beta ** 2) / (2 * var)
    if kind == 2:
        return -np.sqrt(2.0 / var) * np.sum(np.abs(beta))
    return 0.0
