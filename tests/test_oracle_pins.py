"""Pins of the FP64 CPU oracle against facts fixed outside it.

Each test checks the oracle against something other than its own code:
derivatives of Eq. 2 by the complex step, exact rational arithmetic, a
hand-worked fixture, the classical one-drug SCCS estimator, a Poisson GLM
with patient fixed effects fitted by SciPy, a full multivariate Newton on the
textbook multinomial form, the KKT conditions of the lasso, and invariances
of the likelihood.
"""
import dataclasses
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.optimize

import defn
from paper_1208_0945_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def make(patient_ptr, offset, count, cols, J=None, name="hand"):
    J = len(cols) if J is None else J
    col_ptr = np.zeros(J + 1, dtype=np.int64)
    col_ptr[1:] = np.cumsum([len(c) for c in cols])
    row_idx = np.concatenate([np.asarray(c, dtype=np.int32) for c in cols]) if cols else np.zeros(0, np.int32)
    return synth.Problem(name=name, n_patients=len(patient_ptr) - 1,
                         patient_ptr=np.asarray(patient_ptr, np.int64),
                         offset=np.asarray(offset, np.int32), count=np.asarray(count, np.int32),
                         n_cols=J, col_ptr=col_ptr, row_idx=row_idx.astype(np.int32),
                         beta_true=np.zeros(J))


def small(seed, n_patients=150, n_cols=6, p=0.15, era_mean=4.0):
    rng = synth._rng(99, seed)
    beta = synth.sparse_beta(n_cols, 3, 0.5, rng)
    return synth.make_problem("small", n_patients, n_cols, era_mean, np.full(n_cols, p), beta,
                              seed_path=(99, seed, 1))


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ---------------------------------------------------------------- derivatives

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_grad_hess_match_complex_step_of_loglik(oracle_lib, seed):
    """g_j (Eqs. 7-8) equals dL/dbeta_j of Eq. 2 to machine precision; h_j
    (Eq. 9) equals the second derivative to finite-difference accuracy."""
    prob = small(seed)
    X = defn.dense_x(prob)
    beta = synth.random_beta(prob.n_cols, 0.7, seed)
    for j in range(prob.n_cols):
        g, h = oracle_lib.grad_hess(prob, beta, j)
        g_cs = defn.grad_cs(prob, beta, j, X=X)
        h_fd = defn.hess_fd(prob, beta, j, X=X)
        assert rel(g, g_cs) < 1e-11 or abs(g - g_cs) < 1e-10
        assert rel(h, h_fd) < 1e-8
        assert h <= 0.0


def test_grad_hess_with_weights_match_complex_step(oracle_lib):
    prob = small(5)
    X = defn.dense_x(prob)
    weight = synth._rng(5, 5).integers(0, 3, size=prob.n_patients).astype(np.int32)
    beta = synth.random_beta(prob.n_cols, 0.5, 3)
    for j in range(prob.n_cols):
        g, h = oracle_lib.grad_hess(prob, beta, j, weight=weight)
        assert abs(g - defn.grad_cs(prob, beta, j, weight, X)) < 1e-10 * max(1, abs(g))
        assert rel(h, defn.hess_fd(prob, beta, j, weight, X)) < 1e-8


def test_loglik_matches_complex_definition(oracle_lib):
    prob = small(7)
    beta = synth.random_beta(prob.n_cols, 0.4, 7)
    assert rel(oracle_lib.loglik(prob, beta), float(np.real(defn.loglik(prob, beta)))) < 1e-13


def test_textbook_full_gradient_hessian_match_complex_step():
    """The multinomial-form helpers used by the Newton pins are themselves
    pinned to Eq. 2 by the complex step."""
    prob = small(3, n_cols=4)
    X = defn.dense_x(prob)
    beta = synth.random_beta(prob.n_cols, 0.5, 1)
    g, H = defn.grad_hess_full(prob, beta, X=X)
    for j in range(prob.n_cols):
        assert abs(g[j] - defn.grad_cs(prob, beta, j, X=X)) < 1e-9 * max(1, abs(g[j]))
        assert rel(H[j, j], defn.hess_fd(prob, beta, j, X=X)) < 1e-8
    # an off-diagonal entry by differencing gradient j along k
    eps = 1e-4
    bp = beta.copy(); bp[1] += eps
    bm = beta.copy(); bm[1] -= eps
    d = (defn.grad_cs(prob, bp, 0, X=X) - defn.grad_cs(prob, bm, 0, X=X)) / (2 * eps)
    assert abs(H[0, 1] - d) < 1e-6 * max(1.0, abs(d))


# ---------------------------------------------------------------- exact values

def test_first_coordinate_at_zero_is_exact_rational(oracle_lib):
    """At beta = 0 the weights are the integer era lengths, so g_j and h_j are
    exact rationals computed here with Fractions from Eq. 2's structure."""
    prob = synth.tiny(n_patients=200, n_cols=5, seed=3)
    pid = defn.patient_of_row(prob)
    den = [Fraction(0)] * prob.n_patients
    n = [0] * prob.n_patients
    for k in range(prob.n_rows):
        den[pid[k]] += int(prob.offset[k])
        n[pid[k]] += int(prob.count[k])
    for j in range(prob.n_cols):
        rows = prob.column(j)
        num = {}
        yx = 0
        for k in rows:
            num[pid[k]] = num.get(pid[k], Fraction(0)) + int(prob.offset[k])
            yx += int(prob.count[k])
        G = sum(n[i] * (v / den[i]) for i, v in num.items())
        H = sum(n[i] * (v / den[i]) * (1 - v / den[i]) for i, v in num.items())
        g, h = oracle_lib.grad_hess(prob, np.zeros(prob.n_cols), j)
        assert rel(g, float(yx - G)) < 1e-13 or abs(g - float(yx - G)) < 1e-12
        assert rel(h, float(-H)) < 1e-13


def test_golden_two_patient_fixture(oracle_lib):
    with open(os.path.join(HERE, "golden", "two_patient.json")) as f:
        fx = json.load(f)
    P = fx["problem"]
    cols = [P["row_idx"][P["col_ptr"][j]:P["col_ptr"][j + 1]] for j in range(2)]
    prob = make(P["patient_ptr"], P["offset"], P["count"], cols)
    z = fx["at_beta_zero"]
    for j in range(2):
        g, h = oracle_lib.grad_hess(prob, np.zeros(2), j)
        assert abs(g - float(Fraction(z["g"][j]))) < 1e-15
        assert abs(h - float(Fraction(z["h"][j]))) < 1e-15
    assert abs(oracle_lib.loglik(prob, np.zeros(2)) - (-2 * math.log(60) - 2 * math.log(20))) < 1e-12
    r = oracle_lib.ccd(prob, oracle_lib.PRIOR_NORMAL, 1.0, 1, want_trace=True)
    nv = fx["first_visit_normal_var1"]
    assert abs(r["trace"][0, 0, 2] - float(Fraction(nv["dbeta0"]))) < 1e-15
    assert abs(r["trust"][0] - float(Fraction(nv["trust0"]))) < 1e-15
    r = oracle_lib.ccd(prob, oracle_lib.PRIOR_LAPLACE, 2.0, 1, want_trace=True)
    lv = fx["first_visits_laplace_var2"]
    for j in range(2):
        assert abs(r["trace"][0, j, 2] - float(Fraction(lv["dbeta"][j]))) < 1e-15
        assert abs(r["trust"][j] - float(Fraction(lv["trust"][j]))) < 1e-15


# ---------------------------------------------------------------- step rules

def test_newton_step_rules(oracle_lib):
    """Each branch of the single-coordinate step, values computed by hand."""
    ns = oracle_lib.newton_step
    N, LAP, NONE = oracle_lib.PRIOR_NORMAL, oracle_lib.PRIOR_LAPLACE, oracle_lib.PRIOR_NONE
    # Normal, var 2: -(g - b/var)/(h - 1/var) = -(3 - 0.5)/(-2 - 0.5) = 1
    assert ns(N, 2.0, 1.0, 3.0, -2.0) == pytest.approx(1.0, abs=1e-15)
    # none: plain Newton -g/h
    assert ns(NONE, 1.0, 0.3, 1.0, -4.0) == pytest.approx(0.25, abs=1e-15)
    assert ns(NONE, 1.0, 0.3, 1.0, 0.0) == 0.0
    # Laplace var 2 (lambda 1)
    assert ns(LAP, 2.0, 0.0, 0.5, -1.0) == 0.0          # |g| <= lambda: stay at 0
    assert ns(LAP, 2.0, 0.0, 1.0, -1.0) == 0.0          # tie: stay at 0
    assert ns(LAP, 2.0, 0.0, -1.0, -1.0) == 0.0         # tie on the other side
    assert ns(LAP, 2.0, 0.0, 3.0, -4.0) == pytest.approx(0.5)    # -(3-1)/(-4)
    assert ns(LAP, 2.0, 0.0, -3.0, -4.0) == pytest.approx(-0.5)  # -(-3+1)/(-4)
    assert ns(LAP, 2.0, 0.2, 2.0, -2.0) == pytest.approx(0.5)    # positive branch
    assert ns(LAP, 2.0, 0.2, -3.0, -2.0) == pytest.approx(-0.2)  # would cross: stop at 0
    assert ns(LAP, 2.0, -0.2, 3.0, -2.0) == pytest.approx(0.2)   # would cross: stop at 0
    assert ns(LAP, 2.0, -0.2, -2.0, -2.0) == pytest.approx(-0.5)
    assert ns(LAP, 2.0, 0.2, 2.0, 0.0) == 0.0           # no curvature
    # lambda = sqrt(2/var): var 0.5 gives lambda 2
    assert ns(LAP, 0.5, 0.0, 1.9, -1.0) == 0.0
    assert ns(LAP, 0.5, 0.0, 2.5, -1.0) == pytest.approx(0.5)


def test_trust_region_rules(oracle_lib):
    tc = oracle_lib.trust_clamp
    assert tc(0.3, 1.0) == (0.3, 0.6)
    assert tc(5.0, 1.0) == (1.0, 2.0)
    assert tc(-5.0, 0.25) == (-0.25, 0.5)
    assert tc(0.0, 1.0) == (0.0, 0.5)
    assert tc(0.1, 1.0) == (0.1, 0.5)


# ---------------------------------------------------------------- optima

def _ccd_converged(oracle_lib, prob, kind, var, weight=None, tol=1e-15, sweeps=3000):
    r = oracle_lib.ccd(prob, kind, var, sweeps, oracle_lib.CRIT_REL_LOGPOST, tol, weight=weight)
    return r


@pytest.mark.parametrize("kind,var", [(1, 1.0), (1, 0.1), (0, 1.0)])
def test_ccd_reaches_full_newton_optimum(oracle_lib, kind, var):
    """Multivariate Newton on P with the textbook Hessian (tiny, J = 6)."""
    prob = small(11, n_patients=300, n_cols=6, p=0.2)
    X = defn.dense_x(prob)
    b = np.zeros(prob.n_cols)
    for _ in range(60):
        g, H = defn.grad_hess_full(prob, b, X=X)
        if kind == 1:
            g = g - b / var
            H = H - np.eye(len(b)) / var
        step = np.linalg.solve(H, -g)
        b = b + step
        if np.max(np.abs(step)) < 1e-15:
            break
    g, _ = defn.grad_hess_full(prob, b, X=X)
    assert np.max(np.abs(g - (b / var if kind == 1 else 0))) < 1e-9
    r = _ccd_converged(oracle_lib, prob, kind, var)
    assert r["converged"]
    assert np.max(np.abs(r["beta"] - b)) < 1e-8
    # stationarity through the complex-step gradient: g_j - beta_j/var = 0
    for j in range(prob.n_cols):
        gj = defn.grad_cs(prob, r["beta"], j, X=X)
        target = r["beta"][j] / var if kind == 1 else 0.0
        assert abs(gj - target) < 1e-7


@pytest.mark.parametrize("var", [2.0, 0.05])
def test_ccd_laplace_satisfies_kkt_and_matches_lbfgsb(oracle_lib, var):
    prob = small(13, n_patients=300, n_cols=8, p=0.2)
    X = defn.dense_x(prob)
    lam = math.sqrt(2.0 / var)
    r = _ccd_converged(oracle_lib, prob, oracle_lib.PRIOR_LAPLACE, var)
    assert r["converged"]
    beta = r["beta"]
    for j in range(prob.n_cols):
        gj = defn.grad_cs(prob, beta, j, X=X)
        if beta[j] != 0.0:
            assert abs(gj - lam * np.sign(beta[j])) < 1e-6
        else:
            assert abs(gj) <= lam + 1e-9
    # split-variable bound-constrained fit with SciPy
    J = prob.n_cols

    def f(uv):
        u, v = uv[:J], uv[J:]
        b = u - v
        g, _ = defn.grad_hess_full(prob, b, X=X)
        val = -float(np.real(defn.loglik(prob, b, X=X))) + lam * np.sum(uv)
        return val, np.concatenate([-g + lam, g + lam])
    res = scipy.optimize.minimize(f, np.zeros(2 * J), jac=True, method="L-BFGS-B",
                                  bounds=[(0, None)] * (2 * J),
                                  options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 5000})
    b_ref = res.x[:J] - res.x[J:]
    assert np.max(np.abs(b_ref - beta)) < 1e-5
    # support agrees away from the KKT boundary
    for j in range(J):
        if abs(b_ref[j]) > 1e-4:
            assert beta[j] != 0.0


def test_classical_one_drug_sccs_estimator(oracle_lib):
    """One drug, two eras per patient with l_exposed = rho * l_unexposed: the
    conditional MLE is log(Y_exposed / (rho Y_unexposed))."""
    rng = np.random.default_rng(2024)
    N, rho = 400, 3
    l0 = rng.integers(5, 100, size=N)
    offset = np.stack([l0, rho * l0], axis=1).ravel()
    y = rng.poisson(0.02 * offset.reshape(N, 2) * np.array([1.0, 1.7]))
    y[y.sum(axis=1) == 0, 0] = 1
    count = y.ravel()
    prob = make(np.arange(0, 2 * N + 1, 2), offset, count, [np.arange(1, 2 * N, 2)])
    Y1, Y0 = y[:, 1].sum(), y[:, 0].sum()
    r = _ccd_converged(oracle_lib, prob, oracle_lib.PRIOR_NONE, 1.0)
    assert r["beta"][0] == pytest.approx(math.log(Y1 / (rho * Y0)), abs=1e-10)
    # Normal prior: root of Y1 - n rho e^b / (1 + rho e^b) - b / var
    n = count.sum()
    var = 0.05
    root = scipy.optimize.brentq(lambda b: Y1 - n * rho * math.exp(b) / (1 + rho * math.exp(b)) - b / var,
                                 -5, 5, xtol=1e-15)
    r = _ccd_converged(oracle_lib, prob, oracle_lib.PRIOR_NORMAL, var)
    assert r["beta"][0] == pytest.approx(root, abs=1e-10)


@pytest.mark.parametrize("kind,var", [(0, 1.0), (1, 0.5)])
def test_matches_poisson_glm_with_patient_fixed_effects(oracle_lib, kind, var):
    """Conditioning on n_i equals profiling out patient intercepts: a Poisson
    GLM with one free intercept per patient and offset log l gives the same
    beta (SciPy optimiser on the unconditional likelihood)."""
    prob = small(17, n_patients=120, n_cols=4, p=0.25)
    X = defn.dense_x(prob)
    pid = defn.patient_of_row(prob)
    y = prob.count.astype(float)
    logl = np.log(prob.offset.astype(float))
    N, J = prob.n_patients, prob.n_cols

    def f(th):
        phi, b = th[:N], th[N:]
        eta = phi[pid] + X @ b + logl
        mu = np.exp(eta)
        val = -np.sum(y * eta - mu)
        r = y - mu
        gphi = -np.bincount(pid, weights=r, minlength=N)
        gb = -(X.T @ r)
        if kind == 1:
            val += np.sum(b ** 2) / (2 * var)
            gb = gb + b / var
        return val, np.concatenate([gphi, gb])
    res = scipy.optimize.minimize(f, np.zeros(N + J), jac=True, method="L-BFGS-B",
                                  options={"ftol": 1e-16, "gtol": 1e-11, "maxiter": 20000, "maxcor": 50})
    b_glm = res.x[N:]
    r = _ccd_converged(oracle_lib, prob, kind, var)
    assert np.max(np.abs(r["beta"] - b_glm)) < 2e-5


# ---------------------------------------------------------------- invariances

def _fit(oracle_lib, prob, kind=1, var=0.5):
    return _ccd_converged(oracle_lib, prob, kind, var)["beta"]


def _rebuild(prob, patient_order=None, era_perm_seed=None, scale_patient=None,
             extra_patients=0, extra_single=0):
    """Rebuild a problem with reordered patients/eras, a scaled patient, or
    extra patients that carry no information."""
    X = defn.dense_x(prob)
    pat = []
    order = range(prob.n_patients) if patient_order is None else patient_order
    rng = np.random.default_rng(era_perm_seed) if era_perm_seed is not None else None
    for i in order:
        lo, hi = prob.patient_ptr[i], prob.patient_ptr[i + 1]
        rows = np.arange(lo, hi)
        if rng is not None:
            rows = rng.permutation(rows)
        l = prob.offset[rows].astype(np.int64)
        if scale_patient is not None and i == scale_patient[0]:
            l = l * scale_patient[1]
        pat.append((l, prob.count[rows], X[rows]))
    zrng = np.random.default_rng(5)
    for _ in range(extra_patients):   # n_i = 0 patients
        k = int(zrng.integers(1, 5))
        pat.append((zrng.integers(1, 365, size=k), np.zeros(k, np.int64),
                    (zrng.random((k, prob.n_cols)) < 0.3).astype(float)))
    for _ in range(extra_single):     # one-era patients with events
        pat.append((zrng.integers(1, 365, size=1), np.array([2]),
                    (zrng.random((1, prob.n_cols)) < 0.5).astype(float)))
    ptr = np.zeros(len(pat) + 1, np.int64)
    ptr[1:] = np.cumsum([len(p[0]) for p in pat])
    offset = np.concatenate([p[0] for p in pat])
    count = np.concatenate([p[1] for p in pat])
    Xn = np.concatenate([p[2] for p in pat])
    cols = [np.flatnonzero(Xn[:, j]) for j in range(prob.n_cols)]
    return make(ptr, offset, count, cols)


def test_invariances(oracle_lib):
    prob = small(21, n_patients=200, n_cols=5, p=0.2)
    base = _fit(oracle_lib, prob)
    perm = np.random.default_rng(1).permutation(prob.n_patients)
    for variant in (_rebuild(prob, patient_order=perm),
                    _rebuild(prob, era_perm_seed=4),
                    _rebuild(prob, scale_patient=(3, 7)),
                    _rebuild(prob, extra_patients=25),
                    _rebuild(prob, extra_single=25)):
        assert np.max(np.abs(_fit(oracle_lib, variant) - base)) < 1e-9


def test_merging_identical_eras_is_invariant(oracle_lib):
    # patient 0 has eras 0 and 1 with the same exposure (drug 0 only)
    ptr = [0, 3, 6, 8]
    offset = [10, 15, 40, 20, 30, 25, 50, 60]
    count = [1, 0, 1, 2, 0, 1, 1, 1]
    cols = [[0, 1, 3, 6], [2, 3, 4, 7]]
    merged = make([0, 2, 5, 7], [25, 40, 20, 30, 25, 50, 60], [1, 1, 2, 0, 1, 1, 1],
                  [[0, 2, 5], [1, 2, 3, 6]])
    a = _fit(oracle_lib, make(ptr, offset, count, cols))
    b = _fit(oracle_lib, merged)
    assert np.max(np.abs(a - b)) < 1e-10


def test_duplicate_column_splits_equally_under_normal(oracle_lib):
    prob = small(23, n_patients=200, n_cols=3, p=0.25)
    cols = [prob.column(j) for j in range(prob.n_cols)] + [prob.column(1)]
    dup = make(prob.patient_ptr, prob.offset, prob.count, cols)
    # the antisymmetric direction is curved only by the prior, so CCD needs
    # many cycles there: run a fixed number instead of a log-posterior test
    b = oracle_lib.ccd(dup, 1, 0.5, 3000)["beta"]
    assert abs(b[1] - b[3]) < 1e-10


def test_rel_logpost_and_dxbeta_criteria(oracle_lib):
    prob = synth.tiny()
    r1 = oracle_lib.ccd(prob, 1, 1.0, 500, oracle_lib.CRIT_REL_LOGPOST, 1e-8)
    assert r1["converged"] and r1["sweeps"] < 500
    lp = r1["logpost_trace"]
    assert lp[-1] >= lp[0]
    r2 = oracle_lib.ccd(prob, 1, 1.0, 500, oracle_lib.CRIT_ABS_DXBETA, 5e-4)
    assert r2["converged"]
    r3 = oracle_lib.ccd(prob, 1, 1.0, 7, oracle_lib.CRIT_FIXED, 0.0)
    assert r3["sweeps"] == 7 and not r3["converged"]
    # warm start from a finished fit does not move (up to the tolerance)
    r4 = oracle_lib.ccd(prob, 1, 1.0, 1, beta0=r1["beta"], trust0=r1["trust"])
    assert np.max(np.abs(r4["beta"] - r1["beta"])) < 1e-3


def test_golden_second_visits_follow_the_sequential_order(oracle_lib):
    """Algorithm 1 visits coordinates one after the other: coordinate 1 sees
    the weights that coordinate 0's step left behind, and sweep 2's first
    visit sees both steps (hand-derived closed forms in exp(6/13))."""
    with open(os.path.join(HERE, "golden", "two_patient.json")) as f:
        fx = json.load(f)
    P = fx["problem"]
    cols = [P["row_idx"][P["col_ptr"][j]:P["col_ptr"][j + 1]] for j in range(2)]
    prob = make(P["patient_ptr"], P["offset"], P["count"], cols)
    sv = fx["second_visits_normal_var1"]
    env = {"exp": math.exp, "log": math.log, "max": max, "min": min}
    for k in ("E", "g1", "h1", "dbeta1", "trust1", "F", "logpost_sweep1", "W0_sweep2", "g0_sweep2",
              "h0_sweep2", "dbeta0_sweep2"):
        env[k] = eval(sv[k], {"__builtins__": {}}, env)
    r = oracle_lib.ccd(prob, oracle_lib.PRIOR_NORMAL, 1.0, 2, want_trace=True)
    tr = r["trace"]
    assert tr[0, 1, 0] == pytest.approx(env["g1"], rel=1e-14)
    assert tr[0, 1, 1] == pytest.approx(env["h1"], rel=1e-14)
    assert tr[0, 1, 2] == pytest.approx(env["dbeta1"], rel=1e-14)
    assert r["logpost_trace"][0] == pytest.approx(env["logpost_sweep1"], rel=1e-14)
    assert tr[1, 0, 0] == pytest.approx(env["g0_sweep2"], rel=1e-13)
    assert tr[1, 0, 1] == pytest.approx(env["h0_sweep2"], rel=1e-13)
    assert tr[1, 0, 2] == pytest.approx(env["dbeta0_sweep2"], rel=1e-13)
    r1 = oracle_lib.ccd(prob, oracle_lib.PRIOR_NORMAL, 1.0, 1)
    assert r1["trust"][1] == pytest.approx(env["trust1"], rel=1e-14)
    assert r1["beta"][1] == pytest.approx(env["dbeta1"], rel=1e-14)


# ---------------------------------------------------------------- log prior

def test_log_prior_hand_values(oracle_lib):
    """Eq. 3 with constants dropped: Normal -sum b^2 / (2 var); Laplace
    -lambda sum |b| with lambda = sqrt(2 / var)."""
    b = [1.0, -2.0, 0.0]
    assert oracle_lib.log_prior(oracle_lib.PRIOR_NORMAL, 0.5, b) == pytest.approx(-5.0, abs=1e-15)
    assert oracle_lib.log_prior(oracle_lib.PRIOR_NORMAL, 2.0, b) == pytest.approx(-1.25, abs=1e-15)
    assert oracle_lib.log_prior(oracle_lib.PRIOR_LAPLACE, 2.0, b) == pytest.approx(-3.0, abs=1e-15)    # lambda 1
    assert oracle_lib.log_prior(oracle_lib.PRIOR_LAPLACE, 0.5, b) == pytest.approx(-6.0, abs=1e-15)    # lambda 2
    assert oracle_lib.log_prior(oracle_lib.PRIOR_LAPLACE, 0.08, b) == pytest.approx(-15.0, abs=1e-13)  # lambda 5
    assert oracle_lib.log_prior(oracle_lib.PRIOR_NONE, 1.0, b) == 0.0
    rng = np.random.default_rng(8)
    for _ in range(5):
        beta = rng.normal(size=40) * (rng.random(40) < 0.5)
        for kind in (0, 1, 2):
            var = float(rng.uniform(0.01, 5.0))
            assert oracle_lib.log_prior(kind, var, beta) == pytest.approx(defn.log_prior(kind, var, beta),
                                                                        rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("kind,var", [(1, 0.5), (1, 2.0), (2, 2.0), (2, 0.5), (2, 0.05)])
def test_log_prior_density_has_the_stated_variance(oracle_lib, kind, var):
    """The prior's second argument is its variance (Laplace(0, var) included):
    exp(log p) of one coordinate, normalised by numerical integration, has
    mean 0 and variance var.  A Laplace rate of 1/var or 1/sqrt(var) fails."""
    import scipy.integrate as si
    lp0 = oracle_lib.log_prior(kind, var, [0.0])

    def dens(b, power):
        return b ** power * math.exp(oracle_lib.log_prior(kind, var, [b]) - lp0)
    pieces = [(-math.inf, 0.0), (0.0, math.inf)]   # the Laplace kink sits at 0
    Z = sum(si.quad(dens, lo, hi, args=(0,), epsabs=0, epsrel=1e-12)[0] for lo, hi in pieces)
    M1 = sum(si.quad(dens, lo, hi, args=(1,), epsabs=0, epsrel=1e-12)[0] for lo, hi in pieces)
    M2 = sum(si.quad(dens, lo, hi, args=(2,), epsabs=0, epsrel=1e-12)[0] for lo, hi in pieces)
    assert abs(M1 / Z) < 1e-10
    assert M2 / Z == pytest.approx(var, rel=1e-9)


# ---------------------------------------------------------------- stopping rules

def _sweep_betas(oracle_lib, prob, kind, var, n):
    """beta after sweeps 0..n, rebuilt from the oracle's per-visit steps."""
    r = oracle_lib.ccd(prob, kind, var, n, want_trace=True)
    steps = r["trace"][:, :, 2]
    betas = np.zeros((n + 1, prob.n_cols))
    for t in range(n):
        betas[t + 1] = betas[t] + steps[t]
    return betas, r


@pytest.mark.parametrize("kind,var", [(1, 1.0), (2, 0.5)])
def test_rel_logpost_rule_fires_at_the_first_qualifying_sweep(oracle_lib, kind, var):
    """Section 2.2 reading R6: stop after sweep t, the first with
    |P_t - P_{t-1}| < tol |P_t|, P_0 at the start point; P from Eq. 2 and
    Eq. 3 evaluated independently (defn) on the oracle's per-sweep beta."""
    prob = synth.tiny(n_patients=300, n_cols=8, seed=5)
    n = 12
    betas, r = _sweep_betas(oracle_lib, prob, kind, var, n)
    X = defn.dense_x(prob)
    P = np.array([float(np.real(defn.loglik(prob, b, X=X))) + defn.log_prior(kind, var, b) for b in betas])
    # the oracle's per-sweep log posterior is Eq. 2 + Eq. 3 at each sweep's beta
    assert np.allclose(r["logpost_trace"], P[1:], rtol=1e-12, atol=0)
    ratio = np.abs(np.diff(P)) / np.abs(P[1:])       # ratio[t-1] belongs to sweep t
    # thresholds half-way (geometrically) between consecutive ratios: the rule
    # must fire exactly at the sweep whose ratio first drops below
    fired = 0
    for t in range(2, 9):
        # sweeps whose change is above rounding level, well below the earlier ones
        if not (1e-14 < ratio[t - 1] < ratio[: t - 1].min() / 4):
            continue
        tol = math.sqrt(ratio[t - 1] * ratio[: t - 1].min())
        rr = oracle_lib.ccd(prob, kind, var, 50, oracle_lib.CRIT_REL_LOGPOST, tol)
        assert rr["converged"] and rr["sweeps"] == t, (t, tol, ratio[:t])
        assert np.array_equal(rr["beta"], betas[t])
        fired += 1
    assert fired >= 2


@pytest.mark.parametrize("kind,var", [(1, 1.0), (2, 0.5)])
def test_abs_dxbeta_rule_fires_at_the_first_qualifying_sweep(oracle_lib, kind, var):
    """Section 2.2: stop after the first sweep whose sum over eras of
    |(X beta)_t - (X beta)_{t-1}| falls below eps, with X beta formed from
    the dense design (defn) and the oracle's per-sweep beta."""
    prob = synth.tiny(n_patients=300, n_cols=8, seed=6)
    n = 12
    betas, _ = _sweep_betas(oracle_lib, prob, kind, var, n)
    X = defn.dense_x(prob)
    S = np.array([np.sum(np.abs(X @ (betas[t] - betas[t - 1]))) for t in range(1, n + 1)])
    fired = 0
    for t in range(2, 9):
        if not (1e-12 < S[t - 1] < S[: t - 1].min() / 4):
            continue
        eps = math.sqrt(S[t - 1] * S[: t - 1].min())
        rr = oracle_lib.ccd(prob, kind, var, 50, oracle_lib.CRIT_ABS_DXBETA, eps)
        assert rr["converged"] and rr["sweeps"] == t, (t, eps, S[:t])
        assert np.array_equal(rr["beta"], betas[t])
        fired += 1
    assert fired >= 2
    # the paper's own threshold, 5e-4 absolute
    t_paper = int(np.argmax(S < 5e-4)) + 1
    assert S[t_paper - 1] < 5e-4 <= S[: t_paper - 1].min()
    rr = oracle_lib.ccd(prob, kind, var, 50, oracle_lib.CRIT_ABS_DXBETA, 5e-4)
    assert rr["sweeps"] == t_paper


def test_patient_with_zero_total_length_adds_nothing(oracle_lib):
    """A patient whose eras all have length 0 has den_i = 0 and (validation
    requires y_k = 0 where l_k = 0) n_i = 0: Eq. 2 gives it no term, so adding
    it to a column leaves every fit unchanged and finite."""
    prob = small(31, n_patients=120, n_cols=4, p=0.25)
    base = _fit(oracle_lib, prob)
    X = defn.dense_x(prob)
    ptr = np.concatenate([prob.patient_ptr, [prob.n_rows + 3]]).astype(np.int64)
    offset = np.concatenate([prob.offset, [0, 0, 0]])
    count = np.concatenate([prob.count, [0, 0, 0]])
    Xn = np.vstack([X, np.ones((3, prob.n_cols))])
    cols = [np.flatnonzero(Xn[:, j]) for j in range(prob.n_cols)]
    p2 = make(ptr, offset, count, cols)
    for kind, var in ((1, 0.5), (2, 2.0), (0, 1.0)):
        a = _ccd_converged(oracle_lib, prob, kind, var)["beta"]
        b = _ccd_converged(oracle_lib, p2, kind, var)["beta"]
        assert np.all(np.isfinite(b))
        assert np.max(np.abs(a - b)) < 1e-12
    for j in range(prob.n_cols):
        g, h = oracle_lib.grad_hess(p2, base, j)
        g0, h0 = oracle_lib.grad_hess(prob, base, j)
        assert g == pytest.approx(g0, rel=1e-13, abs=1e-13) and h == pytest.approx(h0, rel=1e-13)


# ---------------------------------------------------------------- bootstrap summary (Section 2.5)

def test_bootstrap_quantiles_match_numpy_and_hand_values(oracle_lib):
    """The percentile rule is linear interpolation between order statistics;
    numpy's default quantile is that rule, and small cases are done by hand."""
    rng = np.random.default_rng(11)
    B = rng.normal(size=(37, 9))
    B[rng.random(B.shape) < 0.3] = 0.0          # exact zeros, as under the Laplace prior
    B[:, 4] = 0.0                                # a coefficient that never enters
    B[:5, 5] = 2.5                               # ties
    for level in (0.95, 0.9, 0.5):
        lo, hi, p = oracle_lib.bootstrap_summary(B, level)
        assert np.allclose(lo, np.quantile(B, 0.5 * (1 - level), axis=0), rtol=0, atol=1e-15)
        assert np.allclose(hi, np.quantile(B, 0.5 * (1 + level), axis=0), rtol=0, atol=1e-15)
        assert np.array_equal(p, (B != 0).mean(axis=0))
    # R = 5, values 1..5 (shuffled): the 25 % / 75 % quantiles sit on order statistics 2 and 4
    lo, hi, p = oracle_lib.bootstrap_summary(np.array([[3.0], [1.0], [5.0], [2.0], [4.0]]), 0.5)
    assert (lo[0], hi[0], p[0]) == (2.0, 4.0, 1.0)
    # R = 4, values 0, 0, 1, 3 at level 0.95: positions 0.075 and 2.925
    lo, hi, p = oracle_lib.bootstrap_summary(np.array([[0.0], [3.0], [0.0], [1.0]]), 0.95)
    assert lo[0] == 0.0 and abs(hi[0] - (1.0 + 0.925 * 2.0)) < 1e-15 and p[0] == 0.5
    # a single replicate: both bounds are its value
    lo, hi, p = oracle_lib.bootstrap_summary(np.array([[-0.7, 0.0]]), 0.95)
    assert lo.tolist() == [-0.7, 0.0] and hi.tolist() == [-0.7, 0.0] and p.tolist() == [1.0, 0.0]


def test_bootstrap_weights_are_resample_counts():
    """Replicate weights are multiplicities of N draws with replacement: each
    row sums to N, and across many replicates each patient's mean is 1."""
    W = synth.bootstrap_weights(400, 300, seed=2)
    assert W.shape == (300, 400) and (W >= 0).all()
    assert (W.sum(axis=1) == 400).all()
    assert abs(W.mean() - 1.0) < 1e-12
    assert abs(W.mean(axis=0).mean() - 1.0) < 1e-12 and W.mean(axis=0).std() < 0.15


def test_bootstrap_replicate_with_unit_weights_is_the_plain_fit(oracle_lib):
    """A replicate that draws every patient once is the original fit, and one
    that draws a patient twice equals the fit on the data with that patient
    duplicated (the weight multiplies the patient's terms of Eq. 2)."""
    prob = synth.tiny(n_patients=120, n_cols=6, seed=9)
    ones = np.ones((1, prob.n_patients), dtype=np.int32)
    r = oracle_lib.bootstrap(prob, oracle_lib.PRIOR_NORMAL, 1.0, ones, 12)
    ref = oracle_lib.ccd(prob, oracle_lib.PRIOR_NORMAL, 1.0, 12)["beta"]
    assert np.array_equal(r["beta"][0], ref)
    w = ones.copy()
    w[0, 7] = 2
    w[0, 8] = 0
    rw = oracle_lib.bootstrap(prob, oracle_lib.PRIOR_NORMAL, 1.0, w, 12)
    dup = _resample(prob, [i for i in range(prob.n_patients) if i != 8] + [7])
    rd = oracle_lib.ccd(dup, oracle_lib.PRIOR_NORMAL, 1.0, 12)["beta"]
    assert np.max(np.abs(rw["beta"][0] - rd)) <= 1e-12 * max(1.0, np.max(np.abs(rd)))


def _resample(prob, patients):
    """The problem made of the listed patients (repeats allowed), in order."""
    X = defn.dense_x(prob)
    rows = [np.arange(prob.patient_ptr[i], prob.patient_ptr[i + 1]) for i in patients]
    ptr = np.zeros(len(rows) + 1, np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    allr = np.concatenate(rows)
    Xn = X[allr]
    return make(ptr, prob.offset[allr], prob.count[allr], [np.flatnonzero(Xn[:, j]) for j in range(prob.n_cols)])


# ---------------------------------------------------------------- non-binary covariates (Section 4)

def _valued_small(seed=0, n_patients=250):
    return synth.valued(n_patients=n_patients, n_drugs=5, n_dose=2, n_dense=2, seed=seed)


@pytest.mark.parametrize("seed", [0, 1])
def test_valued_grad_hess_match_complex_step(oracle_lib, seed):
    """With covariate values, g_j and h_j (the general form of Eqs. 7-9:
    -sum omega n (M[w x^2]/den - (M[w x]/den)^2)) against derivatives of
    Eq. 2 taken by the complex step, for drug, dose and dense columns."""
    prob = _valued_small(seed)
    X = defn.dense_x(prob)
    rng = np.random.default_rng(seed)
    for beta in (np.zeros(prob.n_cols), rng.normal(0, 0.3, prob.n_cols)):
        for j in range(prob.n_cols):
            g, h = oracle_lib.grad_hess(prob, beta, j)
            gc = defn.grad_cs(prob, beta, j, X=X)
            hf = defn.hess_fd(prob, beta, j, X=X)
            assert abs(g - gc) <= 1e-11 * max(1.0, abs(gc))
            assert abs(h - hf) <= 1e-8 * abs(hf)
            assert h <= 0.0
    assert oracle_lib.loglik(prob, beta) == pytest.approx(float(np.real(defn.loglik(prob, beta, X=X))), rel=1e-13)


@pytest.mark.parametrize("kind,var", [(1, 1.0), (0, 1.0)])
def test_valued_ccd_reaches_full_newton_optimum(oracle_lib, kind, var):
    """Multivariate Newton with the textbook Hessian -sum n_i Cov_i(x) on
    real-valued x, against CCD run to convergence."""
    prob = _valued_small(2, n_patients=400)
    X = defn.dense_x(prob)
    b = np.zeros(prob.n_cols)
    for _ in range(80):
        g, H = defn.grad_hess_full(prob, b, X=X)
        if kind == 1:
            g = g - b / var
            H = H - np.eye(len(b)) / var
        step = np.linalg.solve(H, -g)
        b = b + step
        if np.max(np.abs(step)) < 1e-15:
            break
    r = _ccd_converged(oracle_lib, prob, kind, var)
    assert r["converged"]
    assert np.max(np.abs(r["beta"] - b)) < 1e-8


def test_valued_matches_poisson_glm_with_patient_fixed_effects(oracle_lib):
    """Profiling out patient intercepts of a Poisson GLM with real-valued
    covariates gives the conditional MLE."""
    prob = _valued_small(3, n_patients=120)
    X = defn.dense_x(prob)
    pid = defn.patient_of_row(prob)
    y = prob.count.astype(float)
    logl = np.log(prob.offset.astype(float))
    N, J = prob.n_patients, prob.n_cols

    def f(th):
        phi, b = th[:N], th[N:]
        eta = phi[pid] + X @ b + logl
        mu = np.exp(eta)
        r = y - mu
        return -np.sum(y * eta - mu), np.concatenate([-np.bincount(pid, weights=r, minlength=N), -(X.T @ r)])
    res = scipy.optimize.minimize(f, np.zeros(N + J), jac=True, method="L-BFGS-B",
                                  options={"ftol": 1e-16, "gtol": 1e-11, "maxiter": 20000, "maxcor": 50})
    r = _ccd_converged(oracle_lib, prob, 0, 1.0)
    assert np.max(np.abs(r["beta"] - res.x[N:])) < 2e-5


def test_valued_scaling_a_column_rescales_its_coefficient(oracle_lib):
    """Without a prior, multiplying column j's values by c divides the MLE's
    beta_j by c and leaves the others."""
    prob = _valued_small(4, n_patients=300)
    # a fixed number of cycles: the log posterior is flat to 1e-15 well
    # before beta is settled to 1e-9
    base = oracle_lib.ccd(prob, 0, 1.0, 400)["beta"]
    J = prob.n_cols
    for j, c in ((J - 2, 2.5), (J - 4, 0.4)):
        v = prob.value.copy()
        v[prob.col_ptr[j]:prob.col_ptr[j + 1]] *= c
        scaled = dataclasses.replace(prob, value=v)
        b = oracle_lib.ccd(scaled, 0, 1.0, 400)["beta"]
        expect = base.copy()
        expect[j] /= c
        assert np.max(np.abs(b - expect)) < 1e-9


def test_valued_all_ones_reproduces_the_binary_path(oracle_lib):
    """Values of 1 at every stored entry are the binary model: same
    trajectory as the binary problem up to rounding (the valued form
    evaluates B - A^2 where the binary one evaluates W(1 - W))."""
    prob = small(5, n_patients=300, n_cols=6, p=0.2)
    ones = dataclasses.replace(prob, value=np.ones(prob.nnz))
    for kind, var in ((1, 0.5), (2, 0.3)):
        a = oracle_lib.ccd(prob, kind, var, 12)
        b = oracle_lib.ccd(ones, kind, var, 12)
        assert np.max(np.abs(a["beta"] - b["beta"])) <= 1e-12 * max(1.0, np.max(np.abs(a["beta"])))
        assert np.array_equal(a["beta"] == 0.0, b["beta"] == 0.0)


def test_valued_generator_shapes():
    """Dense columns cover every era and vary within patients; dose values
    are positive; drugs are binary."""
    prob = synth.valued(n_patients=500, n_drugs=6, n_dose=3, n_dense=2, seed=1)
    c = np.diff(prob.col_ptr)
    assert (c[-2:] == prob.n_rows).all()
    d0 = prob.col_ptr[6]
    assert np.all(prob.value[:d0] == 1.0)
    assert np.all(prob.value[d0:prob.col_ptr[9]] > 0.0) and np.any(prob.value[d0:prob.col_ptr[9]] != 1.0)
    age = prob.value[prob.col_ptr[-3]:prob.col_ptr[-2]]
    pid = defn.patient_of_row(prob)
    within = np.bincount(pid, weights=age ** 2) / np.diff(prob.patient_ptr) - \
        (np.bincount(pid, weights=age) / np.diff(prob.patient_ptr)) ** 2
    assert np.mean(within > 1e-12) > 0.5


# ---------------------------------------------------------------- prior-variance search (Section 2.5)

def test_cv_search_finds_the_grid_maximum(oracle_lib):
    """The bracketing + golden-section search ends within its tolerance of
    the maximum that a brute-force scan of the predictive log-likelihood on a
    fine log10 grid finds; its bracket holds that maximum; each reported
    value equals a direct evaluation."""
    prob = synth.zipf_problem("zipf_small", 1500, 12, 0.15, seed_path=(8, 7))
    folds = synth.cv_folds(prob.n_patients, 4, seed=3)
    for kind in (1, 2):
        r = oracle_lib.cv_search(prob, folds, 4, kind, 1e-2, 10.0, 0.05, 40, 400, tol=1e-12)
        assert r["bracketed"]
        grid = np.linspace(-3.0, 2.0, 101)
        vals = [oracle_lib.cv_predictive_loglik(prob, folds, 4, kind, 10.0 ** t, 400, tol=1e-12)[0] for t in grid]
        t_best = grid[int(np.argmax(vals))]
        t_found = np.log10(r["variance"][r["best"]])
        assert abs(t_found - t_best) <= 0.05 + 0.05        # search tolerance + grid spacing
        assert r["pred_loglik"][r["best"]] >= max(vals) - 1e-6 * abs(max(vals))
        k = len(r["variance"]) // 2
        direct = oracle_lib.cv_predictive_loglik(prob, folds, 4, kind, r["variance"][k], 400, tol=1e-12)[0]
        assert abs(direct - r["pred_loglik"][k]) <= 1e-8 * abs(direct)


def test_cv_predictive_loglik_is_the_heldout_sum(oracle_lib):
    """Definition check: with two folds the predictive log-likelihood is
    L(beta_A; fold B) + L(beta_B; fold A), each beta fitted on the other
    fold alone."""
    prob = small(31, n_patients=200, n_cols=4, p=0.25)
    folds = (np.arange(prob.n_patients) % 2).astype(np.int32)
    pl, B = oracle_lib.cv_predictive_loglik(prob, folds, 2, 1, 0.5, 200, tol=1e-13)
    bA = oracle_lib.ccd(prob, 1, 0.5, 200, oracle_lib.CRIT_REL_LOGPOST, 1e-13, weight=(folds == 1).astype(np.int32))["beta"]
    bB = oracle_lib.ccd(prob, 1, 0.5, 200, oracle_lib.CRIT_REL_LOGPOST, 1e-13, weight=(folds == 0).astype(np.int32))["beta"]
    expect = float(np.real(defn.loglik(prob, bA, weight=(folds == 0)))) + \
        float(np.real(defn.loglik(prob, bB, weight=(folds == 1))))
    assert abs(pl - expect) <= 1e-10 * abs(expect)


# ---------------------------------------------------------------- grouped prior (Section 4)

def _class_precision(class_of, var, class_var):
    """The prior precision matrix: the inverse of var I + class_var 1 1' within
    each class, inverted numerically (not by the closed form the oracle uses)."""
    J = len(class_of)
    Q = np.zeros((J, J))
    for c in np.unique(class_of):
        idx = np.flatnonzero(class_of == c)
        S = var * np.eye(len(idx)) + class_var * np.ones((len(idx), len(idx)))
        Q[np.ix_(idx, idx)] = np.linalg.inv(S)
    return Q


def test_grouped_prior_map_matches_full_newton(oracle_lib):
    """MAP under beta ~ N(0, blockdiag(var I + class_var 1 1')): full
    multivariate Newton with the numerically inverted prior covariance
    against CCD under the grouped prior; stationarity g = Q beta."""
    prob = small(41, n_patients=400, n_cols=8, p=0.2)
    class_of = np.array([0, 0, 1, 1, 1, 2, 0, 2], dtype=np.int32)
    var, cvar = 0.3, 0.8
    Q = _class_precision(class_of, var, cvar)
    X = defn.dense_x(prob)
    b = np.zeros(prob.n_cols)
    for _ in range(60):
        g, H = defn.grad_hess_full(prob, b, X=X)
        step = np.linalg.solve(H - Q, -(g - Q @ b))
        b = b + step
        if np.max(np.abs(step)) < 1e-15:
            break
    r = oracle_lib.ccd_grouped(prob, var, class_of, cvar, 3000, oracle_lib.CRIT_FIXED)
    assert np.max(np.abs(r["beta"] - b)) < 1e-9
    g, _ = defn.grad_hess_full(prob, r["beta"], X=X)
    assert np.max(np.abs(g - Q @ r["beta"])) < 1e-8


def test_grouped_log_prior_against_the_gaussian_density(oracle_lib):
    """Differences of the log prior equal differences of -b'Qb/2 with Q the
    numerically inverted covariance (the dropped constant cancels)."""
    class_of = np.array([0, 1, 0, 2, 1, 0], dtype=np.int32)
    var, cvar = 0.5, 2.0
    Q = _class_precision(class_of, var, cvar)
    rng = np.random.default_rng(4)
    for _ in range(5):
        b1, b2 = rng.normal(size=6), rng.normal(size=6)
        d_or = oracle_lib.log_prior_grouped(var, class_of, cvar, b1) - oracle_lib.log_prior_grouped(var, class_of, cvar, b2)
        d_ref = -0.5 * (b1 @ Q @ b1) + 0.5 * (b2 @ Q @ b2)
        assert abs(d_or - d_ref) < 1e-12 * max(1.0, abs(d_ref))


def test_grouped_prior_special_cases(oracle_lib):
    """class_var = 0 is the independent Normal prior (the same steps, bit for
    bit); a class of one drug is a Normal prior with variance
    var + class_var."""
    prob = small(43, n_patients=300, n_cols=6, p=0.2)
    a = oracle_lib.ccd(prob, 1, 0.4, 15)
    b = oracle_lib.ccd_grouped(prob, 0.4, np.array([0, 0, 1, 1, 1, 0]), 0.0, 15)
    assert np.array_equal(a["beta"], b["beta"]) and np.array_equal(a["trust"], b["trust"])
    singles = np.arange(prob.n_cols, dtype=np.int32)
    c = oracle_lib.ccd_grouped(prob, 0.4, singles, 0.6, 400)
    d = oracle_lib.ccd(prob, 1, 1.0, 400)
    assert np.max(np.abs(c["beta"] - d["beta"])) < 1e-12
    # hand value of one step: g = 2, h = -5, var = 0.5, kappa = 0.25, beta = 0.2, S = 1
    dv = oracle_lib.newton_step_grouped(0.5, 0.25, 0.2, 1.0, 2.0, -5.0)
    assert dv == pytest.approx(-(2.0 - (0.2 - 0.25) / 0.5) / (-5.0 - 0.75 / 0.5), rel=1e-15)
