"""GPU parity for non-binary and dense covariates (the general form of
Eqs. 7-9 with stored values x_kj) against the oracle.

Problems from synth.valued: binary drugs, sparse dose columns (lognormal
values) and dense columns on every era (an age-like and a seasonal
covariate, both varying within patients).  FP64 trajectories must match the
oracle's to 1e-9 relative (same exact zeros under the Laplace prior); the
mixed form to 1e-6.
"""
import numpy as np
import pytest

import oracle
from paper_1208_0945_amd import synth

pytestmark = pytest.mark.gpu
FP64_TOL = 1e-9
MIXED_TOL = 1e-6


@pytest.fixture(scope="module")
def sccs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_0945_amd import sccs as s
    s.lib()
    return s


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def prob():
    return synth.valued(n_patients=6000, n_drugs=40, n_dose=6, n_dense=2, seed=0)


@pytest.mark.parametrize("kind,var,sweeps", [(1, 1.0, 6), (2, 0.5, 8), (0, 1.0, 5)])
@pytest.mark.parametrize("n_workgroups,max_group", [(0, 0), (37, 1), (64, 2)])
def test_valued_trajectory_matches_oracle(sccs, prob, kind, var, sweeps, n_workgroups, max_group):
    ref = oracle.ccd(prob, kind, var, sweeps)
    with sccs.Handle(prob, n_workgroups=n_workgroups, max_group=max_group) as h:
        h.set_prior(kind, var)
        h.sweep(sweeps)
        beta, trust = h.get_beta()
    err = rel_inf(beta, ref["beta"])
    print(f"prior {kind}: rel error {err:.2e}")
    assert err <= FP64_TOL
    assert np.array_equal(beta == 0.0, ref["beta"] == 0.0)
    assert np.max(np.abs(trust - ref["trust"])) <= 1e-9 * np.max(ref["trust"])


def test_valued_grad_hess_at_warm_start(sccs, prob):
    """g_j, h_j of every column at a warm start (set_beta: exact refresh of
    exp(X beta) with the values) against the oracle."""
    beta0 = np.random.default_rng(3).normal(0.0, 0.2, prob.n_cols)
    with sccs.Handle(prob) as h:
        h.set_prior(sccs.PRIOR_NORMAL, 1.0)
        h.set_beta(beta0)
        for j in range(prob.n_cols):
            g, hh = h.grad_hess(j)
            go, ho = oracle.grad_hess(prob, beta0, j)
            scale = max(1.0, abs(go), float(np.abs(prob.value[prob.col_ptr[j]:prob.col_ptr[j + 1]]).sum()))
            assert abs(g - go) <= 1e-11 * scale, (j, g, go)
            assert abs(hh - ho) <= 1e-10 * abs(ho), (j, hh, ho)


def test_valued_objective_and_fit_to_convergence(sccs, prob):
    ref = oracle.ccd(prob, oracle.PRIOR_NORMAL, 1.0, 200, oracle.CRIT_REL_LOGPOST, 1e-12)
    assert ref["converged"]
    with sccs.Handle(prob) as h:
        h.set_prior(sccs.PRIOR_NORMAL, 1.0)
        r = h.fit(sccs.CRIT_REL_LOGPOST, 200, 1e-12)
        beta, _ = h.get_beta()
        L, P = h.objective()
    assert r["converged"] and r["sweeps"] == ref["sweeps"]
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL
    assert abs(L - ref["loglik"]) <= 1e-12 * abs(ref["loglik"])
    assert abs(P - ref["logpost"]) <= 1e-12 * abs(ref["logpost"])


def test_valued_abs_dxbeta_rule(sccs, prob):
    """Sum over eras of |change of x_k'beta| (with the values) < tol."""
    ref = oracle.ccd(prob, oracle.PRIOR_LAPLACE, 0.5, 100, oracle.CRIT_ABS_DXBETA, 5e-4)
    assert ref["converged"]
    with sccs.Handle(prob) as h:
        h.set_prior(sccs.PRIOR_LAPLACE, 0.5)
        r = h.fit(sccs.CRIT_ABS_DXBETA, 100, 5e-4)
        beta, _ = h.get_beta()
    assert r["converged"] and r["sweeps"] == ref["sweeps"]
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL


def test_valued_mixed_precision(sccs, prob):
    ref = oracle.ccd(prob, oracle.PRIOR_NORMAL, 1.0, 6)["beta"]
    for refresh in (-1, 0, 3):
        with sccs.Handle(prob, precision=1, refresh_period=refresh) as h:
            h.set_prior(sccs.PRIOR_NORMAL, 1.0)
            h.sweep(6)
            beta, _ = h.get_beta()
        err = rel_inf(beta, ref)
        print(f"mixed, refresh {refresh}: rel error {err:.2e}")
        assert err <= MIXED_TOL


def test_valued_long_segments_and_dense_only(sccs):
    """Patients with more than 64 eras put whole dense-column segments past
    one wavefront (the long-tile path); a problem of dense columns alone."""
    long = synth.valued(n_patients=400, n_drugs=4, n_dose=2, n_dense=2, seed=2, era_mean=90.0)
    assert np.max(np.diff(long.patient_ptr)) > 64
    dense = synth.valued(n_patients=3000, n_drugs=0, n_dose=0, n_dense=2, seed=4)
    for p, kind, var in ((long, 1, 1.0), (long, 2, 0.5), (dense, 0, 1.0)):
        ref = oracle.ccd(p, kind, var, 7)["beta"]
        with sccs.Handle(p, n_workgroups=16) as h:
            h.set_prior(kind, var)
            h.sweep(7)
            beta, _ = h.get_beta()
        assert rel_inf(beta, ref) <= FP64_TOL
        assert np.array_equal(beta == 0.0, ref == 0.0)


def test_valued_exact_refresh_keeps_the_trajectory(sccs, prob):
    """FP64 with an exact recomputation of exp(X beta) from the values every
    2 sweeps follows the same trajectory."""
    ref = oracle.ccd(prob, oracle.PRIOR_LAPLACE, 0.5, 6)["beta"]
    with sccs.Handle(prob, refresh_period=2) as h:
        h.set_prior(sccs.PRIOR_LAPLACE, 0.5)
        h.sweep(6)
        beta, _ = h.get_beta()
    assert rel_inf(beta, ref) <= FP64_TOL


def test_batched_form_rejects_values(sccs, prob):
    spec = sccs.FitSpec(0, [(sccs.PRIOR_NORMAL, 1.0)])
    with pytest.raises(sccs.SccsError):
        sccs.Batch([prob], [spec])
