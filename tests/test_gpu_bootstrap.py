"""GPU bootstrap (sccs_bootstrap, Section 2.5) against the oracle.

Each replicate refits the MAP beta under patient multiplicities drawn by
resampling patients with replacement (synth.bootstrap_weights, shared by both
sides).  70 replicates need two launches of the batched kernel (64 fits, then
6 in the same workspace), so the re-initialisation of fits between launches
is exercised.  Per replicate, beta must match the oracle's fit with the same
weights (FP64, 1e-9 relative, same exact zeros); the share of nonzero
estimates must be equal and the percentile bounds must agree to the size of
the beta differences.
"""
import numpy as np
import pytest

import oracle
from paper_1208_0945_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sccs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_0945_amd import sccs as s
    s.lib()
    return s


@pytest.fixture(params=[0, 1], ids=["partitioned", "lockstep"])
def engine(request):
    """Engine of the batched form underneath: fits on disjoint workgroup
    ranges (0) or all fits in lockstep (1)."""
    return request.param


def _check(sccs, got, ref, tol):
    scale = max(float(np.max(np.abs(ref["beta"]))), 1e-300)
    err = float(np.max(np.abs(got["beta"] - ref["beta"]))) / scale
    print(f"max rel beta error over replicates {err:.2e}")
    assert err <= tol
    assert np.array_equal(got["beta"] == 0.0, ref["beta"] == 0.0)
    assert np.array_equal(got["p_nonzero"], ref["p_hat"])
    assert np.max(np.abs(got["lo"] - ref["lo"])) <= tol * scale
    assert np.max(np.abs(got["hi"] - ref["hi"])) <= tol * scale


@pytest.mark.parametrize("kind,var", [(2, 0.05), (1, 1.0)])
def test_bootstrap_fixed_sweeps(sccs, engine, kind, var):
    prob = synth.tiny(n_patients=1500, n_cols=20, seed=5)
    W = synth.bootstrap_weights(prob.n_patients, 70, seed=1)
    ref = oracle.bootstrap(prob, kind, var, W, 15)
    got = sccs.bootstrap(prob, kind, var, W, criterion=sccs.CRIT_FIXED, max_sweeps=15, engine=engine)
    assert (got["sweeps"] == 15).all()
    if kind == 2:
        assert 0.0 < ref["p_hat"].min() < 1.0 or 0.0 < ref["p_hat"].max() < 1.0   # some coefficients drop out
    _check(sccs, got, ref, 1e-9)


def test_bootstrap_to_convergence(sccs, engine):
    """REL_LOGPOST per replicate: the GPU runs each replicate for the oracle's
    sweep count (both stop at the first sweep whose relative change falls
    below the tolerance)."""
    prob = synth.tiny(n_patients=1500, n_cols=20, seed=5)
    W = synth.bootstrap_weights(prob.n_patients, 9, seed=4)
    ref = oracle.bootstrap(prob, 2, 0.05, W, 200, oracle.CRIT_REL_LOGPOST, 1e-10)
    got = sccs.bootstrap(prob, 2, 0.05, W, criterion=sccs.CRIT_REL_LOGPOST, max_sweeps=200, tol=1e-10,
                         engine=engine)
    assert got["converged"].all()
    assert np.array_equal(got["sweeps"], ref["sweeps"])
    _check(sccs, got, ref, 1e-9)


def test_bootstrap_mixed_precision(sccs, engine):
    prob = synth.tiny(n_patients=1500, n_cols=20, seed=5)
    W = synth.bootstrap_weights(prob.n_patients, 12, seed=6)
    ref = oracle.bootstrap(prob, 1, 1.0, W, 15)
    got = sccs.bootstrap(prob, 1, 1.0, W, criterion=sccs.CRIT_FIXED, max_sweeps=15, precision=1,
                         engine=engine)
    scale = float(np.max(np.abs(ref["beta"])))
    err = float(np.max(np.abs(got["beta"] - ref["beta"]))) / scale
    print(f"mixed: max rel beta error {err:.2e}")
    assert err <= 1e-6
    assert np.max(np.abs(got["lo"] - ref["lo"])) <= 1e-6 * scale


def test_bootstrap_argument_errors(sccs):
    prob = synth.tiny(n_patients=50, n_cols=4, seed=1)
    W = synth.bootstrap_weights(prob.n_patients, 3, seed=1)
    with pytest.raises(sccs.SccsError):
        sccs.bootstrap(prob, 2, 1.0, W, level=1.0)
    bad = W.copy()
    bad[1, 3] = -1
    with pytest.raises(sccs.SccsError):
        sccs.bootstrap(prob, 2, 1.0, bad)


def test_bootstrap_relabelled(sccs):
    """The bootstrap under the independence relabelling (partitioned engine):
    the oracle bootstraps the renumbered problem with the same multiplicities
    and its results are mapped back to the problem's numbering."""
    prob = synth.tiny(n_patients=1500, n_cols=20, seed=5)
    W = synth.bootstrap_weights(prob.n_patients, 70, seed=1)
    order = oracle.independent_order(prob, 4)
    r = oracle.bootstrap(synth.permute_columns(prob, order), 2, 0.05, W, 15)
    ref = {k: np.empty_like(r[k]) for k in ("beta", "lo", "hi", "p_hat")}
    ref["beta"][:, order] = r["beta"]
    for k in ("lo", "hi", "p_hat"):
        ref[k][order] = r[k]
    got = sccs.bootstrap(prob, 2, 0.05, W, criterion=sccs.CRIT_FIXED, max_sweeps=15, column_order=1)
    _check(sccs, got, ref, 1e-9)
