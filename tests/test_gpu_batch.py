"""GPU parity of the batched form, each fit checked against the FP64 oracle
run fit by fit, under both engines: fits on disjoint workgroup ranges of one
launch (each running the single-fit sweep), and all fits advanced in
lockstep on every workgroup.

Configurations mirror the batched workloads at reduced size: independent
outcomes over one shared drug vocabulary with uneven patient counts, and
patient-level cross-validation folds walking a prior-variance path with warm
starts (trust region reset per link).
"""
import numpy as np
import pytest

import oracle
from paper_1208_0945_amd import synth

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9


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
    """Both engines of the batched form: fits on disjoint workgroup ranges
    (0), or all fits in lockstep on every workgroup (1)."""
    return request.param


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def outcomes(n_fits, n_cols=60, lo=2000, hi=30000, seed=0):
    sizes = synth.outcome_sizes(n_fits, lo=lo, hi=hi, seed=seed)
    return synth.batched_outcomes(n_fits, n_cols=n_cols, seed=seed, sizes=sizes)


@pytest.mark.parametrize("n_workgroups", [0, 24])
def test_outcomes_uneven_sizes_relabelled(sccs, n_workgroups):
    """Partitioned engine, drugs renumbered for independence, 24 outcomes
    whose patient counts span two orders of magnitude (so the launch shapes
    give the large fits more workgroups; on 24 workgroups at most three fits
    share a launch): every fit against the oracle on its renumbered
    problem."""
    probs = outcomes(24, n_cols=48, lo=600, hi=60000, seed=3)
    with sccs.Batch(probs, [sccs.FitSpec(f, [(sccs.PRIOR_LAPLACE, 2.0)]) for f in range(len(probs))],
                    n_workgroups=n_workgroups, engine=0, column_order=1) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=5)
        for f, p in enumerate(probs):
            beta, res = b.get(f, 0)
            order = oracle.independent_order(p, 4)
            ref = oracle.ccd(synth.permute_columns(p, order), oracle.PRIOR_LAPLACE, 2.0, 5)
            want = np.empty_like(ref["beta"])
            want[order] = ref["beta"]
            assert res["sweeps"] == 5
            assert rel_inf(beta, want) <= FP64_TOL, f
            assert abs(res["logpost"] - ref["logpost"]) <= 1e-10 * abs(ref["logpost"])


@pytest.mark.parametrize("n_fits,n_workgroups", [(1, 0), (5, 0), (20, 0), (5, 7)])
def test_outcomes_fixed_sweeps_match_oracle(sccs, engine, n_fits, n_workgroups):
    probs = outcomes(n_fits)
    with sccs.Batch(probs, [sccs.FitSpec(f, [(sccs.PRIOR_LAPLACE, 2.0)]) for f in range(n_fits)],
                    n_workgroups=n_workgroups, engine=engine) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=6)
        for f, p in enumerate(probs):
            beta, res = b.get(f, 0)
            ref = oracle.ccd(p, oracle.PRIOR_LAPLACE, 2.0, 6)
            assert res["sweeps"] == 6
            assert rel_inf(beta, ref["beta"]) <= FP64_TOL, f
            assert abs(res["logpost"] - ref["logpost"]) <= 1e-10 * abs(ref["logpost"])


def test_sixty_four_fits_and_limit(sccs, engine):
    """The maximum batch (64 fits over 8 small problems; two launches of 32
    fits in the partitioned engine), every fit against the oracle; a 65th
    fit is rejected."""
    probs = outcomes(8, n_cols=24, lo=500, hi=4000, seed=5)
    specs = [sccs.FitSpec(f % 8, [(sccs.PRIOR_NORMAL, 0.25 * (1 + f // 8))]) for f in range(64)]
    with sccs.Batch(probs, specs, engine=engine) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=3)
        for f in range(64):
            ref = oracle.ccd(probs[f % 8], oracle.PRIOR_NORMAL, 0.25 * (1 + f // 8), 3)
            beta, _ = b.get(f)
            assert rel_inf(beta, ref["beta"]) <= FP64_TOL, f
    with pytest.raises(sccs.SccsError):
        sccs.Batch(probs, specs + [specs[0]], engine=engine)


def test_outcomes_to_convergence(sccs, engine):
    probs = outcomes(6, seed=3)
    with sccs.Batch(probs, [sccs.FitSpec(f, [(sccs.PRIOR_NORMAL, 0.5)]) for f in range(6)], engine=engine) as b:
        b.run(sccs.CRIT_REL_LOGPOST, max_sweeps=300, tol=1e-10)
        for f, p in enumerate(probs):
            beta, res = b.get(f, 0)
            ref = oracle.ccd(p, oracle.PRIOR_NORMAL, 0.5, 300, oracle.CRIT_REL_LOGPOST, 1e-10)
            assert res["converged"] and abs(res["sweeps"] - ref["sweeps"]) <= 1
            assert rel_inf(beta, ref["beta"]) <= 1e-7


def test_cv_folds_with_warm_started_prior_path(sccs, engine):
    """10 folds x a 4-step Laplace variance path (ascending, warm starts).
    Each link runs a fixed number of sweeps so the trajectory is compared
    exactly; the oracle replays the same warm-start chain."""
    prob = synth.zipf_problem("cvsmall", 6000, 50, 0.1, seed_path=(9, 1))
    folds = synth.cv_folds(prob.n_patients, 10, seed=2)
    grid = [0.01, 0.1, 1.0, 10.0]
    specs = [sccs.FitSpec(0, [(sccs.PRIOR_LAPLACE, v) for v in grid], weight=(folds != k).astype(np.int32))
             for k in range(10)]
    with sccs.Batch([prob], specs, engine=engine) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=4)
        for k in range(10):
            w = (folds != k).astype(np.int32)
            beta = np.zeros(prob.n_cols)
            for l, v in enumerate(grid):
                ref = oracle.ccd(prob, oracle.PRIOR_LAPLACE, v, 4, beta0=beta, weight=w)
                beta = ref["beta"]
                got, res = b.get(k, l)
                assert res["sweeps"] == 4
                assert rel_inf(got, beta) <= FP64_TOL, (k, l)
                # held-out Eq. 2 over fold k's patients at the oracle's iterate
                ho = oracle.loglik(prob, beta, weight=(folds == k).astype(np.int32))
                assert abs(b.heldout(k, l) - ho) <= 1e-8 * abs(ho), (k, l)


def test_bootstrap_replicates(sccs, engine):
    """Bootstrap replicates as integer patient multiplicities (Section 2.5);
    the out-of-bag patients (weight 0) form each replicate's held-out set."""
    prob = synth.zipf_problem("boot", 3000, 30, 0.1, seed_path=(9, 3))
    wts = synth.bootstrap_weights(prob.n_patients, 6, seed=4)
    specs = [sccs.FitSpec(0, [(sccs.PRIOR_NORMAL, 0.5)], weight=w) for w in wts]
    with sccs.Batch([prob], specs, engine=engine) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=5)
        for r, w in enumerate(wts):
            ref = oracle.ccd(prob, oracle.PRIOR_NORMAL, 0.5, 5, weight=w)
            got, res = b.get(r)
            assert rel_inf(got, ref["beta"]) <= FP64_TOL, r
            assert abs(res["logpost"] - ref["logpost"]) <= 1e-10 * abs(ref["logpost"])
            oob = oracle.loglik(prob, ref["beta"], weight=(w == 0).astype(np.int32))
            assert abs(b.heldout(r) - oob) <= 1e-8 * abs(oob), r


@pytest.mark.parametrize("n_reps,max_group", [(20, 0), (20, 1), (6, 2)])
def test_bootstrap_column_groups(sccs, engine, n_reps, max_group):
    """Replicates of one problem share its column groups: 20 replicates give
    groups of up to 3 columns (2 F m <= 128 words), 6 replicates up to the
    requested width; every replicate against the oracle, and the grouped run
    against the one-column-per-group run."""
    prob = synth.zipf_problem("bootg", 4000, 40, 0.03, seed_path=(9, 5))
    wts = synth.bootstrap_weights(prob.n_patients, n_reps, seed=6)
    specs = [sccs.FitSpec(0, [(sccs.PRIOR_LAPLACE, 2.0)], weight=w) for w in wts]
    with sccs.Batch([prob], specs, max_group=max_group, engine=engine) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=6)
        got = [b.get(r)[0] for r in range(n_reps)]
    with sccs.Batch([prob], specs, max_group=1, engine=engine) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=6)
        plain = [b.get(r)[0] for r in range(n_reps)]
    for r in range(n_reps):
        assert rel_inf(got[r], plain[r]) <= 1e-12, r
    for r in (0, n_reps - 1):
        ref = oracle.ccd(prob, oracle.PRIOR_LAPLACE, 2.0, 6, weight=wts[r])
        assert rel_inf(got[r], ref["beta"]) <= FP64_TOL, r
        assert np.array_equal(got[r] == 0.0, ref["beta"] == 0.0)


def test_batch_mixed_precision(sccs, engine):
    probs = outcomes(4, seed=5)
    with sccs.Batch(probs, [sccs.FitSpec(f, [(sccs.PRIOR_LAPLACE, 2.0)]) for f in range(4)],
                    precision=sccs.PREC_MIXED, engine=engine) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=10)
        for f, p in enumerate(probs):
            beta, _ = b.get(f, 0)
            ref = oracle.ccd(p, oracle.PRIOR_LAPLACE, 2.0, 10)
            assert rel_inf(beta, ref["beta"]) <= 1e-6


@pytest.mark.parametrize("refresh", [0, 3])
def test_batch_refresh_periods(sccs, engine, refresh):
    """Exact refreshes every few sweeps (every thread of a workgroup takes
    the refresh and its barrier together), and none at all."""
    probs = outcomes(3, seed=6)
    with sccs.Batch(probs, [sccs.FitSpec(f, [(sccs.PRIOR_LAPLACE, 2.0)]) for f in range(3)],
                    precision=sccs.PREC_MIXED, refresh_period=refresh, engine=engine) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=10)
        for f, p in enumerate(probs):
            beta, res = b.get(f, 0)
            assert res["sweeps"] == 10
            assert rel_inf(beta, oracle.ccd(p, oracle.PRIOR_LAPLACE, 2.0, 10)["beta"]) <= 1e-6


def test_batch_rejects_bad_specs(sccs, engine):
    probs = outcomes(2)
    with pytest.raises(sccs.SccsError):
        sccs.Batch(probs, [sccs.FitSpec(5, [(sccs.PRIOR_NORMAL, 1.0)])], engine=engine)
    with pytest.raises(sccs.SccsError):
        sccs.Batch(probs, [sccs.FitSpec(0, [(sccs.PRIOR_NORMAL, -1.0)])], engine=engine)
    other = synth.tiny(n_cols=7)
    with pytest.raises(sccs.SccsError):
        sccs.Batch([probs[0], other], [sccs.FitSpec(0, [(sccs.PRIOR_NORMAL, 1.0)])], engine=engine)


def test_heldout_needs_weights_and_a_run(sccs, engine):
    """No weights: no held-out set.  Weights without a 0: empty set, L = 0."""
    prob = synth.tiny()
    ones = np.ones(prob.n_patients, dtype=np.int32)
    specs = [sccs.FitSpec(0, [(sccs.PRIOR_NORMAL, 1.0)]), sccs.FitSpec(0, [(sccs.PRIOR_NORMAL, 1.0)], weight=ones)]
    with sccs.Batch([prob], specs, engine=engine) as b:
        with pytest.raises(sccs.SccsError):
            b.heldout(1, 0)            # link has not run
        b.run(sccs.CRIT_FIXED, max_sweeps=2)
        with pytest.raises(sccs.SccsError):
            b.heldout(0, 0)            # no weights
        assert b.heldout(1, 0) == 0.0


def test_batch_autotuner_picks_a_candidate_and_its_schedule_is_exact(sccs, engine):
    """sccs_batch_tune times launch shapes on the batch itself; the batch
    run with the chosen shape still matches the oracle fit by fit."""
    probs = outcomes(6, n_cols=40, lo=3000, hi=20000, seed=3)
    specs = [sccs.FitSpec(f, [(sccs.PRIOR_LAPLACE, 2.0)]) for f in range(len(probs))]
    best, table = sccs.batch_tune(probs, specs, n_sweeps=2, engine=engine)
    assert len(table) >= 6 and all(t["ms_per_sweep"] > 0 for t in table)
    assert any(t["n_workgroups"] == best["n_workgroups"] and t["tile_nnz"] == best["tile_nnz"] for t in table)
    with sccs.Batch(probs, specs, n_workgroups=best["n_workgroups"], tile_nnz=best["tile_nnz"], engine=engine) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=5)
        for f, p in enumerate(probs):
            beta, _ = b.get(f, 0)
            assert rel_inf(beta, oracle.ccd(p, oracle.PRIOR_LAPLACE, 2.0, 5)["beta"]) <= FP64_TOL
