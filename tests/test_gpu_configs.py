"""GPU parity at the benchmark configurations' own sizes.

* Mid (2M patients, ~20M eras, J = 2000, Laplace lambda = 1): 20 sweeps from
  beta = 0 in the benchmark's launch schedule (one sweep per launch on 128
  workgroups, after warm-up sweeps and a reset to zero), and a 100-sweep fit,
  which bounds the drift of the multiplicative state update over a long fit.
  Expected values: tests/golden/mid_laplace_fp64.npz, written by
  tests/golden/make_mid_golden.py from the oracle alone.
* Full scale (10M patients, ~100M eras, J = 4000, ~300M nonzeros, Normal
  variance 0.5): the FP64 and mixed GPU paths against each other at full size,
  FP64 g_j and h_j at the reached beta against the oracle, and both forms on
  the seeded 1 % patient subsample refit to convergence by the oracle.
* Batched outcomes: four of the 64 outcomes at their real sizes (the
  smallest, the largest and two in between) in one launch, 20 sweeps.
* Batched cross-validation: one fold of the mid problem walking the 16-value
  Laplace variance grid with warm starts (2 sweeps per link), beta and the
  held-out log-likelihood of every link against the oracle.

Besides rel_inf (max |difference| / max |beta|), every beta comparison checks
the per-coordinate relative error of the coordinates with |beta_j| >= 1e-3
and, under the Laplace prior, the pattern of exact zeros.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1208_0945_amd import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
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


def errors(beta, ref):
    """(rel_inf, max per-coordinate relative error over |ref_j| >= 1e-3)."""
    ri = float(np.max(np.abs(beta - ref)) / max(np.max(np.abs(ref)), 1e-300))
    big = np.abs(ref) >= 1e-3
    rc = float(np.max(np.abs(beta[big] - ref[big]) / np.abs(ref[big]))) if big.any() else 0.0
    return ri, rc


def check(beta, ref, tol, zeros=True, coord_tol=None):
    ri, rc = errors(beta, ref)
    print(f"rel_inf {ri:.3e}  per-coordinate (|beta| >= 1e-3) {rc:.3e}")
    assert ri <= tol
    assert rc <= (coord_tol if coord_tol is not None else 1e3 * tol)
    if zeros:
        assert np.array_equal(beta == 0.0, ref == 0.0)


@pytest.fixture(scope="module")
def mid():
    return synth.mid()


@pytest.fixture(scope="module")
def mid_golden(mid):
    g = np.load(os.path.join(HERE, "golden", "mid_laplace_fp64.npz"))
    assert str(g["seed_info"]) == mid.seed_info and int(g["nnz"]) == mid.nnz
    return g


def test_mid_twenty_sweeps_in_benchmark_schedule(sccs, mid, mid_golden):
    """5 warm-up sweeps, reset to beta = 0, then sweeps 1..20 one launch each
    on 128 workgroups (the merged-pass form takes over part-way)."""
    with sccs.Handle(mid, n_workgroups=128) as h:
        h.set_prior(sccs.PRIOR_LAPLACE, 2.0)
        for _ in range(5):
            h.sweep(1)
        h.set_beta(np.zeros(mid.n_cols))
        passes = []
        for _ in range(20):
            h.sweep(1)
            passes.append(h.pass_stats()[0])
        beta, trust = h.get_beta()
    print("passes per sweep:", passes)
    check(beta, mid_golden["beta20"], FP64_TOL, coord_tol=1e-6)
    assert np.max(np.abs(trust - mid_golden["trust20"])) <= 1e-9 * np.max(mid_golden["trust20"])


def test_mid_hundred_sweeps_bound_the_update_drift(sccs, mid, mid_golden):
    """100 sweeps in one launch with the default FP64 options (no exact
    refresh: w and den are only ever updated multiplicatively) against the
    oracle, which recomputes den exactly after every step; the log posterior
    after the last sweep agrees as well."""
    with sccs.Handle(mid, n_workgroups=128) as h:
        h.set_prior(sccs.PRIOR_LAPLACE, 2.0)
        lp = h.sweep(100, want_logpost=True)
        beta, _ = h.get_beta()
        L, P = h.objective()
    check(beta, mid_golden["beta100"], FP64_TOL, coord_tol=1e-6)
    ref_lp = float(mid_golden["logpost100"][-1])
    print(f"logpost GPU {lp!r} oracle {ref_lp!r}")
    assert abs(lp - ref_lp) <= 1e-11 * abs(ref_lp)
    assert abs(P - ref_lp) <= 1e-11 * abs(ref_lp)


@pytest.fixture(scope="module")
def full():
    return synth.full()


def test_full_scale_precision_form(sccs, full):
    """Full-scale workload: the mixed form (FP32 w and exp, FP64 sums) stays
    within 1e-6 of the FP64 GPU path over 3 sweeps; the FP64 path's g_j and
    h_j at the reached beta match the oracle's for sampled columns (largest,
    median, smallest)."""
    betas = {}
    with sccs.Handle(full, precision=1) as h:
        h.set_prior(sccs.PRIOR_NORMAL, 0.5)
        h.sweep(3)
        betas[1] = h.get_beta()[0]
    with sccs.Handle(full, precision=0) as h:
        h.set_prior(sccs.PRIOR_NORMAL, 0.5)
        h.sweep(3)
        betas[0] = h.get_beta()[0]
        c = np.diff(full.col_ptr)
        order = np.argsort(c)
        for j in (int(order[-1]), int(order[len(c) // 2]), int(order[0])):
            g, hh = h.grad_hess(j)
            go, ho = oracle.grad_hess(full, betas[0], j)
            scale = max(1.0, float(full.count[full.column(j)].sum()))   # Y'X_j: size of the cancelling terms
            print(f"column {j} (nnz {c[j]}): g {g!r} vs {go!r}, h {hh!r} vs {ho!r}")
            assert abs(g - go) <= 1e-12 * scale
            assert abs(hh - ho) <= 1e-9 * abs(ho)
    check(betas[1], betas[0], MIXED_TOL, zeros=False, coord_tol=1e-4)


def test_full_scale_subsample_refit(sccs, full):
    """The seeded 1 % patient subsample of the full-scale workload (all of the
    chosen patients' eras), refit by the oracle to convergence (relative
    log-posterior change < 1e-12): FP64 GPU within 1e-9, mixed within 1e-6,
    each after the oracle's sweep count."""
    sub = synth.subsample_patients(full, 0.01)
    ref = oracle.ccd(sub, oracle.PRIOR_NORMAL, 0.5, 500, oracle.CRIT_REL_LOGPOST, 1e-12)
    assert ref["converged"]
    print(f"oracle: {ref['sweeps']} sweeps on {sub.n_patients} patients, {sub.nnz} nonzeros")
    for prec, tol, ctol in ((0, FP64_TOL, 1e-6), (1, MIXED_TOL, 1e-4)):
        with sccs.Handle(sub, precision=prec) as h:
            h.set_prior(sccs.PRIOR_NORMAL, 0.5)
            h.sweep(ref["sweeps"])
            beta, _ = h.get_beta()
        check(beta, ref["beta"], tol, zeros=False, coord_tol=ctol)


def test_four_outcomes_at_real_size(sccs):
    """Outcomes 0..63 of the batched-outcomes workload keep their seeds; the
    smallest, the largest and two middle ones run in one launch (FP64, then
    the mixed form), 20 sweeps under Laplace lambda = 1."""
    sizes = synth.outcome_sizes(64)
    order = np.argsort(sizes)
    pick = [int(order[0]), int(order[21]), int(order[42]), int(order[-1])]
    probs = [synth.outcome(f, int(sizes[f])) for f in pick]
    refs = [oracle.ccd(p, oracle.PRIOR_LAPLACE, 2.0, 20)["beta"] for p in probs]
    for prec, tol in ((0, FP64_TOL), (1, MIXED_TOL)):
        specs = [sccs.FitSpec(i, [(sccs.PRIOR_LAPLACE, 2.0)]) for i in range(len(probs))]
        with sccs.Batch(probs, specs, precision=prec) as b:
            b.run(sccs.CRIT_FIXED, max_sweeps=20)
            for i, f in enumerate(pick):
                beta, res = b.get(i, 0)
                print(f"outcome {f} ({probs[i].n_patients} patients), precision {prec}:")
                assert res["sweeps"] == 20
                check(beta, refs[i], tol, zeros=(prec == 0), coord_tol=1e-6 if prec == 0 else 1e-4)


def test_cv_fold_chain_at_mid_size(sccs, mid):
    """One cross-validation fold of the mid problem (training weights 0/1)
    walks the 16 Laplace variances logspace(-3, 1) upward with warm starts and
    the trust region reset per link, 2 fixed sweeps per link, in the mixed form
    of the cross-validation workload and in FP64: beta of every link and the
    held-out log-likelihood (Eq. 2 over the fold's held-out patients) against
    the oracle."""
    folds = synth.cv_folds(mid.n_patients, 10)
    grid = synth.prior_grid(16)
    train = (folds != 3).astype(np.int32)
    held = (folds == 3).astype(np.int32)
    Ptr, Pho = oracle.OracleProblem(mid, train), oracle.OracleProblem(mid, held)
    refs, ref_ho = [], []
    beta = np.zeros(mid.n_cols)
    for v in grid:
        r = oracle.ccd(Ptr, oracle.PRIOR_LAPLACE, float(v), 2, beta0=beta)
        beta = r["beta"]
        refs.append(beta.copy())
        ref_ho.append(oracle.loglik(Pho, beta))
    for prec, tol, ho_tol in ((1, MIXED_TOL, 1e-7), (0, FP64_TOL, 1e-12)):
        spec = sccs.FitSpec(0, [(sccs.PRIOR_LAPLACE, float(v)) for v in grid], weight=train)
        with sccs.Batch([mid], [spec], precision=prec) as b:
            b.run(sccs.CRIT_FIXED, max_sweeps=2)
            for l in range(len(grid)):
                beta, res = b.get(0, l)
                ho = b.heldout(0, l)
                print(f"precision {prec}, link {l} (variance {grid[l]:.4g}): held-out L {ho!r} vs {ref_ho[l]!r}")
                assert res["sweeps"] == 2
                ri, _ = errors(beta, refs[l])
                assert ri <= tol, (l, ri)
                assert abs(ho - ref_ho[l]) <= ho_tol * abs(ref_ho[l])
