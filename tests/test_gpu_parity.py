"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle
on the same seeded inputs.

FP64 results differ from the oracle only in summation order (segmented and
tree sums on the GPU, sequential sums in the oracle; incremental den on the
GPU, recomputed den in the oracle), so trajectories must agree far inside
the 1e-6 relative tolerance on beta; the tests use 1e-9 on small problems.
The mixed-precision form is held to the 1e-6 relative bar on beta.
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


def zipf_small(n_patients=20000, n_cols=300, seed=0, p0=0.1):
    return synth.zipf_problem("zipf_small", n_patients, n_cols, p0, seed_path=(8, seed))


def run_gpu(sccs, prob, kind, var, sweeps, weight=None, precision=0, n_workgroups=0, beta0=None, tile_nnz=0,
            max_group=0):
    with sccs.Handle(prob, weight=weight, precision=precision, n_workgroups=n_workgroups, tile_nnz=tile_nnz,
                     max_group=max_group) as h:
        h.set_prior(kind, var)
        if beta0 is not None:
            h.set_beta(beta0)
        if sweeps:
            h.sweep(sweeps)
        return h.get_beta()


def run_gpu_launches(sccs, prob, kind, var, warm, n_single, **kw):
    """warm sweeps in one launch, then n_single one-sweep launches (so that
    the merged-pass form can take over); returns beta and pass counts."""
    with sccs.Handle(prob, **kw) as h:
        h.set_prior(kind, var)
        h.sweep(warm)
        passes = []
        for _ in range(n_single):
            h.sweep(1)
            passes.append(h.pass_stats()[0])
        return h.get_beta()[0], passes


def test_first_coordinates_at_zero_match_oracle(sccs):
    prob = synth.tiny()
    with sccs.Handle(prob) as h:
        for j in range(prob.n_cols):
            g, hh = h.grad_hess(j)
            go, ho = oracle.grad_hess(prob, np.zeros(prob.n_cols), j)
            assert abs(g - go) <= 1e-12 * max(1.0, abs(go))
            assert abs(hh - ho) <= 1e-12 * abs(ho)


@pytest.mark.parametrize("precision,tol", [(0, 1e-11), (1, 2e-6)])
def test_grad_hess_at_warm_start_match_oracle(sccs, precision, tol):
    prob = zipf_small(n_patients=5000, n_cols=40, seed=1)
    beta = synth.random_beta(prob.n_cols, 0.5, 11)
    with sccs.Handle(prob, precision=precision) as h:
        h.set_beta(beta)
        for j in range(prob.n_cols):
            g, hh = h.grad_hess(j)
            go, ho = oracle.grad_hess(prob, beta, j)
            # g = Y'X_j - N'W: its error is relative to the size of the two terms
            scale = max(1.0, float(prob.count[prob.column(j)].sum()))
            assert abs(g - go) <= tol * scale, (j, g, go)
            assert abs(hh - ho) <= tol * abs(ho), (j, hh, ho)


def test_grad_hess_inside_column_groups(sccs):
    """Columns at every position of multi-column groups (this problem has
    groups of up to four pairwise patient-disjoint columns)."""
    prob = zipf_small()
    beta = synth.random_beta(prob.n_cols, 0.3, 5)
    with sccs.Handle(prob) as h:
        h.set_beta(beta)
        for j in range(0, prob.n_cols, 3):
            g, hh = h.grad_hess(j)
            go, ho = oracle.grad_hess(prob, beta, j)
            scale = max(1.0, float(prob.count[prob.column(j)].sum()))
            assert abs(g - go) <= 1e-12 * scale, (j, g, go)
            assert abs(hh - ho) <= 1e-11 * abs(ho), (j, hh, ho)


@pytest.mark.parametrize("kind,var", [(1, 1.0), (2, 2.0), (0, 1.0), (2, 0.02)])
@pytest.mark.parametrize("sweeps", [1, 2, 20])
def test_tiny_trajectory_matches_oracle(sccs, kind, var, sweeps):
    prob = synth.tiny()
    ref = oracle.ccd(prob, kind, var, sweeps)
    beta, trust = run_gpu(sccs, prob, kind, var, sweeps)
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL
    assert np.max(np.abs(trust - ref["trust"])) <= 1e-9 * np.max(ref["trust"])
    assert np.array_equal(beta == 0.0, ref["beta"] == 0.0)


def test_tiny_fit_to_convergence(sccs):
    """Config: tiny, Normal var 1, until relative log-posterior change < 1e-8."""
    prob = synth.tiny()
    ref = oracle.ccd(prob, 1, 1.0, 500, oracle.CRIT_REL_LOGPOST, 1e-8)
    with sccs.Handle(prob) as h:
        h.set_prior(1, 1.0)
        r = h.fit(sccs.CRIT_REL_LOGPOST, 500, 1e-8)
        beta, _ = h.get_beta()
        assert r["converged"]
        # the stopping decision is taken on the same sweep (the relative change
        # at the firing sweep is far from the threshold on this problem)
        lp = np.concatenate([[oracle.loglik(prob, np.zeros(prob.n_cols))], ref["logpost_trace"]])
        ratio = np.abs(np.diff(lp)) / np.abs(lp[1:])
        assert ratio[ref["sweeps"] - 1] < 0.5e-8 and ratio[ref["sweeps"] - 2] > 2e-8, ratio
        assert r["sweeps"] == ref["sweeps"]
        assert abs(r["logpost"] - ref["logpost"]) <= 1e-10 * abs(ref["logpost"])
    # replay exactly the oracle's sweep count
    beta2, _ = run_gpu(sccs, prob, 1, 1.0, ref["sweeps"])
    assert rel_inf(beta2, ref["beta"]) <= FP64_TOL


def test_abs_dxbeta_criterion(sccs):
    """Section 2.2's rule, sum over eras of |change of (X beta)_k| below
    5e-4: the GPU stops after the oracle's sweep, with the oracle's beta."""
    prob = synth.tiny(seed=2)
    ref = oracle.ccd(prob, 2, 2.0, 500, oracle.CRIT_ABS_DXBETA, 5e-4)
    with sccs.Handle(prob) as h:
        h.set_prior(2, 2.0)
        r = h.fit(sccs.CRIT_ABS_DXBETA, 500, 5e-4)
        beta, _ = h.get_beta()
        assert r["converged"] and r["sweeps"] == ref["sweeps"]
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL
    assert np.array_equal(beta == 0.0, ref["beta"] == 0.0)


def test_patient_with_zero_total_length(sccs):
    """A patient whose eras all have length 0 (so n_i = 0 and den_i = 0) in
    every column: the fit stays finite and equals the oracle's."""
    base = zipf_small(n_patients=3000, n_cols=40, seed=4)
    J = base.n_cols
    ptr = np.concatenate([base.patient_ptr, [base.n_rows + 2]]).astype(np.int64)
    offset = np.concatenate([base.offset, [0, 0]]).astype(np.int32)
    count = np.concatenate([base.count, [0, 0]]).astype(np.int32)
    cols = [np.concatenate([base.column(j), [base.n_rows, base.n_rows + 1]]) for j in range(J)]
    col_ptr = np.zeros(J + 1, np.int64)
    col_ptr[1:] = np.cumsum([len(c) for c in cols])
    prob = synth.Problem("zero_len", base.n_patients + 1, ptr, offset, count, J, col_ptr,
                         np.concatenate(cols).astype(np.int32), np.zeros(J))
    for kind, var in ((2, 2.0), (1, 0.5)):
        ref = oracle.ccd(prob, kind, var, 5)
        beta, _ = run_gpu(sccs, prob, kind, var, 5)
        assert np.all(np.isfinite(beta))
        assert rel_inf(beta, ref["beta"]) <= FP64_TOL


@pytest.mark.parametrize("n_workgroups,tile_nnz,max_group",
                         [(1, 0, 0), (3, 0, 0), (64, 0, 0), (0, 0, 0), (0, 16, 0), (97, 32, 0), (0, 0, 1), (5, 0, 2)])
def test_zipf_laplace_20_sweeps(sccs, n_workgroups, tile_nnz, max_group):
    """Mid-shaped (Zipf columns, 1+Poisson(9) eras) at 20k patients, Laplace
    lambda = 1, 20 sweeps; several workgroup counts (ownership splits), tile
    sizes and column-group sizes (1 = one column per reduction)."""
    prob = zipf_small()
    ref = oracle.ccd(prob, 2, 2.0, 20)
    beta, _ = run_gpu(sccs, prob, 2, 2.0, 20, n_workgroups=n_workgroups, tile_nnz=tile_nnz, max_group=max_group)
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL
    assert np.array_equal(beta == 0.0, ref["beta"] == 0.0)


@pytest.mark.parametrize("n_workgroups,tile_nnz,max_group",
                         [(1, 0, 0), (3, 0, 0), (64, 0, 0), (0, 0, 0), (0, 16, 0), (97, 32, 0), (0, 0, 1), (5, 0, 2)])
def test_zipf_laplace_merged_form(sccs, n_workgroups, tile_nnz, max_group):
    """The same shapes with single-sweep launches after a warm-up launch, so
    that the merged-pass form takes over once most steps are zero (Laplace
    lambda = 2): beta after 40 sweeps against the oracle's."""
    prob = zipf_small()
    ref = oracle.ccd(prob, 2, 0.5, 40)
    with sccs.Handle(prob, n_workgroups=n_workgroups, tile_nnz=tile_nnz, max_group=max_group) as h:
        h.set_prior(2, 0.5)
        h.sweep(10)
        passes = [h.pass_stats()[0]]
        for _ in range(30):
            h.sweep(1)
            passes.append(h.pass_stats()[0])
        beta, _ = h.get_beta()
    print("passes per launch:", passes)
    assert min(passes[1:]) < passes[0] // 10, "the merged form should have taken over"
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL
    assert np.array_equal(beta == 0.0, ref["beta"] == 0.0)


@pytest.mark.parametrize("precision,max_group", [(0, 0), (1, 0), (0, 1)])
def test_merged_passes_match_plain_order(sccs, precision, max_group):
    """Merged passes (consecutive column groups in one reduction when the
    columns linking them are predicted to stay put) against one pass per
    group: the same beta bit for bit after every sweep, also after a prior
    change that makes predicted-quiet columns move (merges rejected and the
    rejected groups visited again); merges and rejections both occur, and
    with one-column groups some passes hold more than two groups; FP64 beta
    equals the oracle's for the same prior chain."""
    prob = zipf_small()
    chain = [(0.05, 12), (5.0, 8)]
    betas, stats = {}, {}
    for merge in (0, 1):
        with sccs.Handle(prob, precision=precision, merge_passes=merge, max_group=max_group) as h:
            seq, st = [], []
            for var, n in chain:
                h.set_prior(2, var)
                for _ in range(n):
                    h.sweep(1)
                    seq.append(h.get_beta()[0])
                    st.append(h.pass_stats())
            betas[merge], stats[merge] = seq, st
    for k, (b0, b1) in enumerate(zip(betas[0], betas[1])):
        assert np.array_equal(b0, b1), f"sweep {k}"
    print("passes/rejects/zero steps per sweep, merged:", stats[1], "plain:", stats[0][0])
    assert len({p for p, _, _ in stats[0]}) == 1 and all(r == 0 for _, r, _ in stats[0])
    assert sum(p for p, _, _ in stats[1]) < sum(p for p, _, _ in stats[0])
    if max_group == 1:
        n_groups = stats[0][0][0]
        assert 2 * min(p for p, _, _ in stats[1]) < n_groups, "some pass holds three groups or more"
    assert sum(r for _, r, _ in stats[1]) > 0
    # a zero step leaves beta_j unchanged (not conversely: a step can be lost
    # in rounding); both forms count the same zero steps
    for k in range(1, len(betas[0])):
        unchanged = int(np.sum(betas[0][k] == betas[0][k - 1]))
        assert 0 <= stats[0][k][2] <= unchanged
        assert stats[1][k][2] == stats[0][k][2], k
    if precision == 0:
        r1 = oracle.ccd(prob, 2, 0.05, 12)
        r2 = oracle.ccd(prob, 2, 5.0, 8, beta0=r1["beta"], trust0=r1["trust"])
        assert rel_inf(betas[1][-1], r2["beta"]) <= FP64_TOL


def ragged_problem():
    """Patients from 1 to 300 eras; a column covering every era of the long
    patients (segments longer than one wavefront), an empty column, a single
    nonzero column and patients without events."""
    rng = np.random.default_rng(77)
    sizes = np.concatenate([[300, 1, 130, 65, 64, 63, 2], rng.integers(1, 12, size=400)])
    ptr = np.zeros(len(sizes) + 1, np.int64)
    ptr[1:] = np.cumsum(sizes)
    K = int(ptr[-1])
    offset = rng.integers(1, 365, size=K).astype(np.int32)
    count = rng.poisson(0.3, size=K).astype(np.int32)
    count[ptr[5]:ptr[6]] = 0                      # a patient with n_i = 0
    count[ptr[0]] = max(count[ptr[0]], 1)
    cols = []
    long_rows = np.concatenate([np.arange(ptr[i], ptr[i + 1]) for i in (0, 2, 3, 4)])
    cols.append(np.unique(np.concatenate([long_rows, np.flatnonzero(rng.random(K) < 0.1)])))
    cols.append(np.zeros(0, np.int64))            # empty column
    cols.append(np.array([ptr[7]]))               # one nonzero
    for _ in range(5):
        cols.append(np.flatnonzero(rng.random(K) < rng.uniform(0.02, 0.5)))
    col_ptr = np.zeros(len(cols) + 1, np.int64)
    col_ptr[1:] = np.cumsum([len(c) for c in cols])
    return synth.Problem("ragged", len(sizes), ptr, offset, count, len(cols), col_ptr,
                         np.concatenate(cols).astype(np.int32), np.zeros(len(cols)))


@pytest.mark.parametrize("kind,var", [(1, 0.5), (2, 0.5)])
@pytest.mark.parametrize("n_workgroups", [1, 5, 0])
def test_ragged_and_long_segments(sccs, kind, var, n_workgroups):
    prob = ragged_problem()
    ref = oracle.ccd(prob, kind, var, 10)
    beta, _ = run_gpu(sccs, prob, kind, var, 10, n_workgroups=n_workgroups)
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL
    assert beta[1] == 0.0  # empty column never moves
    # the same with one-sweep launches from sweep 5 on (merged passes once
    # most steps are zero)
    ref = oracle.ccd(prob, kind, var, 30)
    beta, passes = run_gpu_launches(sccs, prob, kind, var, 5, 25, n_workgroups=n_workgroups)
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL
    assert beta[1] == 0.0


@pytest.mark.parametrize("mode", ["cv", "bootstrap"])
def test_patient_weights(sccs, mode):
    prob = zipf_small(n_patients=8000, n_cols=100, seed=3)
    if mode == "cv":
        w = (synth.cv_folds(prob.n_patients, 10, seed=1) != 3).astype(np.int32)
    else:
        w = np.random.default_rng(5).multinomial(prob.n_patients, np.full(prob.n_patients, 1.0 / prob.n_patients)).astype(np.int32)
    ref = oracle.ccd(prob, 2, 2.0, 10, weight=w)
    beta, _ = run_gpu(sccs, prob, 2, 2.0, 10, weight=w)
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL


def test_objective_matches_oracle(sccs):
    prob = zipf_small(n_patients=5000, n_cols=50, seed=4)
    with sccs.Handle(prob) as h:
        h.set_prior(2, 0.5)
        h.sweep(3)
        beta, _ = h.get_beta()
        L, P = h.objective()
        lp = h.sweep(1, want_logpost=True)
        beta4, _ = h.get_beta()
    Lo = oracle.loglik(prob, beta)
    assert abs(L - Lo) <= 1e-11 * abs(Lo)
    assert abs(P - (Lo + oracle.log_prior(2, 0.5, beta))) <= 1e-11 * abs(Lo)
    Lo4 = oracle.loglik(prob, beta4) + oracle.log_prior(2, 0.5, beta4)
    assert abs(lp - Lo4) <= 1e-11 * abs(Lo4)


def test_deterministic(sccs):
    prob = zipf_small(n_patients=10000, n_cols=120, seed=5)
    a, _ = run_gpu(sccs, prob, 1, 0.5, 5)
    b, _ = run_gpu(sccs, prob, 1, 0.5, 5)
    assert np.array_equal(a, b)


def test_checkpoint_resume(sccs):
    prob = zipf_small(n_patients=10000, n_cols=120, seed=6)
    straight, _ = run_gpu(sccs, prob, 2, 2.0, 20)
    with sccs.Handle(prob) as h:
        h.set_prior(2, 2.0)
        h.sweep(10)
        beta, trust = h.get_beta()
    with sccs.Handle(prob) as h:
        h.set_prior(2, 2.0)
        h.set_beta(beta, trust)
        h.sweep(10)
        resumed, _ = h.get_beta()
    assert rel_inf(resumed, straight) <= 1e-11
    ref = oracle.ccd(prob, 2, 2.0, 20)
    assert rel_inf(resumed, ref["beta"]) <= FP64_TOL


@pytest.mark.parametrize("kind,var", [(2, 2.0), (1, 0.5)])
def test_mixed_precision_error_bound(sccs, kind, var):
    prob = zipf_small(n_patients=20000, n_cols=200, seed=7)
    ref = oracle.ccd(prob, kind, var, 20)
    beta, _ = run_gpu(sccs, prob, kind, var, 20, precision=1)
    err = rel_inf(beta, ref["beta"])
    print(f"mixed-precision rel_inf error vs FP64 oracle: {err:.3e}")
    assert err <= MIXED_TOL


def test_numeric_failure_reported(sccs):
    """A warm start far outside the range of exp (beta_0 = 800) makes
    w = l e^800 overflow; the first visit then sees a non-finite gradient.
    The library reports it and keeps the last finite beta."""
    prob = synth.tiny()
    beta0 = np.zeros(prob.n_cols)
    beta0[0] = 800.0
    for precision in (0, 1):
        with sccs.Handle(prob, precision=precision) as h:
            h.set_prior(1, 1.0)
            h.set_beta(beta0)
            with pytest.raises(sccs.SccsError) as e:
                h.sweep(2)
            assert e.value.status == sccs.ERR_NUMERIC
            beta, _ = h.get_beta()
            assert np.all(np.isfinite(beta)) and beta[0] == 800.0
            # the handle stays usable after a reset of the start point
            h.set_beta(np.zeros(prob.n_cols))
            h.sweep(1)


def test_errors_without_prior_and_bad_args(sccs):
    prob = synth.tiny()
    with sccs.Handle(prob) as h:
        with pytest.raises(sccs.SccsError) as e:
            h.sweep(1)
        assert e.value.status == sccs.ERR_STATE
        with pytest.raises(sccs.SccsError):
            h.set_prior(1, -1.0)
        with pytest.raises(sccs.SccsError):
            h.grad_hess(prob.n_cols)
        with pytest.raises(sccs.SccsError):
            h.set_beta(np.full(prob.n_cols, np.nan))


def test_maximum_columns_and_limits(sccs):
    """J at the library's maximum (6144 columns: beta, trust and the sweep's
    start copy of beta fill the LDS), against the oracle; one column more is
    rejected at creation."""
    prob = synth.zipf_problem("widest", 3000, 6144, 0.3, seed_path=(12, 1), n_effects=20)
    ref = oracle.ccd(prob, 1, 0.5, 2)
    beta, _ = run_gpu(sccs, prob, 1, 0.5, 2)
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL
    wider = synth.zipf_problem("too_wide", 500, 6145, 0.3, seed_path=(12, 2), n_effects=5)
    with pytest.raises(sccs.SccsError) as e:
        sccs.Handle(wider)
    assert e.value.status == sccs.ERR_INVALID_ARG


def test_no_nonzeros_and_single_patient(sccs):
    """Degenerate inputs: a problem whose columns are all empty (every step
    is zero and beta stays 0, Normal or Laplace), and a single patient."""
    base = synth.tiny(n_patients=50, n_cols=5)
    empty = synth.Problem("empty", base.n_patients, base.patient_ptr, base.offset, base.count, 5,
                          np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(5))
    for kind in (1, 2):
        beta, _ = run_gpu(sccs, empty, kind, 1.0, 3)
        assert np.all(beta == 0.0)
        beta, _ = run_gpu_launches(sccs, empty, kind, 1.0, 1, 3)   # all steps zero: merged form
        assert np.all(beta == 0.0)
    one = synth.Problem("one", 1, np.array([0, 4], np.int64), np.array([10, 20, 30, 40], np.int32),
                        np.array([1, 0, 2, 1], np.int32), 2, np.array([0, 2, 3], np.int64),
                        np.array([0, 2, 1], np.int32), np.zeros(2))
    ref = oracle.ccd(one, 1, 1.0, 5)
    beta, _ = run_gpu(sccs, one, 1, 1.0, 5)
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL
    ref = oracle.ccd(one, 2, 1.0, 60)
    beta, _ = run_gpu_launches(sccs, one, 2, 1.0, 20, 40)
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL


@pytest.mark.parametrize("n_workgroups", [128, 0])
def test_full_size_mid_parity(sccs, n_workgroups):
    """Full mid workload (2M patients, ~20M eras, J = 2000, Laplace lambda = 1)
    in the benchmark's launch configuration (128 workgroups) and with one
    workgroup per CU: the first 3 sweeps against the oracle, then g_j, h_j of
    sampled columns at the reached beta."""
    prob = synth.mid()
    ref = oracle.ccd(prob, 2, 2.0, 3)
    with sccs.Handle(prob, n_workgroups=n_workgroups) as h:
        h.set_prior(2, 2.0)
        h.sweep(3)
        beta, _ = h.get_beta()
        assert rel_inf(beta, ref["beta"]) <= FP64_TOL
        c = np.diff(prob.col_ptr)
        for j in [int(np.argmax(c)), int(np.argmin(c)), int(np.argsort(c)[len(c) // 2]), 7]:
            g, hh = h.grad_hess(j)
            go, ho = oracle.grad_hess(prob, beta, j)
            assert abs(g - go) <= 1e-9 * max(1.0, abs(ho)), (j, g, go)
            assert abs(hh - ho) <= 1e-9 * abs(ho), (j, hh, ho)


def test_full_size_mid_merged_passes_parity(sccs):
    """Full mid workload in the benchmark's launch configuration and schedule
    (128 workgroups, one sweep per launch) until the merged-pass form has run
    a few sweeps: beta after 14 sweeps against the oracle's, the same exact
    zeros, and g_j, h_j of sampled columns at the reached beta."""
    prob = synth.mid()
    ref = oracle.ccd(prob, 2, 2.0, 14)
    with sccs.Handle(prob, n_workgroups=128) as h:
        h.set_prior(2, 2.0)
        passes = []
        for _ in range(14):
            h.sweep(1)
            passes.append(h.pass_stats()[0])
        beta, _ = h.get_beta()
        assert passes[-1] < passes[0], passes   # the last launches merged groups
        assert rel_inf(beta, ref["beta"]) <= FP64_TOL
        assert np.array_equal(beta == 0.0, ref["beta"] == 0.0)
        c = np.diff(prob.col_ptr)
        for j in [int(np.argmax(c)), int(np.argsort(c)[len(c) // 2]), 1999]:
            g, hh = h.grad_hess(j)
            go, ho = oracle.grad_hess(prob, beta, j)
            assert abs(g - go) <= 1e-9 * max(1.0, abs(ho)), (j, g, go)
            assert abs(hh - ho) <= 1e-9 * abs(ho), (j, hh, ho)


def test_autotuner_picks_a_candidate_and_its_schedule_is_exact(sccs):
    prob = zipf_small(n_patients=20000, n_cols=120, seed=9)
    best, table = sccs.tune(prob, sccs.PRIOR_LAPLACE, 2.0, n_sweeps=2)
    assert len(table) >= 6
    assert any(t["n_workgroups"] == best["n_workgroups"] and t["tile_nnz"] == best["tile_nnz"] for t in table)
    assert all(t["ms_per_sweep"] > 0 for t in table)
    ref = oracle.ccd(prob, 2, 2.0, 5)
    beta, _ = run_gpu(sccs, prob, 2, 2.0, 5, **best)
    assert rel_inf(beta, ref["beta"]) <= FP64_TOL


def test_group_times_cover_the_sweep(sccs):
    """sccs_group_times after a one-pass launch with timing on: one stamp per
    column group, non-decreasing, inside the kernel's own time; refused
    without timing, after a merged-pass launch and for valued problems; the
    stamps leave the trajectory unchanged."""
    prob = zipf_small()
    with sccs.Handle(prob, n_workgroups=64, merge_passes=0) as h:
        h.set_prior(sccs.PRIOR_LAPLACE, 2.0)
        h.sweep(1)
        with pytest.raises(sccs.SccsError):
            h.group_times()     # timing is off by default
        h.group_timing(True)
        h.sweep(2)
        t, fc = h.group_times()
        ms = h.last_kernel_ms()
        b_stamped = h.get_beta()[0]
        h.group_timing(False)
        h.sweep(1)
        with pytest.raises(sccs.SccsError):
            h.group_times()
    with sccs.Handle(prob, n_workgroups=64, merge_passes=0) as h:
        h.set_prior(sccs.PRIOR_LAPLACE, 2.0)
        h.sweep(3)
        assert np.array_equal(h.get_beta()[0], b_stamped)
    assert fc[0] == 0 and fc[-1] == prob.n_cols and np.all(np.diff(fc) >= 1)
    assert len(t) == len(fc) - 1 and np.all(t > 0) and np.all(np.diff(t) >= 0)
    assert t[-1] * 1e-3 <= ms
    with sccs.Handle(prob) as h:
        h.set_prior(sccs.PRIOR_LAPLACE, 2.0)
        h.group_timing(True)
        h.sweep(1)          # first launch: one pass per group
        h.group_times()
        h.sweep(30)
        zero_share = h.pass_stats()[2] / (30 * prob.n_cols)
        h.sweep(1)          # merged passes once most steps were zero
        if zero_share >= 0.5:
            with pytest.raises(sccs.SccsError):
                h.group_times()
        else:
            h.group_times()
