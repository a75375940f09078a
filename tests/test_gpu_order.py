"""GPU parity under the independence relabelling (SCCS_ORDER_INDEPENDENT).

The library visits the columns in the order of sccs_column_order; the oracle
runs Algorithm 1 on the problem with its columns renumbered by its own
restatement of that rule (oracle.independent_order, equal to the library's
order bit for bit, see tests/test_order_cpu.py), and its results are mapped
back to the problem's numbering.  Betas, trust bounds, class memberships and
grad_hess's column index stay in the problem's numbering at the ABI.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1208_0945_amd import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FP64_TOL = 1e-9
IND = 1


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


def unpermute(x, order):
    out = np.empty_like(x)
    out[np.asarray(order)] = x
    return out


def oracle_relabelled(prob, kind, var, sweeps, criterion=oracle.CRIT_FIXED, tol=0.0, weight=None, beta0=None):
    order = oracle.independent_order(prob, 4)
    perm = synth.permute_columns(prob, order)
    b0 = None if beta0 is None else np.asarray(beta0)[order]
    r = oracle.ccd(perm, kind, var, sweeps, criterion, tol, beta0=b0, weight=weight)
    return order, unpermute(r["beta"], order), unpermute(r["trust"], order), r


@pytest.fixture(scope="module")
def zipf():
    return synth.zipf_problem("zipf_order", 20000, 120, 0.05, seed_path=(9, 31))


@pytest.mark.parametrize("kind,var,n_workgroups", [(2, 2.0, 0), (1, 0.5, 40), (2, 0.05, 96)])
def test_relabelled_trajectory_matches_oracle(sccs, zipf, kind, var, n_workgroups):
    order, ref_beta, ref_trust, ref = oracle_relabelled(zipf, kind, var, 8)
    with sccs.Handle(zipf, n_workgroups=n_workgroups, column_order=IND) as h:
        assert np.array_equal(h.column_order(), order)
        h.set_prior(kind, var)
        lp = h.sweep(8, want_logpost=True)
        beta, trust = h.get_beta()
    assert rel_inf(beta, ref_beta) <= FP64_TOL
    assert np.max(np.abs(trust - ref_trust)) <= 1e-9 * np.max(ref_trust)
    assert np.array_equal(beta == 0.0, ref_beta == 0.0)
    assert abs(lp - ref["logpost"]) <= 1e-11 * abs(ref["logpost"])


def test_relabelled_fit_stops_at_the_oracle_sweep(sccs, zipf):
    _, ref_beta, _, ref = oracle_relabelled(zipf, 2, 2.0, 300, oracle.CRIT_REL_LOGPOST, 1e-10)
    assert ref["converged"]
    with sccs.Handle(zipf, column_order=IND) as h:
        h.set_prior(sccs.PRIOR_LAPLACE, 2.0)
        r = h.fit(sccs.CRIT_REL_LOGPOST, 300, 1e-10)
        beta, _ = h.get_beta()
    assert r["converged"] and r["sweeps"] == ref["sweeps"]
    assert rel_inf(beta, ref_beta) <= FP64_TOL


def test_relabelled_handle_keeps_the_problem_numbering(sccs, zipf):
    """set_beta / get_beta round trip and grad_hess(j) at a warm start, both
    in the problem's column numbering (g and h at a given beta do not depend
    on the visiting order, so the plain oracle is the reference)."""
    beta = synth.random_beta(zipf.n_cols, 0.3, 12)
    trust = 0.5 + np.arange(zipf.n_cols) / zipf.n_cols
    with sccs.Handle(zipf, column_order=IND) as h:
        h.set_beta(beta, trust)
        b, t = h.get_beta()
        assert np.array_equal(b, beta) and np.array_equal(t, trust)
        for j in range(0, zipf.n_cols, 7):
            g, hh = h.grad_hess(j)
            go, ho = oracle.grad_hess(zipf, beta, j)
            scale = max(1.0, float(zipf.count[zipf.column(j)].sum()))
            assert abs(g - go) <= 1e-12 * scale, (j, g, go)
            assert abs(hh - ho) <= 1e-11 * abs(ho), (j, hh, ho)


def test_relabelled_warm_start_and_mixed_precision(sccs, zipf):
    beta0 = synth.random_beta(zipf.n_cols, 0.2, 3)
    _, ref_beta, _, _ = oracle_relabelled(zipf, 1, 1.0, 5, beta0=beta0)
    with sccs.Handle(zipf, precision=sccs.PREC_MIXED, column_order=IND) as h:
        h.set_prior(sccs.PRIOR_NORMAL, 1.0)
        h.set_beta(beta0)
        h.sweep(5)
        beta, _ = h.get_beta()
    assert rel_inf(beta, ref_beta) <= 1e-6


def test_relabelled_covariate_values(sccs):
    prob = synth.valued(n_patients=6000, n_drugs=40, n_dose=6, n_dense=2, seed=0)
    _, ref_beta, _, _ = oracle_relabelled(prob, 2, 1.0, 6)
    with sccs.Handle(prob, column_order=IND) as h:
        h.set_prior(sccs.PRIOR_LAPLACE, 1.0)
        h.sweep(6)
        beta, _ = h.get_beta()
    assert rel_inf(beta, ref_beta) <= FP64_TOL
    assert np.array_equal(beta == 0.0, ref_beta == 0.0)


def test_relabelled_grouped_prior(sccs, zipf):
    class_of = np.random.default_rng(4).integers(0, 9, size=zipf.n_cols).astype(np.int32)
    order = oracle.independent_order(zipf, 4)
    ref = oracle.ccd_grouped(synth.permute_columns(zipf, order), 0.3, class_of[order], 0.7, 6)
    with sccs.Handle(zipf, column_order=IND) as h:
        h.set_prior_grouped(0.3, 0.7, class_of)
        h.sweep(6)
        beta, _ = h.get_beta()
    assert rel_inf(beta, unpermute(ref["beta"], order)) <= FP64_TOL


def test_relabelled_batch_cv_chain(sccs):
    """Partitioned batched engine: 5 folds walking a 3-value Laplace path with
    warm starts, beta and held-out log-likelihood per link."""
    prob = synth.zipf_problem("cvorder", 8000, 60, 0.1, seed_path=(9, 33))
    folds = synth.cv_folds(prob.n_patients, 5, seed=3)
    grid = [0.05, 0.5, 5.0]
    specs = [sccs.FitSpec(0, [(sccs.PRIOR_LAPLACE, v) for v in grid], weight=(folds != k).astype(np.int32))
             for k in range(5)]
    with sccs.Batch([prob], specs, column_order=IND) as b:
        b.run(sccs.CRIT_FIXED, max_sweeps=3)
        for k in range(5):
            w = (folds != k).astype(np.int32)
            beta = np.zeros(prob.n_cols)
            for l, v in enumerate(grid):
                _, beta, _, _ = oracle_relabelled(prob, oracle.PRIOR_LAPLACE, v, 3, weight=w, beta0=beta)
                got, res = b.get(k, l)
                assert res["sweeps"] == 3
                assert rel_inf(got, beta) <= FP64_TOL, (k, l)
                ho = oracle.loglik(prob, beta, weight=(folds == k).astype(np.int32))
                assert abs(b.heldout(k, l) - ho) <= 1e-8 * abs(ho), (k, l)


def test_lockstep_engine_takes_the_given_order_only(sccs, zipf):
    with pytest.raises(sccs.SccsError):
        sccs.Batch([zipf], [sccs.FitSpec(0, [(sccs.PRIOR_NORMAL, 1.0)])], engine=1, column_order=IND)


def test_mid_twenty_sweeps_relabelled(sccs):
    """The mid workload's benchmark schedule under the relabelling: 5 warm-up
    sweeps, reset to beta = 0, sweeps 1..20 one launch each on 128
    workgroups, against the oracle's iterates written by
    tests/golden/make_mid_golden.py."""
    mid = synth.mid()
    g = np.load(os.path.join(HERE, "golden", "mid_laplace_fp64_independent.npz"))
    assert str(g["seed_info"]) == mid.seed_info and int(g["nnz"]) == mid.nnz
    with sccs.Handle(mid, n_workgroups=128, column_order=IND) as h:
        assert np.array_equal(h.column_order(), g["order"])
        h.set_prior(sccs.PRIOR_LAPLACE, 2.0)
        for _ in range(5):
            h.sweep(1)
        h.set_beta(np.zeros(mid.n_cols))
        for _ in range(20):
            h.sweep(1)
        beta, trust = h.get_beta()
    ref = g["beta20"]
    err = rel_inf(beta, ref)
    big = np.abs(ref) >= 1e-3
    coord = float(np.max(np.abs(beta[big] - ref[big]) / np.abs(ref[big])))
    print(f"mid relabelled: rel_inf {err:.2e}, per-coordinate {coord:.2e}")
    assert err <= FP64_TOL and coord <= 1e-6
    assert np.array_equal(beta == 0.0, ref == 0.0)
    assert np.max(np.abs(trust - g["trust20"])) <= 1e-9 * np.max(g["trust20"])
