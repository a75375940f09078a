"""The allocation-free sweep (sccs_sweep_static) against sccs_sweep.

sccs_sweep_static runs the same kernels as sccs_sweep with the reduction
slots and control block in the library's static device array, so its results
must equal sccs_sweep's bit for bit: two calls in a row on different problems
(the second smaller), a handle that alternates both entry points, and the
mixed-precision form, whose exact refresh count passes through the static
control block.  The FP64 results are also checked against the oracle.
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


def _run(sccs, prob, kind, var, plan, **kw):
    """plan: list of ("s" | "t", n_sweeps) = sccs_sweep / sccs_sweep_static."""
    out = []
    with sccs.Handle(prob, **kw) as h:
        h.set_prior(kind, var)
        for which, n in plan:
            lp = (h.sweep_static if which == "t" else h.sweep)(n, want_logpost=True)
            out.append((lp, h.pass_stats()))
        beta, trust = h.get_beta()
    return beta, trust, out


def test_two_calls_in_a_row_second_smaller(sccs):
    big = synth.zipf_problem("zipf_small", 20000, 300, 0.1, seed_path=(8, 0))
    small = synth.tiny(n_patients=300, n_cols=12, seed=3)
    assert small.n_patients < big.n_patients and small.nnz < big.nnz
    for prob, kind, var, n in ((big, sccs.PRIOR_LAPLACE, 2.0, 4), (small, sccs.PRIOR_NORMAL, 1.0, 3)):
        b_t, t_t, o_t = _run(sccs, prob, kind, var, [("t", n)])
        b_s, t_s, o_s = _run(sccs, prob, kind, var, [("s", n)])
        assert np.array_equal(b_t, b_s) and np.array_equal(t_t, t_s)
        assert o_t == o_s
        ref = oracle.ccd(prob, kind, var, n)["beta"]
        err = float(np.max(np.abs(b_t - ref)) / max(np.max(np.abs(ref)), 1e-300))
        print(f"{prob.name}: {n} sweeps, passes {o_t[0][1]}, rel error vs oracle {err:.2e}")
        assert err <= 1e-9


def test_alternating_entry_points_keep_the_handle_consistent(sccs):
    prob = synth.zipf_problem("zipf_small", 20000, 300, 0.1, seed_path=(8, 0))
    plan = [("t", 3), ("s", 2), ("t", 1), ("t", 1), ("s", 1), ("t", 2)]
    b_t, t_t, o_t = _run(sccs, prob, sccs.PRIOR_LAPLACE, 2.0, plan, n_workgroups=128)
    b_s, t_s, o_s = _run(sccs, prob, sccs.PRIOR_LAPLACE, 2.0, [("s", n) for _, n in plan], n_workgroups=128)
    assert np.array_equal(b_t, b_s) and np.array_equal(t_t, t_s)
    assert [lp for lp, _ in o_t] == [lp for lp, _ in o_s]
    assert [st for _, st in o_t] == [st for _, st in o_s]


def test_mixed_precision_with_refresh(sccs):
    prob = synth.zipf_problem("zipf_small", 20000, 300, 0.1, seed_path=(8, 0))
    plan = [("t", 2), ("t", 2)]
    b_t, _, o_t = _run(sccs, prob, sccs.PRIOR_NORMAL, 0.5, plan, precision=1, refresh_period=3)
    b_s, _, o_s = _run(sccs, prob, sccs.PRIOR_NORMAL, 0.5, [("s", 2), ("s", 2)], precision=1, refresh_period=3)
    assert np.array_equal(b_t, b_s)
    assert o_t == o_s


def test_static_sweep_argument_errors(sccs):
    prob = synth.tiny(n_patients=100, n_cols=5, seed=4)
    with sccs.Handle(prob) as h:
        with pytest.raises(sccs.SccsError) as e:
            h.sweep_static(1)
        assert e.value.status == sccs.ERR_STATE          # no prior yet
        h.set_prior(sccs.PRIOR_NORMAL, 1.0)
        with pytest.raises(sccs.SccsError) as e:
            h.sweep_static(0)
        assert e.value.status == sccs.ERR_INVALID_ARG
