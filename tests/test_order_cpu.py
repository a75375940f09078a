"""The independence relabelling of the columns, on the CPU.

Algorithm 1 visits the coordinates in a fixed cyclic order and leaves the
numbering of the drugs free.  The library can renumber them so that runs of
consecutive columns share no patient (SCCS_ORDER_INDEPENDENT); the oracle's
restatement of that rule (oracle.independent_groups) is pinned here by a
hand-worked example and by the properties the rule implies, checked by brute
force, and the library's sccs_column_order (host code, no GPU needed) must
return exactly the oracle's order.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1208_0945_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def example_problem():
    with open(os.path.join(HERE, "golden", "relabel_example.json")) as f:
        ex = json.load(f)
    ptr = np.array(ex["patient_ptr"], dtype=np.int64)
    cols = ex["columns"]
    col_ptr = np.zeros(len(cols) + 1, dtype=np.int64)
    col_ptr[1:] = np.cumsum([len(c) for c in cols])
    K = int(ptr[-1])
    prob = synth.Problem(name="relabel_example", n_patients=len(ptr) - 1, patient_ptr=ptr,
                         offset=np.ones(K, dtype=np.int32), count=np.ones(K, dtype=np.int32),
                         n_cols=len(cols), col_ptr=col_ptr,
                         row_idx=np.array([r for c in cols for r in c], dtype=np.int32),
                         beta_true=np.zeros(len(cols)))
    return prob, ex["expected"]


def patient_sets(prob):
    pid = np.repeat(np.arange(prob.n_patients), np.diff(prob.patient_ptr))
    return [set(pid[prob.column(j)].tolist()) for j in range(prob.n_cols)]


def problems():
    return [synth.tiny(n_patients=300, n_cols=12, seed=3),
            synth.zipf_problem("zo", 4000, 50, 0.1, seed_path=(9, 21)),
            synth.zipf_problem("zo2", 3000, 80, 0.02, seed_path=(9, 22)),
            synth.valued(n_patients=800, n_drugs=20, seed=4)]


@pytest.mark.parametrize("width", [1, 2, 4])
def test_hand_worked_example(width):
    prob, expected = example_problem()
    assert oracle.independent_groups(prob, width) == expected[str(width)]["groups"]


@pytest.mark.parametrize("width", [1, 2, 3, 4])
def test_relabelling_properties_by_brute_force(width):
    """A permutation; groups of at most `width` pairwise patient-disjoint
    columns; every column's group is the earliest one that could take it at
    the end (each earlier group is full or shares a patient with it, the
    end-state form of joining the earliest-opened fitting group); columns in
    decreasing nonzeros within a group and by group leader."""
    for prob in problems():
        groups = oracle.independent_groups(prob, width)
        order = oracle.independent_order(prob, width)
        assert sorted(order.tolist()) == list(range(prob.n_cols))
        sets = patient_sets(prob)
        nnz = np.diff(prob.col_ptr)
        for gi, g in enumerate(groups):
            assert 1 <= len(g) <= width
            for a in range(len(g)):
                for b in range(a + 1, len(g)):
                    assert not (sets[g[a]] & sets[g[b]]), (prob.name, gi)
            key = [(-int(nnz[j]), j) for j in g]
            assert key == sorted(key)
            for j in g:
                for earlier in groups[:gi]:
                    assert len(earlier) == width or any(sets[j] & sets[k] for k in earlier), (prob.name, j)
        leaders = [(-int(nnz[g[0]]), g[0]) for g in groups]
        assert leaders == sorted(leaders)


def test_consecutive_runs_of_the_relabelled_problem_are_the_groups():
    """Cutting the relabelled columns greedily into runs of pairwise
    patient-disjoint columns (at most 4) gives back exactly the groups: the
    sweep then needs one device-wide reduction per group."""
    for prob in problems():
        groups = oracle.independent_groups(prob, 4)
        perm = synth.permute_columns(prob, oracle.independent_order(prob, 4))
        sets = patient_sets(perm)
        runs, cur, seen = [], [], set()
        for k in range(perm.n_cols):
            if cur and (len(cur) == 4 or sets[k] & seen):
                runs.append(cur)
                cur, seen = [], set()
            cur.append(k)
            seen |= sets[k]
        runs.append(cur)
        assert [len(r) for r in runs] == [len(g) for g in groups]


def test_permute_columns_moves_whole_columns():
    prob = synth.valued(n_patients=200, n_drugs=6, seed=2)
    order = np.array(list(reversed(range(prob.n_cols))))
    perm = synth.permute_columns(prob, order)
    for k, j in enumerate(order):
        assert np.array_equal(perm.column(k), prob.column(j))
        assert np.array_equal(perm.value[perm.col_ptr[k]:perm.col_ptr[k + 1]],
                              prob.value[prob.col_ptr[j]:prob.col_ptr[j + 1]])


@pytest.fixture(scope="module")
def sccs():
    from paper_1208_0945_amd import sccs as s
    try:
        s.lib()
    except OSError as e:
        pytest.skip(f"libsccs not built: {e}")
    return s


@pytest.mark.parametrize("width", [1, 2, 3, 4])
def test_library_order_equals_oracle_order(sccs, width):
    prob, _ = example_problem()
    for p in [prob] + problems():
        assert np.array_equal(sccs.column_order(p, width), oracle.independent_order(p, width)), (p.name, width)


def test_library_order_rejects_bad_width(sccs):
    prob, _ = example_problem()
    for w in (0, 5):
        with pytest.raises(sccs.SccsError):
            sccs.column_order(prob, w)
