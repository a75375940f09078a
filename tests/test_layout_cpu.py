"""Host layout builder (ownership ranges, patient-aligned tiles, index pairs
and the row-compressed copy of X) against brute force, no GPU needed."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1208_0945_amd import sccs, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1208_0945_amd", "csrc")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("layout") / "liblayout_probe.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-I", os.path.join(ROOT, "include"),
                    "-I", CSRC, os.path.join(ROOT, "tests", "layout_probe.cpp"),
                    os.path.join(CSRC, "sccs_layout.cpp"), "-o", out], check=True)
    lib = ctypes.CDLL(out)
    lib.layout_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int] + [ctypes.c_void_p] * 11
    lib.ytx_probe.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    return lib


def run(probe, prob, G, tile_nnz, max_group=1, gdesc=None):
    P = sccs.ProblemArrays(prob)
    K, N, J, nnz = prob.n_rows, prob.n_patients, prob.n_cols, prob.nnz
    pb = np.zeros(G + 1, np.int32)
    rp = np.zeros(2 * max(nnz, 1), np.uint32)
    own = np.zeros(J * (G + 1), np.int32)
    era_ptr = np.zeros(K + 1, np.int32)
    era_col = np.zeros(max(nnz, 1), np.int32)
    gcol = np.zeros(J + 1, np.int32)
    nt, bound, ng = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
    ts = np.zeros(2 * nnz // tile_nnz + 2 * min(nnz, J * G) + 4, np.int32)
    rc = probe.layout_probe(ctypes.addressof(P.s), G, tile_nnz, max_group, pb.ctypes.data, rp.ctypes.data,
                            ts.ctypes.data, ctypes.byref(nt), own.ctypes.data, era_ptr.ctypes.data,
                            era_col.ctypes.data, ctypes.byref(bound), gcol.ctypes.data, ctypes.byref(ng),
                            None if gdesc is None else gdesc.ctypes.data)
    assert rc == 0
    n_groups = ng.value
    if max_group == 1:
        return pb, rp.reshape(-1, 2)[:nnz], ts[:nt.value + 1], own.reshape(J, G + 1), era_ptr, era_col[:nnz], bound.value
    return (pb, rp.reshape(-1, 2)[:nnz], ts[:nt.value + 1], own[:n_groups * (G + 1)].reshape(n_groups, G + 1),
            bound.value, gcol[:n_groups + 1])


@pytest.mark.parametrize("G,tile_nnz", [(1, 64), (7, 64), (64, 32), (256, 16)])
def test_layout_matches_brute_force(probe, G, tile_nnz):
    prob = synth.zipf_problem("lay", 3000, 40, 0.3, seed_path=(11, G))
    pb, rp, ts, own, era_ptr, era_col, bound = run(probe, prob, G, tile_nnz)
    N, J, nnz = prob.n_patients, prob.n_cols, prob.nnz
    era_pid = np.repeat(np.arange(N), np.diff(prob.patient_ptr))
    # index pairs
    assert np.array_equal(rp[:, 0], prob.row_idx)
    assert np.array_equal(rp[:, 1], era_pid[prob.row_idx])
    # ownership: monotone ranges covering all patients
    assert pb[0] == 0 and pb[-1] == N and np.all(np.diff(pb) >= 0)
    owner = np.searchsorted(pb, np.arange(N), side="right") - 1
    # tiles partition [0, nnz) in order, within (column, workgroup) ranges
    assert ts[0] == 0 and ts[-1] == nnz and np.all(np.diff(ts) > 0)
    assert len(ts) - 1 < bound
    for j in range(J):
        lo, hi = prob.col_ptr[j], prob.col_ptr[j + 1]
        assert own[j, 0] == np.searchsorted(ts, lo) or lo == hi
        for b in range(G):
            for t in range(own[j, b], own[j, b + 1]):
                e0, e1 = ts[t], ts[t + 1]
                assert lo <= e0 < e1 <= hi
                pids = rp[e0:e1, 1]
                assert np.all(owner[pids] == b)
                # whole patient segments: no patient continues across a tile edge
                if e0 > lo:
                    assert rp[e0 - 1, 1] != rp[e0, 1] or owner[rp[e0 - 1, 1]] != b
                if e1 - e0 > tile_nnz:
                    assert np.all(pids == pids[0])
        assert own[j, G] == (own[j + 1, 0] if j + 1 < J else len(ts) - 1)
    # compressed row storage
    X = np.zeros((prob.n_rows, J), bool)
    for j in range(J):
        X[prob.column(j), j] = True
    assert np.array_equal(np.diff(era_ptr), X.sum(axis=1))
    for k in range(0, prob.n_rows, 97):
        assert np.array_equal(era_col[era_ptr[k]:era_ptr[k + 1]], np.flatnonzero(X[k]))


def test_long_patient_segment_gets_own_tile(probe):
    # one patient with 150 eras all in column 0, plus a few small patients
    sizes = [150, 3, 2, 4]
    ptr = np.concatenate([[0], np.cumsum(sizes)])
    K = int(ptr[-1])
    prob = synth.Problem("long", len(sizes), ptr.astype(np.int64), np.full(K, 10, np.int32),
                         np.ones(K, np.int32), 1, np.array([0, K], np.int64), np.arange(K, dtype=np.int32),
                         np.zeros(1))
    pb, rp, ts, own, *_ = run(probe, prob, 1, 64)
    lens = np.diff(ts)
    assert lens[0] == 150 and np.all(lens[1:] <= 64)


@pytest.mark.parametrize("G,tile_nnz,max_group", [(1, 64, 4), (7, 32, 4), (64, 16, 2), (256, 64, 4)])
def test_grouped_layout(probe, G, tile_nnz, max_group):
    """Column groups: greedy maximal runs of pairwise patient-disjoint
    columns (at most max_group); the group order of the index pairs; tiles
    within (group, workgroup) blocks holding whole (column, patient)
    segments."""
    prob = synth.zipf_problem("grp", 4000, 60, 0.02, seed_path=(11, 100 + G))
    pb, rp, ts, own, bound, gcol = run(probe, prob, G, tile_nnz, max_group)
    N, J, nnz = prob.n_patients, prob.n_cols, prob.nnz
    era_pid = np.repeat(np.arange(N), np.diff(prob.patient_ptr))
    pats = [set(era_pid[prob.column(j)].tolist()) for j in range(J)]
    # groups: ordered cover of the columns, disjoint inside, maximal
    assert gcol[0] == 0 and gcol[-1] == J and np.all(np.diff(gcol) >= 1) and np.all(np.diff(gcol) <= max_group)
    for g in range(len(gcol) - 1):
        seen = set()
        for j in range(gcol[g], gcol[g + 1]):
            assert not (seen & pats[j]), (g, j)
            seen |= pats[j]
        if gcol[g + 1] < J and gcol[g + 1] - gcol[g] < max_group:
            assert seen & pats[gcol[g + 1]], "a group ended although the next column was disjoint"
    assert len(gcol) - 1 < J, "the synthetic problem should have some disjoint neighbours"
    # index pairs: group order, then workgroup, then column, then CSC order
    owner = np.searchsorted(pb, np.arange(N), side="right") - 1
    expect = []
    for g in range(len(gcol) - 1):
        for b in range(G):
            for c, j in enumerate(range(gcol[g], gcol[g + 1])):
                rows = prob.column(j)
                rows = rows[owner[era_pid[rows]] == b]
                expect.extend((int(r), int(era_pid[r]) | (c << 28)) for r in rows)
    assert np.array_equal(rp, np.array(expect, dtype=np.uint32).reshape(-1, 2))
    # tiles
    assert ts[0] == 0 and ts[-1] == nnz and np.all(np.diff(ts) > 0) and len(ts) - 1 < bound
    pos = 0
    for g in range(len(gcol) - 1):
        for b in range(G):
            n = sum(int(np.sum(owner[era_pid[prob.column(j)]] == b)) for j in range(gcol[g], gcol[g + 1]))
            t0, t1 = own[g, b], own[g, b + 1]
            if n == 0:
                assert t0 == t1
                continue
            assert ts[t0] == pos and ts[t1] == pos + n
            for t in range(t0, t1):
                e0, e1 = ts[t], ts[t + 1]
                keys = rp[e0:e1, 1]
                if e1 - e0 > tile_nnz:
                    assert np.all(keys == keys[0])
                if e0 > pos:
                    assert rp[e0 - 1, 1] != rp[e0, 1]
            pos += n


def test_host_ytx(probe):
    prob = synth.zipf_problem("ytx", 2000, 25, 0.1, seed_path=(11, 7))
    w = (np.arange(prob.n_patients) % 3).astype(np.int32)
    P = sccs.ProblemArrays(prob, w)
    out = np.zeros(prob.n_cols)
    probe.ytx_probe(ctypes.addressof(P.s), out.ctypes.data)
    era_pid = np.repeat(np.arange(prob.n_patients), np.diff(prob.patient_ptr))
    for j in range(prob.n_cols):
        rows = prob.column(j)
        assert out[j] == float(np.sum(w[era_pid[rows]] * prob.count[rows]))


@pytest.mark.parametrize("max_group", [1, 2, 4])
def test_pass_descriptors(probe, max_group):
    """Pass descriptors: first column and width of each group, and the mask
    of the L columns just before the group that share a patient with it
    (bit i for column j0 - L + i; L = columns per merged pass - 1) --
    against sets of patients."""
    prob = synth.zipf_problem("desc", 3000, 70, 0.03, seed_path=(11, 200 + max_group))
    J = prob.n_cols
    gdesc = np.zeros(J, np.uint32)
    pb, rp, ts, own, *rest = run(probe, prob, 16, 64, max_group, gdesc=gdesc)
    gcol = np.arange(J + 1) if max_group == 1 else rest[-1]
    NG = len(gcol) - 1
    era_pid = np.repeat(np.arange(prob.n_patients), np.diff(prob.patient_ptr))
    pats = [set(era_pid[prob.column(j)].tolist()) for j in range(J)]
    L = probe.link_cols()
    assert 1 <= L <= 7
    n_linked = n_window = 0
    for g in range(NG):
        d = int(gdesc[g])
        j0 = gcol[g]
        assert d & 0x1FFF == j0
        assert (d >> 13) & 7 == gcol[g + 1] - j0
        mine = set().union(*(pats[j] for j in range(j0, gcol[g + 1])))
        mask = sum(1 << i for i in range(L) if j0 - L + i >= 0 and pats[j0 - L + i] & mine)
        assert (d >> 16) & ((1 << L) - 1) == mask, g
        assert d >> (16 + L) == 0
        n_linked += bin(mask).count("1")
        n_window += min(L, j0)
    assert 0 < n_linked < n_window, "both linked and independent columns should occur"
