"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/sccs.h declares, and rejects malformed problems and
options before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1208_0945_amd import sccs, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sccs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sccs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    sccs.lib()                       # binds to torch's HIP runtime first
    lib = ctypes.CDLL(sccs.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sccs.EXPORTS)


def test_single_hip_runtime_loaded():
    sccs.lib()
    assert len(sccs._hip_runtimes_mapped()) == 1


def test_last_error_never_null():
    assert isinstance(sccs.lib().sccs_last_error(None), bytes)


def test_default_options():
    o = sccs.options()
    assert o.precision == sccs.PREC_FP64 and o.refresh_period == -1 and o.tile_nnz == 0


def _tiny():
    return synth.tiny(n_patients=50, n_cols=4, seed=1)


def _query(prob, weight=None, n_rows=None, nnz=None, **opt):
    P = sccs.ProblemArrays(prob, weight)
    if n_rows is not None:
        P.s.n_rows = n_rows
    if nnz is not None:
        P.s.nnz = nnz
    o = sccs.options(**opt)
    n = ctypes.c_size_t()
    return sccs.lib().sccs_query_workspace(ctypes.byref(P.s), ctypes.byref(o), ctypes.byref(n))


@pytest.mark.parametrize("case", ["ptr_decreasing", "ptr_end", "row_range", "row_dup", "row_order",
                                  "neg_count", "event_no_time", "neg_len", "colptr_end"])
def test_invalid_problems_rejected(case):
    p = _tiny()
    if case == "ptr_decreasing":
        pp = p.patient_ptr.copy(); pp[5], pp[6] = pp[6], pp[5]
        if pp[5] == pp[6]:
            pp[5] += 1
        p.patient_ptr = pp
    elif case == "ptr_end":
        assert _query(p, n_rows=p.n_rows + 1) == sccs.ERR_INVALID_ARG
        return
    elif case == "row_range":
        r = p.row_idx.copy(); r[-1] = p.n_rows; p.row_idx = r
    elif case == "row_dup":
        r = p.row_idx.copy(); r[1] = r[0]; p.row_idx = r
    elif case == "row_order":
        r = p.row_idx.copy(); r[0], r[1] = r[1], r[0]; p.row_idx = r
    elif case == "neg_count":
        c = p.count.copy(); c[3] = -1; p.count = c
    elif case == "event_no_time":
        c = p.count.copy(); o = p.offset.copy(); c[2] = 1; o[2] = 0; p.count, p.offset = c, o
    elif case == "neg_len":
        o = p.offset.copy(); o[4] = -3; p.offset = o
    elif case == "colptr_end":
        assert _query(p, nnz=p.nnz - 1) == sccs.ERR_INVALID_ARG
        return
    assert _query(p) == sccs.ERR_INVALID_ARG
    assert len(sccs.lib().sccs_last_error(None)) > 0


def test_negative_weight_rejected():
    p = _tiny()
    w = np.ones(p.n_patients, np.int32); w[7] = -1
    assert _query(p, weight=w) == sccs.ERR_INVALID_ARG


@pytest.mark.parametrize("opt", [{"precision": 2}, {"n_workgroups": -1}, {"n_workgroups": 4096},
                                 {"refresh_period": -2}, {"tile_nnz": 4}, {"tile_nnz": 65}])
def test_invalid_options_rejected(opt):
    assert _query(_tiny(), **opt) == sccs.ERR_INVALID_ARG


def test_null_arguments_rejected():
    L = sccs.lib()
    n = ctypes.c_size_t()
    assert L.sccs_query_workspace(None, None, ctypes.byref(n)) == sccs.ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert L.sccs_create(None, None, None, 0, ctypes.byref(h)) == sccs.ERR_INVALID_ARG
    assert L.sccs_destroy(None) == sccs.OK
    assert L.sccs_set_prior(None, 1, 1.0) == sccs.ERR_INVALID_ARG
    assert L.sccs_sweep(None, 1, None) == sccs.ERR_INVALID_ARG
    assert L.sccs_group_timing(None, 1) == sccs.ERR_INVALID_ARG


def _batch_query(probs, specs, **opt):
    parr = (sccs.Problem_ * len(probs))(*[sccs.ProblemArrays(p).s for p in probs])
    keep = [sccs.ProblemArrays(p) for p in probs]
    parr = (sccs.Problem_ * len(keep))(*[k.s for k in keep])
    sarr = (sccs.FitSpec_ * len(specs))(*[s.struct() for s in specs])
    n = ctypes.c_size_t()
    o = sccs.options(**opt)
    return sccs.lib().sccs_batch_query_workspace(ctypes.addressof(parr), len(keep), ctypes.addressof(sarr),
                                                 len(specs), ctypes.byref(o), ctypes.byref(n))


def test_batch_specs_validated_on_host():
    p = _tiny()
    ok_link = [(sccs.PRIOR_NORMAL, 1.0)]
    assert _batch_query([p], [sccs.FitSpec(1, ok_link)]) == sccs.ERR_INVALID_ARG       # bad problem index
    assert _batch_query([p], [sccs.FitSpec(0, [(sccs.PRIOR_LAPLACE, 0.0)])]) == sccs.ERR_INVALID_ARG
    assert _batch_query([p], [sccs.FitSpec(0, [(7, 1.0)])]) == sccs.ERR_INVALID_ARG
    assert _batch_query([p], [sccs.FitSpec(0, [])]) == sccs.ERR_INVALID_ARG
    w = np.ones(p.n_patients, np.int32); w[0] = -2
    assert _batch_query([p], [sccs.FitSpec(0, ok_link, weight=w)]) == sccs.ERR_INVALID_ARG
    other = synth.tiny(n_patients=30, n_cols=5, seed=2)
    assert _batch_query([p, other], [sccs.FitSpec(0, ok_link)]) == sccs.ERR_INVALID_ARG  # J differs
    assert _batch_query([p], [sccs.FitSpec(0, ok_link)] * 65) == sccs.ERR_INVALID_ARG    # > 64 fits


def test_covariate_values_must_be_finite():
    prob = synth.valued(n_patients=60, n_drugs=3, n_dose=1, n_dense=1, seed=1)
    assert _query(prob) != sccs.ERR_INVALID_ARG      # valid (ERR_HIP without a GPU)
    bad = prob.value.copy()
    bad[5] = np.nan
    import dataclasses
    assert _query(dataclasses.replace(prob, value=bad)) == sccs.ERR_INVALID_ARG
