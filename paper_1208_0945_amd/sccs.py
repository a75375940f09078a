"""Thin ctypes binding of libsccs (include/sccs.h).

Argument marshalling only: every step of the CCD path runs in the HIP
library.  PyTorch provides the device workspace and the stream.  The binding
raises if ``libsccs.so`` has not been built -- there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsccs.so")

OK, NOT_CONVERGED = 0, 1
ERR_INVALID_ARG, ERR_WORKSPACE, ERR_HIP, ERR_STATE, ERR_NUMERIC, ERR_SYNC = -1, -2, -3, -4, -5, -6
PRIOR_NONE, PRIOR_NORMAL, PRIOR_LAPLACE, PRIOR_GROUPED = 0, 1, 2, 3
PREC_FP64, PREC_MIXED = 0, 1
CRIT_FIXED, CRIT_REL_LOGPOST, CRIT_ABS_DXBETA = 0, 1, 2
ORDER_GIVEN, ORDER_INDEPENDENT = 0, 1

EXPORTS = ("sccs_default_options", "sccs_query_workspace", "sccs_create", "sccs_destroy",
           "sccs_set_prior", "sccs_set_beta", "sccs_get_beta", "sccs_sweep", "sccs_fit",
           "sccs_grad_hess", "sccs_objective", "sccs_last_kernel_ms", "sccs_pass_stats", "sccs_last_error",
           "sccs_batch_query_workspace", "sccs_batch_create", "sccs_batch_run", "sccs_batch_get",
           "sccs_batch_heldout", "sccs_batch_last_kernel_ms", "sccs_batch_destroy", "sccs_batch_last_error", "sccs_tune",
           "sccs_sweep_static", "sccs_bootstrap_query_workspace", "sccs_bootstrap",
           "sccs_cv_query_workspace", "sccs_cv_search", "sccs_set_prior_grouped", "sccs_group_timing", "sccs_group_times",
           "sccs_batch_tune", "sccs_column_order", "sccs_get_column_order")


class SccsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libsccs status {status}: {msg}")
        self.status = status


class Problem_(ctypes.Structure):
    _fields_ = [("n_patients", ctypes.c_int32), ("n_rows", ctypes.c_int64),
                ("n_cols", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("patient_ptr", ctypes.c_void_p), ("offset", ctypes.c_void_p),
                ("count", ctypes.c_void_p), ("col_ptr", ctypes.c_void_p),
                ("row_idx", ctypes.c_void_p), ("patient_weight", ctypes.c_void_p),
                ("value", ctypes.c_void_p)]


class Options_(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("n_workgroups", ctypes.c_int32),
                ("refresh_period", ctypes.c_int32), ("tile_nnz", ctypes.c_int32),
                ("max_group", ctypes.c_int32), ("merge_passes", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("batch_engine", ctypes.c_int32),
                ("column_order", ctypes.c_int32)]


class FitOpts_(ctypes.Structure):
    _fields_ = [("criterion", ctypes.c_int32), ("max_sweeps", ctypes.c_int32), ("tol", ctypes.c_double)]


class FitSpec_(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int32), ("n_links", ctypes.c_int32),
                ("prior_kind", ctypes.c_void_p), ("variance", ctypes.c_void_p),
                ("patient_weight", ctypes.c_void_p)]


class TuneResult_(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int32), ("best", ctypes.c_int32),
                ("n_workgroups", ctypes.c_int32 * 16), ("tile_nnz", ctypes.c_int32 * 16),
                ("ms_per_sweep", ctypes.c_double * 16)]


class BootstrapOut_(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_void_p), ("ci_lo", ctypes.c_void_p), ("ci_hi", ctypes.c_void_p),
                ("p_nonzero", ctypes.c_void_p), ("sweeps", ctypes.c_void_p), ("converged", ctypes.c_void_p)]


class CvOpts_(ctypes.Structure):
    _fields_ = [("prior_kind", ctypes.c_int32), ("n_folds", ctypes.c_int32), ("fold", ctypes.c_void_p),
                ("var_start", ctypes.c_double), ("bracket_step", ctypes.c_double), ("log10_tol", ctypes.c_double),
                ("max_evals", ctypes.c_int32), ("warm_start", ctypes.c_int32), ("fit", FitOpts_)]


class CvResult_(ctypes.Structure):
    _fields_ = [("n_evals", ctypes.c_int32), ("best", ctypes.c_int32), ("bracketed", ctypes.c_int32),
                ("variance", ctypes.c_double * 64), ("pred_loglik", ctypes.c_double * 64)]


class FitResult_(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("loglik", ctypes.c_double), ("logpost", ctypes.c_double)]


_lib = None

# Handles and batches still open when the interpreter exits are destroyed by
# an atexit hook, i.e. before the C-level exit handlers (HIP's own teardown,
# and a profiler's, if one is attached) run; a destructor that runs later,
# during interpreter finalisation, makes no HIP call at all.
_live = weakref.WeakSet()


def _close_live():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


atexit.register(_close_live)


def _hip_runtimes_mapped():
    try:
        with open("/proc/self/maps") as f:
            return sorted({l.split()[-1] for l in f if "libamdhip64" in l})
    except OSError:
        return []


def lib() -> ctypes.CDLL:
    """Open libsccs.so; raises if it has not been built.

    torch is imported first so that the library binds to the HIP runtime
    torch already uses: its streams and device memory are handed to the
    library, which is only valid within one runtime."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built; run python -m paper_1208_0945_amd.build")
        import torch  # noqa: F401  (loads torch's HIP runtime first)
        L = ctypes.CDLL(LIB_PATH)
        maps = _hip_runtimes_mapped()
        if len(maps) > 1:
            raise RuntimeError(f"two HIP runtimes are loaded ({maps}); import torch before libsccs")
        H = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.sccs_default_options.argtypes = [ctypes.POINTER(Options_)]
        L.sccs_default_options.restype = None
        L.sccs_query_workspace.argtypes = [ctypes.POINTER(Problem_), ctypes.POINTER(Options_),
                                           ctypes.POINTER(ctypes.c_size_t)]
        L.sccs_create.argtypes = [ctypes.POINTER(Problem_), ctypes.POINTER(Options_), ctypes.c_void_p,
                                  ctypes.c_size_t, ctypes.POINTER(H)]
        L.sccs_destroy.argtypes = [H]
        L.sccs_set_prior.argtypes = [H, ctypes.c_int32, ctypes.c_double]
        L.sccs_set_prior_grouped.argtypes = [H, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p]
        L.sccs_set_beta.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p]
        L.sccs_get_beta.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p]
        L.sccs_sweep.argtypes = [H, ctypes.c_int32, dp]
        L.sccs_sweep_static.argtypes = [H, ctypes.c_int32, dp]
        L.sccs_fit.argtypes = [H, ctypes.POINTER(FitOpts_), ctypes.POINTER(FitResult_)]
        L.sccs_grad_hess.argtypes = [H, ctypes.c_int32, dp, dp]
        L.sccs_objective.argtypes = [H, dp, dp]
        L.sccs_last_kernel_ms.argtypes = [H, dp]
        ip = ctypes.POINTER(ctypes.c_int32)
        L.sccs_pass_stats.argtypes = [H, ip, ip, ip]
        L.sccs_group_timing.argtypes = [H, ctypes.c_int32]
        L.sccs_group_times.argtypes = [H, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ip]
        L.sccs_last_error.argtypes = [H]
        L.sccs_last_error.restype = ctypes.c_char_p
        L.sccs_batch_query_workspace.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                                 ctypes.POINTER(Options_), ctypes.POINTER(ctypes.c_size_t)]
        L.sccs_batch_create.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.POINTER(Options_), ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(H)]
        L.sccs_batch_run.argtypes = [H, ctypes.POINTER(FitOpts_)]
        L.sccs_batch_get.argtypes = [H, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(FitResult_)]
        L.sccs_batch_heldout.argtypes = [H, ctypes.c_int32, ctypes.c_int32, dp]
        L.sccs_batch_last_kernel_ms.argtypes = [H, dp]
        L.sccs_batch_destroy.argtypes = [H]
        L.sccs_tune.argtypes = [ctypes.POINTER(Problem_), ctypes.POINTER(Options_), ctypes.c_int32, ctypes.c_double,
                                ctypes.c_int32, ctypes.POINTER(Options_), ctypes.POINTER(TuneResult_)]
        L.sccs_batch_last_error.argtypes = [H]
        L.sccs_batch_last_error.restype = ctypes.c_char_p
        L.sccs_batch_tune.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.POINTER(Options_), ctypes.c_int32, ctypes.POINTER(Options_),
                                      ctypes.POINTER(TuneResult_)]
        L.sccs_bootstrap_query_workspace.argtypes = [ctypes.POINTER(Problem_), ctypes.POINTER(Options_),
                                                     ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.sccs_bootstrap.argtypes = [ctypes.POINTER(Problem_), ctypes.POINTER(Options_), ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.POINTER(FitOpts_), ctypes.c_double,
                                     ctypes.POINTER(BootstrapOut_)]
        L.sccs_cv_query_workspace.argtypes = [ctypes.POINTER(Problem_), ctypes.POINTER(Options_), ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_size_t)]
        L.sccs_cv_search.argtypes = [ctypes.POINTER(Problem_), ctypes.POINTER(Options_), ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.POINTER(CvOpts_), ctypes.POINTER(CvResult_)]
        L.sccs_column_order.argtypes = [ctypes.POINTER(Problem_), ctypes.c_int32, ctypes.c_void_p]
        L.sccs_get_column_order.argtypes = [H, ctypes.c_void_p]
        for name in EXPORTS:
            if name not in ("sccs_default_options", "sccs_last_error", "sccs_batch_last_error"):
                getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class ProblemArrays:
    """Contiguous host copies of a problem plus the C structure that points at them."""

    def __init__(self, prob, weight: Optional[np.ndarray] = None):
        self.patient_ptr = _arr(prob.patient_ptr, np.int64)
        self.offset = _arr(prob.offset, np.int32)
        self.count = _arr(prob.count, np.int32)
        self.col_ptr = _arr(prob.col_ptr, np.int64)
        self.row_idx = _arr(prob.row_idx, np.int32)
        self.weight = None if weight is None else _arr(weight, np.int32)
        v = getattr(prob, "value", None)
        self.value = None if v is None else _arr(v, np.float64)
        self.n_cols = int(prob.n_cols)
        self.s = Problem_(int(prob.n_patients), int(self.patient_ptr[-1]), self.n_cols,
                          int(self.col_ptr[-1]), self.patient_ptr.ctypes.data, self.offset.ctypes.data,
                          self.count.ctypes.data, self.col_ptr.ctypes.data,
                          self.row_idx.ctypes.data if self.row_idx.size else None,
                          None if self.weight is None else self.weight.ctypes.data,
                          None if self.value is None or not self.value.size else self.value.ctypes.data)


def options(precision: int = PREC_FP64, n_workgroups: int = 0, refresh_period: int = -1,
            stream: Optional[int] = None, tile_nnz: int = 0, max_group: int = 0,
            merge_passes: int = 1, batch_engine: int = 0, column_order: int = 0) -> Options_:
    o = Options_()
    lib().sccs_default_options(ctypes.byref(o))
    o.precision = precision
    o.n_workgroups = n_workgroups
    o.refresh_period = refresh_period
    o.tile_nnz = tile_nnz
    o.max_group = max_group
    o.merge_passes = merge_passes
    o.stream = stream
    o.batch_engine = batch_engine
    o.column_order = column_order
    return o


def query_workspace(prob, weight=None, **opt) -> int:
    P = ProblemArrays(prob, weight)
    o = options(**opt)
    n = ctypes.c_size_t()
    st = lib().sccs_query_workspace(ctypes.byref(P.s), ctypes.byref(o), ctypes.byref(n))
    if st != OK:
        raise SccsError(st, lib().sccs_last_error(None).decode())
    return int(n.value)


class Handle:
    """One fit state on the GPU.  The workspace is a torch uint8 tensor kept
    alive by this object; the stream defaults to torch's current stream."""

    def __init__(self, prob, weight=None, precision: int = PREC_FP64, n_workgroups: int = 0,
                 refresh_period: int = -1, stream=None, workspace: str = "torch", tile_nnz: int = 0,
                 max_group: int = 0, merge_passes: int = 1, column_order: int = ORDER_GIVEN):
        import torch
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        P = ProblemArrays(prob, weight)
        o = options(precision, n_workgroups, refresh_period, stream.cuda_stream, tile_nnz, max_group,
                    merge_passes, column_order=column_order)
        n = ctypes.c_size_t()
        L = lib()
        st = L.sccs_query_workspace(ctypes.byref(P.s), ctypes.byref(o), ctypes.byref(n))
        if st != OK:
            raise SccsError(st, L.sccs_last_error(None).decode())
        self.workspace_bytes = int(n.value)
        if workspace == "torch":
            self.ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
            ptr = self.ws.data_ptr()
            ptr = (ptr + 255) & ~255
        else:
            self.ws, ptr = None, None
        h = ctypes.c_void_p()
        st = L.sccs_create(ctypes.byref(P.s), ctypes.byref(o), ptr, self.workspace_bytes, ctypes.byref(h))
        if st != OK:
            raise SccsError(st, L.sccs_last_error(None).decode())
        self.h = h
        self.J = P.n_cols
        self.precision = precision
        _live.add(self)

    def _check(self, st: int, allow=(OK,)) -> int:
        if st not in allow:
            raise SccsError(st, lib().sccs_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            lib().sccs_destroy(self.h)
            self.h = None
            self.ws = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_prior(self, kind: int, variance: float = 1.0):
        self._check(lib().sccs_set_prior(self.h, int(kind), float(variance)))

    def set_prior_grouped(self, variance: float, class_variance: float, class_of):
        """Grouped Normal prior: drugs of one class share a class mean with
        variance class_variance, each drug varies around it with variance."""
        c = _arr(class_of, np.int32)
        n = int(c.max()) + 1 if c.size else 1
        self._check(lib().sccs_set_prior_grouped(self.h, float(variance), float(class_variance), n, c.ctypes.data))

    def set_beta(self, beta, trust=None):
        b = _arr(beta, np.float64)
        t = None if trust is None else _arr(trust, np.float64)
        self._check(lib().sccs_set_beta(self.h, b.ctypes.data, None if t is None else t.ctypes.data))

    def get_beta(self) -> Tuple[np.ndarray, np.ndarray]:
        b = np.zeros(self.J)
        t = np.zeros(self.J)
        self._check(lib().sccs_get_beta(self.h, b.ctypes.data, t.ctypes.data))
        return b, t

    def sweep(self, n: int = 1, want_logpost: bool = False) -> Optional[float]:
        if want_logpost:
            lp = ctypes.c_double()
            self._check(lib().sccs_sweep(self.h, int(n), ctypes.byref(lp)))
            return lp.value
        self._check(lib().sccs_sweep(self.h, int(n), None))
        return None

    def sweep_static(self, n: int = 1, want_logpost: bool = False) -> Optional[float]:
        """sccs_sweep_static: the same sweeps with the reduction scratch taken
        from the library's static device array (no allocation)."""
        lp = ctypes.c_double()
        self._check(lib().sccs_sweep_static(self.h, int(n), ctypes.byref(lp) if want_logpost else None))
        return lp.value if want_logpost else None

    def fit(self, criterion: int = CRIT_REL_LOGPOST, max_sweeps: int = 100, tol: float = 1e-8) -> dict:
        fo = FitOpts_(int(criterion), int(max_sweeps), float(tol))
        r = FitResult_()
        st = self._check(lib().sccs_fit(self.h, ctypes.byref(fo), ctypes.byref(r)), allow=(OK, NOT_CONVERGED))
        return {"status": st, "sweeps": r.sweeps, "converged": bool(r.converged),
                "loglik": r.loglik, "logpost": r.logpost}

    def grad_hess(self, j: int) -> Tuple[float, float]:
        g, h = ctypes.c_double(), ctypes.c_double()
        self._check(lib().sccs_grad_hess(self.h, int(j), ctypes.byref(g), ctypes.byref(h)))
        return g.value, h.value

    def objective(self) -> Tuple[float, float]:
        L_, P_ = ctypes.c_double(), ctypes.c_double()
        self._check(lib().sccs_objective(self.h, ctypes.byref(L_), ctypes.byref(P_)))
        return L_.value, P_.value

    def last_kernel_ms(self) -> float:
        ms = ctypes.c_double()
        self._check(lib().sccs_last_kernel_ms(self.h, ctypes.byref(ms)))
        return ms.value

    def pass_stats(self) -> Tuple[int, int, int]:
        """(device-wide reductions, rejected merges, zero-step visits) of the
        last sweep/fit launch."""
        p, r, z = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().sccs_pass_stats(self.h, ctypes.byref(p), ctypes.byref(r), ctypes.byref(z)))
        return p.value, r.value, z.value

    def column_order(self) -> np.ndarray:
        """The column each sweep position visits (identity for the given order)."""
        out = np.zeros(self.J, dtype=np.int32)
        self._check(lib().sccs_get_column_order(self.h, out.ctypes.data))
        return out

    def group_timing(self, on: bool = True) -> None:
        """Stamp each column group in later sweep launches (read with group_times)."""
        self._check(lib().sccs_group_timing(self.h, 1 if on else 0))

    def group_times(self):
        """(microseconds from the last sweep's start to each column group's
        step, first sweep position of each group) of the last one-pass launch
        made with group_timing on."""
        n = ctypes.c_int32()
        cap = self.J
        t = np.zeros(cap)
        fc = np.zeros(cap + 1, dtype=np.int32)
        self._check(lib().sccs_group_times(self.h, cap, t.ctypes.data, fc.ctypes.data, ctypes.byref(n)))
        k = n.value
        return t[:k], fc[:k + 1]


def column_order(prob, width: int = 4) -> np.ndarray:
    """sccs_column_order: the independence relabelling of prob's columns
    (order[k] is the column a sweep visits k-th).  Host only."""
    P = ProblemArrays(prob)
    out = np.zeros(P.n_cols, dtype=np.int32)
    st = lib().sccs_column_order(ctypes.byref(P.s), int(width), out.ctypes.data)
    if st != OK:
        raise SccsError(st, lib().sccs_last_error(None).decode())
    return out


def tune(prob, prior_kind: int, variance: float, n_sweeps: int = 2, precision: int = PREC_FP64, weight=None):
    """Run the library's autotuner; returns (best options dict, candidate table)."""
    import torch  # noqa: F401
    P = ProblemArrays(prob, weight)
    o = options(precision, 0, -1, torch.cuda.current_stream().cuda_stream)
    best = Options_()
    r = TuneResult_()
    st = lib().sccs_tune(ctypes.byref(P.s), ctypes.byref(o), int(prior_kind), float(variance), int(n_sweeps),
                         ctypes.byref(best), ctypes.byref(r))
    if st != OK:
        raise SccsError(st, lib().sccs_last_error(None).decode())
    table = [{"n_workgroups": r.n_workgroups[k], "tile_nnz": r.tile_nnz[k], "ms_per_sweep": r.ms_per_sweep[k]}
             for k in range(r.n_candidates)]
    return {"n_workgroups": best.n_workgroups, "tile_nnz": best.tile_nnz}, table


def batch_tune(probs, specs, n_sweeps: int = 2, precision: int = PREC_FP64, engine: int = 0):
    """Run the batched form's autotuner; returns (best options dict, candidate table)."""
    import torch
    P = [ProblemArrays(p) for p in probs]
    parr = (Problem_ * len(P))(*[q.s for q in P])
    sarr = (FitSpec_ * len(specs))(*[s.struct() for s in specs])
    o = options(precision, 0, -1, torch.cuda.current_stream().cuda_stream, batch_engine=engine)
    best = Options_()
    r = TuneResult_()
    st = lib().sccs_batch_tune(ctypes.addressof(parr), len(P), ctypes.addressof(sarr), len(specs), ctypes.byref(o),
                               int(n_sweeps), ctypes.byref(best), ctypes.byref(r))
    if st != OK:
        raise SccsError(st, lib().sccs_batch_last_error(None).decode())
    table = [{"n_workgroups": r.n_workgroups[k], "tile_nnz": r.tile_nnz[k], "ms_per_sweep": r.ms_per_sweep[k]}
             for k in range(r.n_candidates)]
    return {"n_workgroups": best.n_workgroups, "tile_nnz": best.tile_nnz}, table


class FitSpec:
    """One fit of a batch: a problem index, a chain of (prior kind, variance)
    links visited with warm starts, and optional patient weights."""

    def __init__(self, problem: int, links, weight=None):
        self.problem = int(problem)
        self.kinds = np.ascontiguousarray([int(k) for k, _ in links], dtype=np.int32)
        self.vars = np.ascontiguousarray([float(v) for _, v in links], dtype=np.float64)
        self.weight = None if weight is None else _arr(weight, np.int32)

    def struct(self) -> FitSpec_:
        return FitSpec_(self.problem, len(self.kinds), self.kinds.ctypes.data, self.vars.ctypes.data,
                        None if self.weight is None else self.weight.ctypes.data)


class Batch:
    """Many fits in one persistent launch (sccs_batch_*)."""

    def __init__(self, probs, specs, precision: int = PREC_FP64, n_workgroups: int = 0,
                 refresh_period: int = -1, stream=None, tile_nnz: int = 0, max_group: int = 0,
                 engine: int = 0, column_order: int = ORDER_GIVEN):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._probs = [ProblemArrays(p) for p in probs]
        self._specs = list(specs)
        parr = (Problem_ * len(self._probs))(*[P.s for P in self._probs])
        sarr = (FitSpec_ * len(self._specs))(*[s.struct() for s in self._specs])
        self._parr, self._sarr = parr, sarr
        o = options(precision, n_workgroups, refresh_period, stream.cuda_stream, tile_nnz, max_group,
                    batch_engine=engine, column_order=column_order)
        L = lib()
        n = ctypes.c_size_t()
        st = L.sccs_batch_query_workspace(ctypes.addressof(parr), len(self._probs), ctypes.addressof(sarr),
                                          len(self._specs), ctypes.byref(o), ctypes.byref(n))
        if st != OK:
            raise SccsError(st, L.sccs_batch_last_error(None).decode())
        self.workspace_bytes = int(n.value)
        self.ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
        ptr = (self.ws.data_ptr() + 255) & ~255
        h = ctypes.c_void_p()
        st = L.sccs_batch_create(ctypes.addressof(parr), len(self._probs), ctypes.addressof(sarr),
                                 len(self._specs), ctypes.byref(o), ptr, self.workspace_bytes, ctypes.byref(h))
        if st != OK:
            raise SccsError(st, L.sccs_batch_last_error(None).decode())
        self.h = h
        self.J = self._probs[0].n_cols
        _live.add(self)

    def _check(self, st):
        if st != OK:
            raise SccsError(st, lib().sccs_batch_last_error(self.h).decode())

    def run(self, criterion: int = CRIT_REL_LOGPOST, max_sweeps: int = 100, tol: float = 1e-8):
        fo = FitOpts_(int(criterion), int(max_sweeps), float(tol))
        self._check(lib().sccs_batch_run(self.h, ctypes.byref(fo)))

    def get(self, fit: int, link: int = 0):
        b = np.zeros(self.J)
        r = FitResult_()
        self._check(lib().sccs_batch_get(self.h, int(fit), int(link), b.ctypes.data, ctypes.byref(r)))
        return b, {"sweeps": r.sweeps, "converged": bool(r.converged), "loglik": r.loglik, "logpost": r.logpost}

    def heldout(self, fit: int, link: int = 0) -> float:
        """Eq. 2 over the fit's weight-0 patients at the link's beta."""
        v = ctypes.c_double()
        self._check(lib().sccs_batch_heldout(self.h, int(fit), int(link), ctypes.byref(v)))
        return v.value

    def last_kernel_ms(self) -> float:
        ms = ctypes.c_double()
        self._check(lib().sccs_batch_last_kernel_ms(self.h, ctypes.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            lib().sccs_batch_destroy(self.h)
            self.h = None
            self.ws = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def bootstrap(prob, prior_kind: int, variance: float, weights, criterion: int = CRIT_REL_LOGPOST,
              max_sweeps: int = 100, tol: float = 1e-8, level: float = 0.95, precision: int = PREC_FP64,
              n_workgroups: int = 0, stream=None, engine: int = 0, column_order: int = ORDER_GIVEN) -> dict:
    """sccs_bootstrap: one fit per row of weights ([R, N] patient
    multiplicities), percentile intervals and the share of nonzero estimates.
    Returns dict(beta [R, J], lo, hi, p_nonzero, sweeps, converged)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    W = _arr(weights, np.int32)
    R = int(W.shape[0])
    P = ProblemArrays(prob)
    if W.ndim != 2 or W.shape[1] != int(prob.n_patients):
        raise ValueError("weights must be [n_replicates, n_patients]")
    o = options(precision, n_workgroups, -1, stream.cuda_stream, batch_engine=engine, column_order=column_order)
    L = lib()
    n = ctypes.c_size_t()
    st = L.sccs_bootstrap_query_workspace(ctypes.byref(P.s), ctypes.byref(o), R, ctypes.byref(n))
    if st != OK:
        raise SccsError(st, L.sccs_batch_last_error(None).decode())
    ws = torch.empty(int(n.value) + 256, dtype=torch.uint8, device="cuda")
    ptr = (ws.data_ptr() + 255) & ~255
    J = P.n_cols
    beta = np.zeros((R, J))
    lo, hi, pnz = np.zeros(J), np.zeros(J), np.zeros(J)
    sw, cv = np.zeros(R, dtype=np.int32), np.zeros(R, dtype=np.int32)
    out = BootstrapOut_(beta.ctypes.data, lo.ctypes.data, hi.ctypes.data, pnz.ctypes.data, sw.ctypes.data,
                        cv.ctypes.data)
    fo = FitOpts_(int(criterion), int(max_sweeps), float(tol))
    st = L.sccs_bootstrap(ctypes.byref(P.s), ctypes.byref(o), ptr, int(n.value), int(prior_kind), float(variance), R,
                          W.ctypes.data, ctypes.byref(fo), float(level), ctypes.byref(out))
    if st != OK:
        raise SccsError(st, L.sccs_batch_last_error(None).decode())
    del ws
    return {"beta": beta, "lo": lo, "hi": hi, "p_nonzero": pnz, "sweeps": sw, "converged": cv.astype(bool)}


def cv_search(prob, folds, n_folds: int, prior_kind: int, var_start: float = 0.01, bracket_step: float = 10.0,
              log10_tol: float = 0.05, max_evals: int = 30, warm_start: bool = True,
              criterion: int = CRIT_REL_LOGPOST, max_sweeps: int = 100, tol: float = 1e-10,
              precision: int = PREC_FP64, n_workgroups: int = 0, stream=None, engine: int = 0,
              column_order: int = ORDER_GIVEN) -> dict:
    """sccs_cv_search: bracketing and golden-section search of the
    cross-validated predictive log-likelihood over the prior variance.
    Returns dict(variance, pred_loglik [per evaluation], best, bracketed)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    P = ProblemArrays(prob)
    fold = _arr(folds, np.int32)
    o = options(precision, n_workgroups, -1, stream.cuda_stream, batch_engine=engine, column_order=column_order)
    L = lib()
    n = ctypes.c_size_t()
    st = L.sccs_cv_query_workspace(ctypes.byref(P.s), ctypes.byref(o), int(n_folds), ctypes.byref(n))
    if st != OK:
        raise SccsError(st, L.sccs_batch_last_error(None).decode())
    ws = torch.empty(int(n.value) + 256, dtype=torch.uint8, device="cuda")
    ptr = (ws.data_ptr() + 255) & ~255
    co = CvOpts_(int(prior_kind), int(n_folds), fold.ctypes.data, float(var_start), float(bracket_step),
                 float(log10_tol), int(max_evals), int(bool(warm_start)),
                 FitOpts_(int(criterion), int(max_sweeps), float(tol)))
    r = CvResult_()
    st = L.sccs_cv_search(ctypes.byref(P.s), ctypes.byref(o), ptr, int(n.value), ctypes.byref(co), ctypes.byref(r))
    if st != OK:
        raise SccsError(st, L.sccs_batch_last_error(None).decode())
    del ws
    k = r.n_evals
    return {"variance": np.array(r.variance[:k]), "pred_loglik": np.array(r.pred_loglik[:k]),
            "best": int(r.best), "bracketed": bool(r.bracketed)}
