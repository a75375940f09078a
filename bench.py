"""Benchmark: CCD sweeps/s of the BSCCS MAP fit on one MI355X.

Workload (the configuration the headline metric is quoted on): 2M patients,
~20M eras (1 + Poisson(9) per patient), J = 2000 binary drugs with Zipf(1.1)
popularity, Laplace prior lambda = 1 (variance 2), FP64.  One step = one full
cyclic sweep over all 2000 coordinates (gather + segmented sums, device-wide
reduction, Newton/trust-region step, sparse update), one persistent launch.
After the warm-up sweeps the fit is reset to beta = 0, so the timed steps
are sweeps 1..K of a fit from zero.

Prints one JSON line.  Besides the required fields it carries:
  roofline      algorithmic bytes of the sweep (stated byte model) / the
                sweep kernel's mean launch time (HIP events on the launch
                stream) against 8 TB/s, and the library's own byte model;
  schedule      device-wide reductions (passes) per sweep and their mean time;
  late_sweeps   the sweeps after the headline ones, timed on their own;
  cpu_baseline  the FP64 C oracle timed on the host on a bounded sample;
  mixed         the mixed-precision form on the same schedule: sweeps/s and
                its relative beta error against the FP64 GPU path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CCD sweeps/sec + HBM GB/s at 20M eras, J=2000; mixed vs FP64 at 1e-6 rel"
HBM_PEAK_GBS = 8000.0


def column_stats(prob):
    """Nonzeros c_j and distinct patients p_j of every column."""
    c = np.diff(prob.col_ptr)
    era_pid = np.repeat(np.arange(prob.n_patients, dtype=np.int64), np.diff(prob.patient_ptr))
    pid = era_pid[prob.row_idx]
    col = np.repeat(np.arange(prob.n_cols), c)
    new = np.ones(len(pid), dtype=bool)
    new[1:] = (pid[1:] != pid[:-1]) | (col[1:] != col[:-1])
    p = np.bincount(col[new], minlength=prob.n_cols)
    return c.astype(np.int64), p.astype(np.int64)


def bytes_per_sweep(c, p, active, precision):
    """Algorithmic bytes of one sweep, per coordinate j with c_j nonzeros and
    p_j distinct patients (the method's own data movement, X beta kept as an
    era array as in Section 2.4 Steps 1-4):
      phase A, every coordinate: 12 c_j + 16 p_j -- per nonzero its row index
        (4 B) and the gathered w_k (8 B); per patient segment its patient
        index (4 B), den_i (8 B) and n_i (4 B);
      phase B, coordinates with a nonzero step: 28 c_j + 8 p_j -- per nonzero
        the read-modify-write of (X beta)_k (16 B), l_k (4 B) and the new w_k
        (8 B); per segment the new den_i (8 B).
    The mixed form stores w in 4 B: 8 c_j + 16 p_j and 24 c_j + 8 p_j."""
    return phase_a_bytes(c, p, precision) + phase_b_bytes(c, p, active, precision)


def phase_a_bytes(c, p, precision):
    wb = 8 if precision == 0 else 4
    return float((4 + wb) * c.sum() + 16 * p.sum())


def phase_b_bytes(c, p, active, precision):
    wb = 8 if precision == 0 else 4
    return float((20 + wb) * c[active].sum() + 8 * p[active].sum())


def bytes_per_sweep_library(c, p, active, precision):
    """The bytes this library's kernel has to move for the same sweep: it
    stores (row, patient) pairs (8 B per nonzero), gathers (den_i, omega_i
    n_i) as one 16-byte pair, and updates w multiplicatively (no X beta
    array, no l read): phase A (8 + wb) c_j + 16 p_j, phase B wb c_j + 8 p_j
    (wb = 8 FP64, 4 mixed)."""
    wb = 8 if precision == 0 else 4
    a = (8 + wb) * c.sum() + 16 * p.sum()
    b = wb * c[active].sum() + 8 * p[active].sum()
    return float(a + b)


def run_form(sccs, prob, precision, steps, warmup, c, p, n_workgroups=0, late=0, refresh_period=-1, column_order=1):
    """warmup sweeps, then beta reset to 0 (exact state recomputation) and
    `steps` timed sweeps from beta = 0, one launch each; then `late` more
    sweeps timed on their own (the fit continuing toward convergence)."""
    import torch
    h = sccs.Handle(prob, precision=precision, n_workgroups=n_workgroups, refresh_period=refresh_period,
                    column_order=column_order)
    h.set_prior(sccs.PRIOR_LAPLACE, 2.0)
    for _ in range(warmup):
        h.sweep(1)
    h.set_beta(np.zeros(prob.n_cols))
    beta_prev, _ = h.get_beta()
    torch.cuda.synchronize()

    def timed(n):
        nonlocal beta_prev
        rec = {"kernel_ms": [], "bytes": [], "bytes_lib": [], "passes": []}
        t0 = time.perf_counter()
        for _ in range(n):
            h.sweep(1)
            rec["kernel_ms"].append(h.last_kernel_ms())
            rec["passes"].append(h.pass_stats())
            beta, _ = h.get_beta()
            moved = beta != beta_prev
            rec["bytes"].append(bytes_per_sweep(c, p, moved, precision))
            rec["bytes_lib"].append(bytes_per_sweep_library(c, p, moved, precision))
            beta_prev = beta
        torch.cuda.synchronize()
        rec["wall_s"] = time.perf_counter() - t0
        return rec

    out = timed(steps)
    out["beta"] = beta_prev.copy()
    if late:
        out["late"] = timed(late)
    h.close()
    return out


def profiled_traffic(kernel_ms):
    """HBM bytes per launch of the sweep kernel from the committed counter
    summary, if the kernel sources are unchanged since the counters were
    taken; otherwise None."""
    path = os.path.join(ROOT, "profiles", "k_ccd_mid_fp64_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kernel_source_sha() != kv.get("kernel_source_sha"):
        return None
    return float(kv["traffic_bytes_per_launch"])


KERNEL_SOURCES = ("sccs_kernels.hpp", "sccs_device.hpp", "sccs_limits.hpp", "sccs_layout.cpp")


def kernel_source_sha() -> str:
    """sha256 (first 16 hex digits) of the sources that decide the sweep
    kernel's memory traffic: device code, launch constants and the layout,
    with comments, indentation and blank lines removed (an edit of comments
    or layout does not change the kernel)."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1208_0945_amd", "csrc")
    code = []
    for f in KERNEL_SOURCES:
        for line in open(os.path.join(csrc, f)):
            line = re.sub(r"//.*", "", line).strip()
            if line:
                code.append(line)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()[:16]


def host_description():
    """CPU model, logical CPUs visible to this process and the C compiler."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        import subprocess
        cc = subprocess.run(["gcc", "--version"], capture_output=True, text=True).stdout.splitlines()[0]
    except Exception:
        cc = "unknown"
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "compiler": cc,
            "flags": "-O2 -std=c99 (no fast-math)"}


def cpu_baseline(prob, sweeps):
    import oracle
    oracle.build(force=False)
    P = oracle.OracleProblem(prob)
    t0 = time.perf_counter()
    oracle.ccd(P, oracle.PRIOR_LAPLACE, 2.0, 0)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.ccd(P, oracle.PRIOR_LAPLACE, 2.0, sweeps)
    t = time.perf_counter() - t0
    per = max(t - t_setup, 1e-9) / sweeps
    return {"value": 1.0 / per, "unit": "sweeps/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {sweeps} CCD sweeps from beta = 0 of the same workload by the "
                      f"single-threaded FP64 C oracle, one-time setup ({t_setup:.2f} s) subtracted; "
                      f"{t:.1f} s total",
            "host": host_description()}


def copy_calibration(n_bytes: int = 1 << 30, reps: int = 3):
    """A plain device copy of known size, to scale the FETCH_SIZE and
    WRITE_SIZE counters of the sweep kernel to bytes."""
    import torch
    src = torch.empty(n_bytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n_bytes, "reps": reps}), flush=True)


def batched_outcomes_bench(sccs, synth, steps, precision, engine=0, column_order=1):
    """64 outcomes over one J = 1000 vocabulary, patient counts log-uniform
    10k..2M, Laplace lambda = 1: one launch runs `steps` sweeps of all 64."""
    t0 = time.perf_counter()
    sizes = synth.outcome_sizes(64)
    probs = synth.batched_outcomes(64, n_cols=1000, sizes=sizes, progress=lambda f: (
        print(f"[bench] outcome {f} generated", file=sys.stderr, flush=True) if f % 8 == 7 else None))
    print(f"[bench] generated 64 outcomes ({sum(p.n_patients for p in probs)} patients, "
          f"{sum(p.nnz for p in probs)} nonzeros) in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    specs = [sccs.FitSpec(f, [(sccs.PRIOR_LAPLACE, 2.0)]) for f in range(len(probs))]
    stats = [column_stats(p) for p in probs]
    t0 = time.perf_counter()
    co = column_order if engine == 0 else 0   # the lockstep engine keeps the given order
    with sccs.Batch(probs, specs, precision=precision, engine=engine, column_order=co) as b:
        print(f"[bench] batch set up in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
        b.run(sccs.CRIT_FIXED, max_sweeps=1)            # warm-up launch (the chains restart from its beta)
        t0 = time.perf_counter()
        b.run(sccs.CRIT_FIXED, max_sweeps=steps)
        wall = time.perf_counter() - t0
        ms = b.last_kernel_ms()
    # algorithmic bytes with every coordinate active (upper bound on phase B)
    tot = sum(bytes_per_sweep(c, p_, np.ones(len(c), bool), precision) for c, p_ in stats) * steps
    return {"metric": "batched outcomes: fit-sweeps/s (64 fits, J=1000, one launch)",
            "value": 64 * steps / wall, "unit": "fit-sweeps/s", "steps": steps, "kernel_ms": ms,
            "achieved_GBs_upper": tot / (ms * 1e-3) / 1e9,
            "dtype": "f64" if precision == 0 else "mixed",
            "config": {"workload": "64 outcomes, J=1000 Zipf(1.1), N log-uniform 1e4..2e6, Laplace lambda=1",
                       "engine": ["partitioned", "lockstep"][engine],
                       "column_order": ["given", "independent"][co],
                       "n_patients_total": int(sum(p.n_patients for p in probs)),
                       "nnz_total": int(sum(p.nnz for p in probs))}}


def cv_bench(sccs, synth, precision, max_sweeps, tol, n_folds=10, n_grid=16, engine=0, column_order=1):
    """The mid problem under 10-fold patient-level cross-validation x 16
    Laplace variances logspace(-3, 1): 10 fold chains walk the grid upward
    with warm starts (partitioned engine: one launch per variance, the folds
    on disjoint workgroup ranges; lockstep engine: one launch for the whole
    grid); then the held-out log-likelihood (Eq. 2 over the held-out
    patients) of every (fold, variance) fit."""
    prob = synth.mid()
    folds = synth.cv_folds(prob.n_patients, n_folds)
    grid = synth.prior_grid(n_grid)
    specs = [sccs.FitSpec(0, [(sccs.PRIOR_LAPLACE, float(v)) for v in grid], weight=(folds != k).astype(np.int32))
             for k in range(n_folds)]
    co = column_order if engine == 0 else 0   # the lockstep engine keeps the given order
    with sccs.Batch([prob], specs, precision=precision, engine=engine, column_order=co) as b:
        t0 = time.perf_counter()
        b.run(sccs.CRIT_REL_LOGPOST, max_sweeps=max_sweeps, tol=tol)
        wall = time.perf_counter() - t0
        ms = b.last_kernel_ms()
        res = [[b.get(k, l) for l in range(n_grid)] for k in range(n_folds)]
        heldout = np.array([[b.heldout(k, l) for l in range(n_grid)] for k in range(n_folds)])
    sw = np.array([[r[1]["sweeps"] for r in row] for row in res])   # [fold, variance]
    sweeps = int(sw.sum())
    # sweeps on the critical path: lockstep, the longest fold chain; partitioned,
    # per variance the slowest fold (each variance is one launch)
    critical = int(sw.sum(axis=1).max()) if engine == 1 else int(sw.max(axis=0).sum())
    c, p = column_stats(prob)
    phase_a = bytes_per_sweep(c, p, np.zeros(len(c), bool), precision)   # every visit's gathers
    mean = heldout.mean(axis=0)
    return {"metric": "batched CV: fit-sweeps/s (10 folds x 16 Laplace variances, warm starts)",
            "value": sweeps / wall, "unit": "fit-sweeps/s", "kernel_ms": ms, "wall_s": wall,
            "total_fit_sweeps": sweeps, "critical_path_sweeps": critical,
            "ms_per_critical_sweep": ms / max(critical, 1),
            # phase A of all folds in every critical-path sweep (a fold that
            # finished early is counted too; phase B is left out)
            "achieved_GBs_phase_a": n_folds * phase_a / (ms / max(critical, 1) * 1e-3) / 1e9,
            "dtype": "f64" if precision == 0 else "mixed",
            "best_variance": float(grid[int(np.argmax(mean))]),
            "heldout_loglik_mean_by_variance": [float(x) for x in mean],
            "config": {"workload": f"mid SCCS ({prob.n_patients} patients, J={prob.n_cols}) x 10 folds x 16 variances",
                       "engine": ["partitioned", "lockstep"][engine],
                       "column_order": ["given", "independent"][co],
                       "max_sweeps_per_link": max_sweeps, "tol": tol}}


def full_bench(sccs, synth, steps, refit=True, column_order=1):
    """Full-scale workload, precision form against the FP64 GPU path: 10M
    patients, ~100M eras, J = 4000 Zipf drugs (p_j = 0.482 rank^-1.1),
    Normal prior variance 0.5; `steps` sweeps each; then a seeded 1% patient
    subsample refit to convergence by the GPU (both forms) and the oracle."""
    import oracle
    t0 = time.perf_counter()
    prob = synth.full()
    print(f"[bench] generated {prob.summary()} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    out = {"metric": "full-scale SCCS: sweeps/s, FP64 and mixed, and mixed error vs the FP64 oracle",
           "config": {"workload": "full SCCS: 10M patients, J=4000 Zipf(1.1) p0=0.482, Normal var 0.5",
                      "n_patients": prob.n_patients, "n_eras": prob.n_rows, "nnz": prob.nnz,
                      "column_order": ["given", "independent"][column_order]}}
    c, p = column_stats(prob)
    betas = {}
    for prec, name in ((0, "fp64"), (1, "mixed")):
        t0 = time.perf_counter()
        with sccs.Handle(prob, precision=prec, column_order=column_order) as h:
            print(f"[bench] {name} handle set up in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
            h.set_prior(sccs.PRIOR_NORMAL, 0.5)
            h.sweep(1)
            t0 = time.perf_counter()
            h.sweep(steps)
            wall = time.perf_counter() - t0
            ms = h.last_kernel_ms() / steps
            beta = h.get_beta()[0]
            # Normal prior: every coordinate moves
            algo = bytes_per_sweep(c, p, np.ones(len(c), bool), prec)
            out[name] = {"sweeps_per_s": steps / wall, "kernel_ms_per_sweep": ms,
                         "algo_bytes_per_sweep": algo, "achieved_GBs": algo / (ms * 1e-3) / 1e9,
                         "frac_of_8TBs": algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            betas[name] = beta
        print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)
    out["mixed_vs_fp64_gpu_rel_err"] = float(np.max(np.abs(betas["mixed"] - betas["fp64"])) /
                                            np.max(np.abs(betas["fp64"])))
    if not refit:
        return out
    sub = synth.subsample_patients(prob, 0.01)
    del prob
    ref = oracle.ccd(sub, oracle.PRIOR_NORMAL, 0.5, 500, oracle.CRIT_REL_LOGPOST, 1e-12)
    print(f"[bench] oracle refit of the 1% subsample: {ref['sweeps']} sweeps", file=sys.stderr, flush=True)
    errs = {}
    for prec, name in ((0, "fp64"), (1, "mixed")):
        # the given order: the oracle's trajectory, sweep for sweep
        with sccs.Handle(sub, precision=prec) as h:
            h.set_prior(sccs.PRIOR_NORMAL, 0.5)
            h.sweep(ref["sweeps"])
            b = h.get_beta()[0]
        errs[name] = float(np.max(np.abs(b - ref["beta"])) / np.max(np.abs(ref["beta"])))
    out["subsample_refit"] = {"n_patients": sub.n_patients, "nnz": sub.nnz, "oracle_sweeps": ref["sweeps"],
                              "rel_err_vs_oracle": errs}
    return out


def paper_fit_bench(sccs, synth, max_sweeps=1000, column_order=1):
    """One MAP fit to convergence at the size of the paper's largest dataset
    (3.6M patients, ~75M eras, J = 1428; synthetic, mid-like popularity)
    under the paper's stopping rule, sum_k |change of (X beta)_k| over a
    sweep below 5e-4, from beta = 0, FP64 and mixed.  The paper's own time
    for its real dataset of that size is context only."""
    t0 = time.perf_counter()
    prob = synth.paper_shaped()
    print(f"[bench] generated {prob.summary()} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    out = {"metric": "MAP fit to convergence at the paper's largest size: wall seconds (lower is better)",
           "unit": "s", "higher_is_better": False,
           "config": {"workload": "3.6M patients, J=1428 Zipf(1.1) p0=0.1, eras 1+Poisson(19.83), "
                                  "Normal var 1, stop when sum|d(X beta)| < 5e-4",
                      "column_order": ["given", "independent"][column_order],
                      "n_patients": prob.n_patients, "n_eras": prob.n_rows, "nnz": prob.nnz},
           "paper_context": "29 s on one Tesla C2050 for a real claims dataset of 3.6M patients, "
                            "75M eras, 1428 drugs (Section 4); other data and hardware"}
    # The mixed form's FP32 w puts a floor of roughly 1e-7 relative on every
    # Newton step, i.e. sum|d(X beta)| of order 1 at K = 75M: it cannot meet
    # the absolute rule, so it runs a capped number of sweeps and reports its
    # distance from the FP64 fit instead.
    betas = {}
    for prec, name, cap in ((0, "fp64", max_sweeps), (1, "mixed", 30)):
        t0 = time.perf_counter()
        with sccs.Handle(prob, precision=prec, column_order=column_order) as h:
            setup = time.perf_counter() - t0
            h.set_prior(sccs.PRIOR_NORMAL, 1.0)
            t0 = time.perf_counter()
            r = h.fit(sccs.CRIT_ABS_DXBETA, max_sweeps=cap, tol=5e-4)
            wall = time.perf_counter() - t0
            betas[name] = h.get_beta()[0]
            out[name] = {"fit_s": wall, "setup_s": setup, "sweeps": r["sweeps"], "converged": r["converged"],
                         "ms_per_sweep": wall * 1e3 / max(r["sweeps"], 1), "logpost": r["logpost"]}
        print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)
    out["mixed"]["beta_rel_err_vs_fp64_gpu"] = float(np.max(np.abs(betas["mixed"] - betas["fp64"])) /
                                                     np.max(np.abs(betas["fp64"])))
    out["value"] = out["fp64"]["fit_s"]
    out["dtype"] = "f64"
    return out


def valued_bench(sccs, synth, steps):
    """Non-binary and dense covariates (values x_kj on the stored entries):
    2M patients, 1 + Poisson(6) eras, 200 binary Zipf drugs, 20 sparse dose
    columns (lognormal doses), 2 dense columns on every era (age-like and
    seasonal); Normal prior variance 1 (every coordinate moves); FP64 and
    mixed, `steps` sweeps from beta = 0 after one warm-up sweep.  Algorithmic
    bytes per coordinate: phase A 20 c_j + 16 p_j (row index, value and w
    per nonzero), phase B 36 c_j + 8 p_j (the binary form's bytes plus the
    value)."""
    t0 = time.perf_counter()
    prob = synth.valued(n_patients=2_000_000, n_drugs=200, n_dose=20, n_dense=2)
    print(f"[bench] generated {prob.summary()} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    c, p = column_stats(prob)
    out = {"metric": "non-binary and dense covariates: sweeps/s, FP64 and mixed", "unit": "sweeps/s",
           "config": {"workload": "2M patients, 200 drugs + 20 dose + 2 dense columns, Normal var 1",
                      "n_patients": prob.n_patients, "n_eras": prob.n_rows, "nnz": prob.nnz}}
    betas = {}
    for prec, name in ((0, "fp64"), (1, "mixed")):
        with sccs.Handle(prob, precision=prec) as h:
            h.set_prior(sccs.PRIOR_NORMAL, 1.0)
            h.sweep(1)
            h.set_beta(np.zeros(prob.n_cols))
            t0 = time.perf_counter()
            h.sweep(steps)
            wall = time.perf_counter() - t0
            ms = h.last_kernel_ms() / steps
            wb = 8 if prec == 0 else 4
            algo = float((12 + wb) * c.sum() + 16 * p.sum() + (28 + wb) * c.sum() + 8 * p.sum())
            out[name] = {"sweeps_per_s": steps / wall, "kernel_ms_per_sweep": ms, "algo_bytes_per_sweep": algo,
                         "achieved_GBs": algo / (ms * 1e-3) / 1e9,
                         "frac_of_8TBs": algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            betas[name] = h.get_beta()[0]
        print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)
    out["mixed_vs_fp64_gpu_rel_err"] = float(np.max(np.abs(betas["mixed"] - betas["fp64"])) /
                                            np.max(np.abs(betas["fp64"])))
    out["value"] = out["fp64"]["sweeps_per_s"]
    out["dtype"] = "f64"
    return out


def bootstrap_bench(sccs, synth, n_reps=200, n_patients=200_000):
    """The bootstrap procedure of Section 2.5 at the paper's replicate count:
    200 replicates of a mid-like problem of 200k patients (J = 2000), each
    resampling the patients with replacement, Laplace prior lambda = 1, each
    replicate fitted to a relative change of the log posterior below 1e-8
    (at most 50 sweeps); percentile intervals and the share of nonzero
    estimates."""
    prob = synth.mid(n_patients=n_patients)
    W = synth.bootstrap_weights(prob.n_patients, n_reps, seed=0)
    t0 = time.perf_counter()
    r = sccs.bootstrap(prob, sccs.PRIOR_LAPLACE, 2.0, W, criterion=sccs.CRIT_REL_LOGPOST, max_sweeps=50,
                       tol=1e-8, column_order=1)
    wall = time.perf_counter() - t0
    fit_sweeps = int(np.sum(r["sweeps"]))
    return {"metric": "bootstrap, 200 replicates: wall seconds (lower is better)", "unit": "s",
            "higher_is_better": False, "value": wall,
            "config": {"workload": f"mid-like, {prob.n_patients} patients, J={prob.n_cols}, {n_reps} replicates, "
                                   "Laplace lambda 1, rel. logpost 1e-8, <= 50 sweeps",
                       "nnz": prob.nnz},
            "fit_sweeps": fit_sweeps, "fit_sweeps_per_s": fit_sweeps / wall,
            "converged": int(np.sum(r["converged"])),
            "nonzero_share_median": float(np.median(r["p_nonzero"])), "dtype": "f64"}


def search_bench(sccs, synth, n_patients=2_000_000, n_folds=10):
    """The prior-variance search of Section 2.5 on the mid problem: 10
    patient folds, bracketing upward from variance 0.01 by factors of 10,
    then golden-section steps on log10(variance) to a width of 0.05, each
    evaluation a warm-started fit of every fold to a relative change of the
    log posterior below 1e-10 and the held-out log-likelihood."""
    prob = synth.mid(n_patients=n_patients)
    folds = synth.cv_folds(prob.n_patients, n_folds)
    t0 = time.perf_counter()
    r = sccs.cv_search(prob, folds, n_folds, sccs.PRIOR_LAPLACE, column_order=1)
    wall = time.perf_counter() - t0
    return {"metric": "cross-validated prior-variance search: wall seconds (lower is better)", "unit": "s",
            "higher_is_better": False, "value": wall,
            "config": {"workload": f"mid, {prob.n_patients} patients, {n_folds} folds, Laplace, bracket x10 "
                                   "from 0.01, golden section to 0.05 in log10"},
            "evaluations": len(r["variance"]), "best_variance": float(r["variance"][r["best"]]),
            "bracketed": bool(r["bracketed"]), "dtype": "f64"}


def coord_curve(sccs, synth, workload, n_workgroups, sweeps_at=(1, 2, 10), c_star=240_000, column_order=1):
    """Achieved bandwidth per coordinate against its column size (one-pass
    form, FP64, from beta = 0 under the workload's prior).  For each listed
    sweep the device stamps the moment every column group's steps are
    taken; a group's time is the gap to the previous group's stamp.  That gap
    holds the previous group's update (phase B) and this group's gathers and
    reduction (phase A), so its algorithmic bytes are phase A's of this
    group's columns plus phase B's of the previous group's moved columns.  Reported: the curve
    (median GB/s per power-of-two bucket of the group's nonzeros) and, over
    the columns with at least c_star nonzeros, the nonzero-weighted
    fraction of HBM peak (their bytes over their time)."""
    import torch
    if workload == "full":
        prob, kind, var = synth.full(), sccs.PRIOR_NORMAL, 0.5
    else:
        prob, kind, var = synth.mid(), sccs.PRIOR_LAPLACE, 2.0
    c, p = column_stats(prob)
    out = {"workload": f"{workload} SCCS: {prob.n_patients} patients, {prob.n_rows} eras, J={prob.n_cols}, "
                       f"{prob.nnz} nonzeros, FP64, one pass per column group, {n_workgroups or 'all'} workgroups, "
                       f"{['given', 'independent'][column_order]} column order",
           "c_star": c_star, "sweeps": {}}
    with sccs.Handle(prob, n_workgroups=n_workgroups, merge_passes=0, column_order=column_order) as h:
        h.set_prior(kind, var)
        h.group_timing(True)
        order = h.column_order()   # sweep position -> column
        c, p = c[order], p[order]
        beta_prev = np.zeros(prob.n_cols)
        for s in range(1, max(sweeps_at) + 1):
            h.sweep(1)
            beta, _ = h.get_beta()
            if s not in sweeps_at:
                beta_prev = beta
                continue
            t, fc = h.group_times()
            moved = (beta != beta_prev)[order]
            beta_prev = beta
            dt = np.diff(np.concatenate([[0.0], t]))
            ng = len(dt)
            gc = np.array([c[fc[g]:fc[g + 1]].sum() for g in range(ng)])
            ga = np.array([phase_a_bytes(c[fc[g]:fc[g + 1]], p[fc[g]:fc[g + 1]], 0) for g in range(ng)])
            gbb = np.array([phase_b_bytes(c[fc[g]:fc[g + 1]], p[fc[g]:fc[g + 1]], moved[fc[g]:fc[g + 1]], 0)
                            for g in range(ng)])
            gb = ga + np.concatenate([[0.0], gbb[:-1]])
            gbs = gb / (dt * 1e-6) / 1e9
            buckets = []
            lo = 1
            while lo <= gc.max():
                sel = (gc >= lo) & (gc < 2 * lo)
                if sel.any():
                    buckets.append({"nnz_from": int(lo), "nnz_to": int(2 * lo - 1), "groups": int(sel.sum()),
                                    "median_us": float(np.median(dt[sel])),
                                    "median_GBs": float(np.median(gbs[sel])),
                                    "sum_GBs": float(gb[sel].sum() / (dt[sel].sum() * 1e-6) / 1e9)})
                lo *= 2
            big = gc >= c_star
            frac_big = float(gb[big].sum() / (dt[big].sum() * 1e-6) / 1e9 / HBM_PEAK_GBS) if big.any() else None
            out["sweeps"][str(s)] = {
                "sweep_ms": float(t[-1] * 1e-3), "groups": ng, "moved_columns": int(moved.sum()),
                "groups_at_or_above_c_star": int(big.sum()),
                "nnz_share_at_or_above_c_star": float(gc[big].sum() / gc.sum()),
                "time_share_at_or_above_c_star": float(dt[big].sum() / dt.sum()),
                "frac_of_peak_at_or_above_c_star": frac_big,
                "whole_sweep_GBs": float(gb.sum() / (t[-1] * 1e-6) / 1e9),
                "buckets": buckets}
            print(f"[bench] coordinate curve, sweep {s}: {t[-1] * 1e-3:.2f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--late", type=int, default=20,
                    help="sweeps timed after the headline ones, continuing the fit (0 = none)")
    ap.add_argument("--patients", type=int, default=2_000_000)
    ap.add_argument("--cols", type=int, default=2000)
    ap.add_argument("--cpu-sweeps", type=int, default=12)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=["mid", "outcomes", "cv", "full", "paper", "valued", "bootstrap", "search"],
                    default="mid")
    ap.add_argument("--tune", action="store_true", help="run the autotuner on the mid workload and print its table")
    ap.add_argument("--mixed-only", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--print-sha", action="store_true", help="print the sweep kernel's source hash and exit")
    ap.add_argument("--cv-max-sweeps", type=int, default=50)
    ap.add_argument("--column-order", type=int, choices=[0, 1], default=1,
                    help="0 the problem's column order, 1 the library's independence relabelling")
    ap.add_argument("--no-given", action="store_true", help="skip the given-order comparison run")
    ap.add_argument("--batch-engine", type=int, choices=[0, 1], default=0,
                    help="batched workloads: 0 fits on disjoint workgroup ranges, 1 all fits in lockstep")
    ap.add_argument("--cv-tol", type=float, default=1e-8)
    ap.add_argument("--coord-curve", action="store_true",
                    help="per-coordinate achieved bandwidth against column size (mid or full workload)")
    # The single fit is bound by its chain of device-wide reductions, not by
    # bandwidth: on mid, 128 persistent workgroups (16 per XCD, half the CUs)
    # finish a sweep about 2 % sooner than one per CU, because each
    # reduction has half the members.  0 = one workgroup per CU.
    ap.add_argument("--workgroups", type=int, default=128)
    # the mixed form (one pass per group throughout) is fastest on every CU
    ap.add_argument("--mixed-workgroups", type=int, default=0)
    # sweeps between exact recomputations of the FP32 weights in the mixed
    # form (-1: the library's default, every sweep)
    ap.add_argument("--mixed-refresh", type=int, default=-1)
    args = ap.parse_args()
    if args.print_sha:
        print(kernel_source_sha())
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(patient sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_1208_0945_amd import sccs, synth
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "outcomes":
        for prec in ((1,) if args.mixed_only else (0, 1)):
            print(json.dumps(batched_outcomes_bench(sccs, synth, args.steps, prec, args.batch_engine,
                                                    args.column_order)), flush=True)
        return
    if args.tune:
        prob = synth.mid(n_patients=args.patients, n_cols=args.cols)
        best, table = sccs.tune(prob, sccs.PRIOR_LAPLACE, 2.0, n_sweeps=3)
        print(json.dumps({"tune_best": best, "candidates": table}), flush=True)
        return
    if args.coord_curve:
        print(json.dumps(coord_curve(sccs, synth, args.workload, args.workgroups if args.workload == "mid" else 0,
                                     column_order=args.column_order)), flush=True)
        return
    if args.workload == "valued":
        print(json.dumps(valued_bench(sccs, synth, args.steps)), flush=True)
        return
    if args.workload == "bootstrap":
        print(json.dumps(bootstrap_bench(sccs, synth)), flush=True)
        return
    if args.workload == "search":
        print(json.dumps(search_bench(sccs, synth)), flush=True)
        return
    if args.workload == "paper":
        print(json.dumps(paper_fit_bench(sccs, synth, column_order=args.column_order)), flush=True)
        return
    if args.workload == "full":
        print(json.dumps(full_bench(sccs, synth, args.steps, refit=not args.no_cpu, column_order=args.column_order)),
              flush=True)
        return
    if args.workload == "cv":
        print(json.dumps(cv_bench(sccs, synth, 1 if args.mixed_only else 0, args.cv_max_sweeps, args.cv_tol,
                                  engine=args.batch_engine, column_order=args.column_order)), flush=True)
        return

    t0 = time.perf_counter()
    prob = synth.mid(n_patients=args.patients, n_cols=args.cols)
    print(f"[bench] generated {prob.summary()} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    c, p = column_stats(prob)

    fp = run_form(sccs, prob, 0, args.steps, args.warmup, c, p, args.workgroups, late=args.late,
                  column_order=args.column_order)
    print(f"[bench] fp64 done: {args.steps / fp['wall_s']:.1f} sweeps/s", file=sys.stderr, flush=True)
    ms = float(np.mean(fp["kernel_ms"]))
    algo = float(np.mean(fp["bytes"]))
    achieved = algo / (ms * 1e-3) / 1e9

    def sched(r):
        return {"passes_per_sweep_mean": float(np.mean([q[0] for q in r["passes"]])),
                "passes_last_sweep": int(r["passes"][-1][0]),
                "rejected_merges_per_sweep_mean": float(np.mean([q[1] for q in r["passes"]])),
                "zero_step_share_mean": float(np.mean([q[2] for q in r["passes"]])) / prob.n_cols,
                "us_per_pass_mean": 1e3 * float(np.sum(r["kernel_ms"])) / float(np.sum([q[0] for q in r["passes"]])),
                "kernel_ms_per_sweep": [round(x, 4) for x in r["kernel_ms"]]}
    out = {
        "metric": METRIC,
        "value": args.steps / fp["wall_s"],
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"mid SCCS: {prob.n_patients} patients, {prob.n_rows} eras, J={prob.n_cols} "
                               f"Zipf(1.1) drugs, {prob.nnz} nonzeros, Laplace lambda=1, FP64; "
                               f"sweeps 1..{args.steps} from beta = 0, one sweep per step",
                   "n_patients": prob.n_patients, "n_eras": prob.n_rows, "n_cols": prob.n_cols,
                   "nnz": prob.nnz, "prior": "laplace", "variance": 2.0, "parallelism": "single GPU",
                   "n_workgroups": args.workgroups,
                   # Algorithm 1 cycles over the drugs in a fixed order; with
                   # "independent" the library numbers them so that runs of
                   # consecutive drugs share no patient (same data, same sweeps)
                   "column_order": ["given", "independent"][args.column_order]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic(ms),
                     "kernel": ("k_ccd<double, false> (one pass per column group)" if args.column_order else
                                "k_ccd<double, *> (one-pass-per-group and merged-pass forms)"), "kernel_ms_mean": ms,
                     "algo_bytes_per_launch": algo,
                     "byte_model": "per coordinate 12 c_j + 16 p_j, plus 28 c_j + 8 p_j when its step is "
                                   "nonzero (c_j nonzeros, p_j patients of column j)",
                     "achieved_library_bytes": float(np.mean(fp["bytes_lib"])) / (ms * 1e-3) / 1e9,
                     "library_byte_model": "per coordinate 16 c_j + 16 p_j, plus 8 c_j + 8 p_j when its step is "
                                           "nonzero (what this kernel moves: (row, patient) pairs, 16-byte "
                                           "(den, omega n) gathers, multiplicative w update)",
                     # the sweep is a chain of device-wide reductions (one per
                     # pass): their latency, not HBM bandwidth, sets its time
                     "limiter": "latency of the chain of device-wide reductions, one per pass"},
        "schedule": sched(fp),
    }
    if args.late:
        lt = fp["late"]
        lms = float(np.mean(lt["kernel_ms"]))
        out["late_sweeps"] = {"sweeps": f"{args.steps + 1}..{args.steps + args.late}",
                              "value": args.late / lt["wall_s"], "unit": "sweeps/s", "kernel_ms_mean": lms,
                              "achieved_GBs": float(np.mean(lt["bytes"])) / (lms * 1e-3) / 1e9,
                              "schedule": sched(lt)}
    if args.column_order and not args.no_given:
        gv = run_form(sccs, prob, 0, args.steps, args.warmup, c, p, args.workgroups, column_order=0)
        gms = float(np.mean(gv["kernel_ms"]))
        out["given_order"] = {"value": args.steps / gv["wall_s"], "unit": "sweeps/s", "kernel_ms_mean": gms,
                              "achieved_GBs": float(np.mean(gv["bytes"])) / (gms * 1e-3) / 1e9,
                              "schedule": sched(gv),
                              "note": "same workload and schedule, drugs visited in the problem's own order"}
        print(f"[bench] given order: {out['given_order']['value']:.1f} sweeps/s", file=sys.stderr, flush=True)
    if not args.no_mixed:
        mx = run_form(sccs, prob, 1, args.steps, args.warmup, c, p, args.mixed_workgroups,
                      refresh_period=args.mixed_refresh, column_order=args.column_order)
        err = float(np.max(np.abs(mx["beta"] - fp["beta"])) / max(np.max(np.abs(fp["beta"])), 1e-300))
        mms = float(np.mean(mx["kernel_ms"]))
        out["mixed"] = {"value": args.steps / mx["wall_s"], "unit": "sweeps/s",
                        "kernel_ms_mean": mms,
                        "achieved_GBs": float(np.mean(mx["bytes"])) / (mms * 1e-3) / 1e9,
                        "rel_err_vs_fp64_gpu": err,
                        "n_workgroups": args.mixed_workgroups,
                        "refresh_period": args.mixed_refresh,
                        "sweeps_compared": f"1..{args.steps} from beta = 0"}
        print(f"[bench] mixed done: {out['mixed']['value']:.1f} sweeps/s, rel err {err:.2e}",
              file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
