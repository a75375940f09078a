"""Seeded synthetic era data for the self-controlled case series (SCCS) model.

This module only draws data.  It holds none of the fitting arithmetic (no
likelihood, gradient, Newton step or derived per-patient/per-column totals):
both the CPU oracle and the GPU path compute everything they need from the
raw arrays returned here.

Data model (Section 2.1 of the paper): patient i has K_i exposure eras; era k
has a length l_ik in days, a binary drug-exposure vector x_ik over J drugs and
an adverse-event count y_ik ~ Poisson(l_ik * exp(x_ik' beta) * rate).  The
cases-only design keeps only patients with n_i = sum_k y_ik >= 1; a patient
whose draw gives n_i = 0 has its count vector redrawn (eras, lengths and
exposures kept) until n_i >= 1.

The paper's claims data are proprietary; these generators stand in for them
with the shapes of the workloads the method is measured on:

* eras per patient  K_i = 1 + Poisson(mu)            (mu = 4 tiny, 9 otherwise)
* era length        l_ik ~ UniformInt[1, 365]
* exposure          x_ikj ~ Bernoulli(p_j), independent per era and drug;
                    p_j = p0 * rank_j^(-1.1) (Zipf popularity) with the ranks
                    given by a seeded permutation of the drug ids
* true effects      a few nonzero beta_j ~ Normal(0, var)
* counts            rate 1e-3 per day

Layout of a ``Problem`` (all numpy, C-contiguous):

* ``patient_ptr`` int64 [N+1]: eras of patient i are rows
  patient_ptr[i] .. patient_ptr[i+1]-1 (rows grouped by patient).
* ``offset`` int32 [K]: l_ik; ``count`` int32 [K]: y_ik.
* ``col_ptr`` int64 [J+1], ``row_idx`` int32 [nnz]: X in compressed column
  storage; rows strictly ascending inside each column; values are all one
  unless ``value`` (float64 [nnz]) holds non-binary covariate values.

Non-binary covariates (``valued``; the paper's discussion names dense
covariates such as baseline measurements): besides binary drugs, sparse
"dose" columns whose exposed eras carry a dose level, and dense columns
present on every era that vary within a patient (an age-like covariate,
baseline age plus elapsed time, standardised; a seasonal cosine of the era's
calendar position).  A covariate constant within a patient cancels from the
conditional likelihood, so only within-patient variation is generated.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

ROOT_SEED = 12080945
RATE_PER_DAY = 1e-3


@dataclasses.dataclass
class Problem:
    name: str
    n_patients: int
    patient_ptr: np.ndarray
    offset: np.ndarray
    count: np.ndarray
    n_cols: int
    col_ptr: np.ndarray
    row_idx: np.ndarray
    beta_true: np.ndarray
    seed_info: str = ""
    value: Optional[np.ndarray] = None   # float64 [nnz] covariate values (CSC order), None = binary

    @property
    def n_rows(self) -> int:
        return int(self.patient_ptr[-1])

    @property
    def nnz(self) -> int:
        return int(self.col_ptr[-1])

    def column(self, j: int) -> np.ndarray:
        return self.row_idx[self.col_ptr[j]:self.col_ptr[j + 1]]

    def summary(self) -> dict:
        c = np.diff(self.col_ptr)
        return {"name": self.name, "N": self.n_patients, "K": self.n_rows,
                "J": self.n_cols, "nnz": self.nnz,
                "col_nnz_min": int(c.min()) if len(c) else 0,
                "col_nnz_median": float(np.median(c)) if len(c) else 0.0,
                "col_nnz_max": int(c.max()) if len(c) else 0}


def _rng(*path: int) -> np.random.Generator:
    """Child generator addressed by a path of integers under the root seed."""
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=tuple(int(p) for p in path))
    return np.random.Generator(np.random.PCG64(ss))


def _bernoulli_rows(rng: np.random.Generator, n_rows: int, p: float) -> np.ndarray:
    """Sorted row indices of an independent Bernoulli(p) column of length n_rows.

    Drawn as a geometric-gap process, which gives exactly the distribution of
    n_rows independent Bernoulli draws while costing O(nnz) draws.
    """
    if p <= 0.0 or n_rows == 0:
        return np.zeros(0, dtype=np.int32)
    if p >= 1.0:
        return np.arange(n_rows, dtype=np.int32)
    chunks = []
    pos = -1
    expect = n_rows * p
    batch = int(expect + 6.0 * math.sqrt(expect + 1.0) + 64)
    while True:
        gaps = rng.geometric(p, size=batch).astype(np.int64)
        rows = pos + np.cumsum(gaps)
        if rows[-1] >= n_rows:
            chunks.append(rows[rows < n_rows])
            break
        chunks.append(rows)
        pos = int(rows[-1])
        batch = max(64, int((n_rows - pos) * p * 1.2) + 64)
    return np.concatenate(chunks).astype(np.int32)


def make_problem(name: str, n_patients: int, n_cols: int, era_mean: float,
                 incl_prob: Sequence[float], beta_true: np.ndarray,
                 seed_path: Sequence[int], rate: float = RATE_PER_DAY,
                 max_len: int = 365) -> Problem:
    """Draw one cases-only SCCS problem.

    incl_prob[j] is the per-era exposure probability of drug j; beta_true[j]
    its true log relative incidence.
    """
    incl_prob = np.asarray(incl_prob, dtype=np.float64)
    beta_true = np.asarray(beta_true, dtype=np.float64)
    assert incl_prob.shape == (n_cols,) and beta_true.shape == (n_cols,)
    rng_eras = _rng(*seed_path, 0)
    k_i = 1 + rng_eras.poisson(era_mean, size=n_patients).astype(np.int64)
    patient_ptr = np.zeros(n_patients + 1, dtype=np.int64)
    np.cumsum(k_i, out=patient_ptr[1:])
    n_rows = int(patient_ptr[-1])
    offset = rng_eras.integers(1, max_len + 1, size=n_rows, dtype=np.int32)

    cols: List[np.ndarray] = []
    for j in range(n_cols):
        cols.append(_bernoulli_rows(_rng(*seed_path, 1, j), n_rows, float(incl_prob[j])))
    col_ptr = np.zeros(n_cols + 1, dtype=np.int64)
    np.cumsum([len(c) for c in cols], out=col_ptr[1:])
    row_idx = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)

    # true linear predictor per era (data model only)
    eta_true = np.zeros(n_rows, dtype=np.float64)
    for j in np.flatnonzero(beta_true):
        eta_true[cols[j]] += beta_true[j]
    mean = offset.astype(np.float64) * np.exp(eta_true) * rate

    rng_y = _rng(*seed_path, 2)
    count = rng_y.poisson(mean).astype(np.int32)
    pid = np.repeat(np.arange(n_patients, dtype=np.int64), k_i)
    # redraw the count vector of every patient without an event
    todo = np.flatnonzero(np.bincount(pid, weights=count, minlength=n_patients) == 0)
    rounds = 0
    while todo.size:
        rows = _rows_of(patient_ptr, todo)
        count[rows] = rng_y.poisson(mean[rows]).astype(np.int32)
        tot = np.bincount(np.searchsorted(patient_ptr, rows, side="right") - 1,
                          weights=count[rows], minlength=n_patients)[todo]
        todo = todo[tot == 0]
        rounds += 1
        if rounds > 1_000_000:
            raise RuntimeError("count redraw did not terminate")
    return Problem(name=name, n_patients=n_patients, patient_ptr=patient_ptr,
                   offset=offset, count=count, n_cols=n_cols, col_ptr=col_ptr,
                   row_idx=row_idx, beta_true=beta_true,
                   seed_info=f"root={ROOT_SEED} path={tuple(seed_path)}")


def valued(n_patients: int = 5000, n_drugs: int = 40, n_dose: int = 6, n_dense: int = 2, seed: int = 0,
           era_mean: float = 6.0) -> Problem:
    """Cases-only SCCS data with non-binary covariates: n_drugs binary drugs
    (Zipf popularity, p0 = 0.1), n_dose sparse dose columns (exposed with
    probability 0.1, dose ~ lognormal(0, 0.5)), and n_dense dense columns on
    every era (even index: age-like, (baseline age + elapsed years - 50) / 10
    with baseline ~ U[20, 80]; odd index: cos(2 pi t / 365) at the era's
    midpoint t in days since the patient's first era).  Columns are ordered
    drugs, doses, dense.  True effects: 8 drugs ~ N(0, 0.5), every dose
    column ~ N(0, 0.2), dense columns 0.3 and -0.2 alternately."""
    path = (10, seed)
    rng = _rng(*path, 9)
    J = n_drugs + n_dose + n_dense
    probs = zipf_probs(n_drugs, 0.1, 1.1, rng)
    beta = np.zeros(J)
    beta[:n_drugs] = sparse_beta(n_drugs, min(8, n_drugs), 0.5, rng)
    beta[n_drugs:n_drugs + n_dose] = rng.normal(0.0, math.sqrt(0.2), size=n_dose)
    beta[n_drugs + n_dose:] = [0.3 if c % 2 == 0 else -0.2 for c in range(n_dense)]
    rng_eras = _rng(*path, 0)
    k_i = 1 + rng_eras.poisson(era_mean, size=n_patients).astype(np.int64)
    patient_ptr = np.zeros(n_patients + 1, dtype=np.int64)
    np.cumsum(k_i, out=patient_ptr[1:])
    K = int(patient_ptr[-1])
    offset = rng_eras.integers(1, 366, size=K, dtype=np.int32)
    pid = np.repeat(np.arange(n_patients, dtype=np.int64), k_i)
    # days from the patient's first era to each era's midpoint
    start = np.cumsum(offset.astype(np.float64)) - offset
    start -= start[patient_ptr[:-1]][pid]
    mid_t = start + 0.5 * offset
    cols, vals = [], []
    for j in range(n_drugs):
        r = _bernoulli_rows(_rng(*path, 1, j), K, float(probs[j]))
        cols.append(r)
        vals.append(np.ones(len(r)))
    for c in range(n_dose):
        g = _rng(*path, 3, c)
        r = _bernoulli_rows(g, K, 0.1)
        cols.append(r)
        vals.append(np.exp(g.normal(0.0, 0.5, size=len(r))))
    base_age = _rng(*path, 4).uniform(20.0, 80.0, size=n_patients)
    for c in range(n_dense):
        cols.append(np.arange(K, dtype=np.int32))
        if c % 2 == 0:
            vals.append((base_age[pid] + mid_t / 365.0 - 50.0) / 10.0)
        else:
            vals.append(np.cos(2.0 * math.pi * mid_t / 365.0))
    col_ptr = np.zeros(J + 1, dtype=np.int64)
    np.cumsum([len(c) for c in cols], out=col_ptr[1:])
    row_idx = np.concatenate(cols).astype(np.int32)
    value = np.concatenate(vals).astype(np.float64)
    eta_true = np.zeros(K)
    for j in range(J):
        eta_true[cols[j]] += beta[j] * vals[j]
    mean = offset.astype(np.float64) * np.exp(eta_true) * RATE_PER_DAY
    rng_y = _rng(*path, 2)
    count = rng_y.poisson(mean).astype(np.int32)
    todo = np.flatnonzero(np.bincount(pid, weights=count, minlength=n_patients) == 0)
    while todo.size:
        rows = _rows_of(patient_ptr, todo)
        count[rows] = rng_y.poisson(mean[rows]).astype(np.int32)
        tot = np.bincount(pid[rows], weights=count[rows], minlength=n_patients)[todo]
        todo = todo[tot == 0]
    return Problem(name="valued", n_patients=n_patients, patient_ptr=patient_ptr, offset=offset, count=count,
                   n_cols=J, col_ptr=col_ptr, row_idx=row_idx, beta_true=beta,
                   seed_info=f"root={ROOT_SEED} path={path}", value=value)


def _rows_of(patient_ptr: np.ndarray, pats: np.ndarray) -> np.ndarray:
    lo = patient_ptr[pats]
    hi = patient_ptr[pats + 1]
    lens = hi - lo
    starts = np.repeat(lo - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    return starts + np.arange(int(lens.sum()))


def zipf_probs(n_cols: int, p0: float, exponent: float, rng: np.random.Generator) -> np.ndarray:
    """Per-drug exposure probability p0 * rank^-exponent with permuted ranks."""
    ranks = rng.permutation(n_cols) + 1
    return p0 * ranks.astype(np.float64) ** (-exponent)


def sparse_beta(n_cols: int, n_nonzero: int, var: float, rng: np.random.Generator) -> np.ndarray:
    beta = np.zeros(n_cols, dtype=np.float64)
    idx = rng.choice(n_cols, size=min(n_nonzero, n_cols), replace=False)
    beta[idx] = rng.normal(0.0, math.sqrt(var), size=len(idx))
    return beta


# ---------------------------------------------------------------- workloads

def tiny(n_patients: int = 1000, n_cols: int = 20, seed: int = 0) -> Problem:
    """1,000 patients, 1+Poisson(4) eras, J=20 drugs at p=0.05, 5 true effects
    ~N(0, 0.5) (variance)."""
    rng = _rng(1, seed, 9)
    beta = sparse_beta(n_cols, 5, 0.5, rng)
    return make_problem("tiny", n_patients, n_cols, 4.0, np.full(n_cols, 0.05), beta,
                        seed_path=(1, seed))


def zipf_problem(name: str, n_patients: int, n_cols: int, p0: float, seed_path: Sequence[int],
                 era_mean: float = 9.0, n_effects: int = 50, effect_var: float = 0.7,
                 exponent: float = 1.1) -> Problem:
    rng = _rng(*seed_path, 9)
    probs = zipf_probs(n_cols, p0, exponent, rng)
    beta = sparse_beta(n_cols, n_effects, effect_var, rng)
    return make_problem(name, n_patients, n_cols, era_mean, probs, beta, seed_path=seed_path)


def mid(n_patients: int = 2_000_000, n_cols: int = 2000, seed: int = 0) -> Problem:
    """2M patients, ~20M eras (1+Poisson(9)), J=2000 Zipf(1.1) drugs with
    p_j = 0.1 rank^-1.1, 50 true effects ~N(0, 0.7)."""
    return zipf_problem("mid", n_patients, n_cols, 0.1, seed_path=(2, seed))


def full(n_patients: int = 10_000_000, n_cols: int = 4000, seed: int = 0) -> Problem:
    """10M patients, ~100M eras, J=4000 Zipf drugs with p_j = 0.482 rank^-1.1."""
    return zipf_problem("full", n_patients, n_cols, 0.482, seed_path=(3, seed))


def paper_shaped(n_patients: int = 3_600_000, n_cols: int = 1428, seed: int = 0) -> Problem:
    """The size of the paper's largest dataset (Section 4: 3.6M cases-only
    patients, 75M exposure eras, 1428 drugs), with the mid generator's drug
    popularity: eras 1 + Poisson(19.83) per patient (~20.8 on average, so
    K ~ 75M), p_j = 0.1 rank^-1.1, 50 true effects ~N(0, 0.7).  The real
    claims data are not available; only the sizes are the paper's."""
    return zipf_problem("paper", n_patients, n_cols, 0.1, seed_path=(9, seed), era_mean=19.83)


def outcome_sizes(n_fits: int = 64, lo: float = 1e4, hi: float = 2e6, seed: int = 0) -> np.ndarray:
    rng = _rng(4, seed, 99)
    return np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_fits))).astype(np.int64)


def outcome_vocabulary(n_cols: int = 1000, seed: int = 0) -> np.ndarray:
    """Per-drug exposure probabilities shared by every outcome of a batch."""
    return zipf_probs(n_cols, 0.1, 1.1, _rng(4, seed, 9))


def outcome(f: int, n_patients: int, n_cols: int = 1000, seed: int = 0,
            probs: Optional[np.ndarray] = None) -> Problem:
    """Outcome f of a batch over one shared vocabulary: the same problem that
    batched_outcomes returns at position f for this size."""
    if probs is None:
        probs = outcome_vocabulary(n_cols, seed)
    beta = sparse_beta(n_cols, 50, 0.7, _rng(4, seed, 10, f))
    return make_problem(f"outcome{f}", int(n_patients), n_cols, 9.0, probs, beta, seed_path=(4, seed, f))


def batched_outcomes(n_fits: int = 64, n_cols: int = 1000, seed: int = 0,
                     sizes: Optional[Sequence[int]] = None, progress=None) -> List[Problem]:
    """Independent outcomes over one shared J-drug vocabulary (shared Zipf
    popularity), patient counts log-uniform 10k..2M."""
    if sizes is None:
        sizes = outcome_sizes(n_fits, seed=seed)
    probs = outcome_vocabulary(n_cols, seed)
    out = []
    for f, n in enumerate(sizes):
        out.append(outcome(f, int(n), n_cols, seed, probs))
        if progress is not None:
            progress(f)
    return out


def cv_folds(n_patients: int, n_folds: int = 10, seed: int = 0) -> np.ndarray:
    """Patient-level fold id (0..n_folds-1), a seeded balanced assignment."""
    rng = _rng(5, seed)
    return (rng.permutation(n_patients) % n_folds).astype(np.int32)


def bootstrap_weights(n_patients: int, n_reps: int, seed: int = 0) -> np.ndarray:
    """[n_reps, n_patients] patient multiplicities of seeded bootstrap
    resamples (n_patients draws with replacement each)."""
    rng = _rng(7, seed)
    return np.stack([np.bincount(rng.integers(0, n_patients, size=n_patients), minlength=n_patients)
                     for _ in range(n_reps)]).astype(np.int32)


def prior_grid(n: int = 16, lo: float = 1e-3, hi: float = 10.0) -> np.ndarray:
    """Prior variances log-spaced from lo to hi, ascending."""
    return np.logspace(math.log10(lo), math.log10(hi), n)


def subsample_patients(prob: Problem, frac: float, seed: int = 0) -> Problem:
    """The sub-problem made of a seeded fraction of the patients (all their
    eras), with rows and columns renumbered; data selection only."""
    rng = _rng(6, seed)
    keep = np.sort(rng.choice(prob.n_patients, size=max(1, int(round(frac * prob.n_patients))), replace=False))
    lens = np.diff(prob.patient_ptr)[keep]
    ptr = np.zeros(len(keep) + 1, dtype=np.int64)
    np.cumsum(lens, out=ptr[1:])
    rows = _rows_of(prob.patient_ptr, keep)            # old row of each new row
    new_of_old = np.full(prob.n_rows, -1, dtype=np.int64)
    new_of_old[rows] = np.arange(len(rows))
    mapped = new_of_old[prob.row_idx]
    col = np.repeat(np.arange(prob.n_cols), np.diff(prob.col_ptr))
    sel = mapped >= 0
    col_ptr = np.zeros(prob.n_cols + 1, dtype=np.int64)
    np.cumsum(np.bincount(col[sel], minlength=prob.n_cols), out=col_ptr[1:])
    return Problem(name=f"{prob.name}_sub{frac:g}", n_patients=len(keep), patient_ptr=ptr,
                   offset=prob.offset[rows].copy(), count=prob.count[rows].copy(), n_cols=prob.n_cols,
                   col_ptr=col_ptr, row_idx=mapped[sel].astype(np.int32), beta_true=prob.beta_true.copy(),
                   seed_info=prob.seed_info + f" subsample={frac} seed={seed}")


def random_beta(n_cols: int, scale: float, seed: int) -> np.ndarray:
    """A seeded coefficient vector for evaluating derivatives away from zero."""
    return _rng(7, seed).normal(0.0, scale, size=n_cols)


def permute_columns(prob: Problem, order) -> Problem:
    """The problem with its columns renumbered: column k of the result is
    column order[k] of prob (values follow their entries); data layout only."""
    order = np.asarray(order, dtype=np.int64)
    lens = np.diff(prob.col_ptr)[order]
    col_ptr = np.zeros(prob.n_cols + 1, dtype=np.int64)
    np.cumsum(lens, out=col_ptr[1:])
    src = np.concatenate([np.arange(prob.col_ptr[j], prob.col_ptr[j + 1]) for j in order]) if prob.nnz else \
        np.zeros(0, dtype=np.int64)
    return Problem(name=f"{prob.name}_perm", n_patients=prob.n_patients, patient_ptr=prob.patient_ptr,
                   offset=prob.offset, count=prob.count, n_cols=prob.n_cols, col_ptr=col_ptr,
                   row_idx=prob.row_idx[src].copy(), beta_true=prob.beta_true[order].copy(),
                   seed_info=prob.seed_info + " columns permuted",
                   value=None if prob.value is None else prob.value[src].copy())
