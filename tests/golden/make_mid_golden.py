"""Write the FP64 oracle's iterates on the mid workload (2M patients, ~20M
eras, J = 2000 Zipf(1.1) drugs, Laplace prior with variance 2, i.e.
lambda = 1), Algorithm 1 from beta = 0:

* tests/golden/mid_laplace_fp64.npz: the columns in the given order; beta
  and the trust bounds after 20 and after 100 sweeps, and the log posterior
  after every sweep;
* tests/golden/mid_laplace_fp64_independent.npz: the columns visited in the
  independence relabelling (oracle.independent_order, width 4); the order,
  and beta and the trust bounds after 20 sweeps in the problem's own column
  numbering.

Only the seeded generator and the oracle are called; the GPU tests
regenerate the same problem from its seeds.

    python tests/golden/make_mid_golden.py [--independent-only]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1208_0945_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "mid_laplace_fp64.npz")
OUT_IND = os.path.join(HERE, "mid_laplace_fp64_independent.npz")


def independent(prob):
    t0 = time.perf_counter()
    order = oracle.independent_order(prob, 4)
    perm = synth.permute_columns(prob, order)
    r20 = oracle.ccd(oracle.OracleProblem(perm), oracle.PRIOR_LAPLACE, 2.0, 20)
    print(f"relabelled: 20 sweeps in {time.perf_counter() - t0:.1f} s", flush=True)
    beta, trust = np.empty(prob.n_cols), np.empty(prob.n_cols)
    beta[order] = r20["beta"]
    trust[order] = r20["trust"]
    np.savez_compressed(OUT_IND, order=order, beta20=beta, trust20=trust,
                        seed_info=np.array(prob.seed_info), nnz=np.array(prob.nnz))
    print(OUT_IND)


def main():
    oracle.build(force=False)
    prob = synth.mid()
    independent(prob)
    if "--independent-only" in sys.argv:
        return
    P = oracle.OracleProblem(prob)
    t0 = time.perf_counter()
    r20 = oracle.ccd(P, oracle.PRIOR_LAPLACE, 2.0, 20)
    print(f"20 sweeps in {time.perf_counter() - t0:.1f} s", flush=True)
    t0 = time.perf_counter()
    r100 = oracle.ccd(P, oracle.PRIOR_LAPLACE, 2.0, 100)
    print(f"100 sweeps in {time.perf_counter() - t0:.1f} s", flush=True)
    np.savez_compressed(OUT, beta20=r20["beta"], trust20=r20["trust"], beta100=r100["beta"],
                        trust100=r100["trust"], logpost100=r100["logpost_trace"],
                        seed_info=np.array(prob.seed_info), nnz=np.array(prob.nnz))
    print(OUT)


if __name__ == "__main__":
    main()
