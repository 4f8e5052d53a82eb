"""Writes emccd_oracle_thetas.npz: the FP64 oracle's minimisers (damped Newton on the exact Hessian)
for every target of the seeded many-small-pairs EMCCD workload at its default size (158 targets of a
482^2 field, m = 19, Huber loss with the EMCCD model variance and the shared flat), without and with
the smoothness penalty at lambda = 1.  Each target is stored with the FP64 sum of its image, so a
reader can check that its own seeded inputs are the ones solved here.  Calls only the oracle and the
seeded input generator; about 13 s of CPU per solve, spread over worker processes.

    python tests/golden/make_emccd_oracle.py [--workers 6]
"""
import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

OUT = os.path.join(HERE, "emccd_oracle_thetas.npz")
N_TARGETS, SIZE, M = 158, 482, 19
LAMBDAS = (0.0, 1.0)


_BATCH = []


def batch():
    # made once per worker process
    if not _BATCH:
        from synthetic import starfield as sf
        _BATCH.append(sf.config_emccd(n_epochs=N_TARGETS, size=SIZE, m=M, workers=1))
    return _BATCH[0]


def solve_target(k):
    import oracle
    b = batch()
    e = b.epochs[k]
    out = []
    for lam in LAMBDAS:
        o = oracle.Objective(rho="huber", var="emccd_model", gain=b.gain, excess=b.meta["excess"],
                             flat=b.meta["flat"].astype(np.float64), lam=lam)
        out.append(oracle.solve(b.R, e.I, M, o))
    return k, float(np.sum(e.I, dtype=np.float64)), out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    a = ap.parse_args()
    # one BLAS thread per worker process
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    import multiprocessing as mp
    theta = np.zeros((len(LAMBDAS), N_TARGETS, M * M + 1))
    sums = np.zeros(N_TARGETS)
    with mp.get_context("spawn").Pool(a.workers) as pool:
        for n, (k, s, ths) in enumerate(pool.imap_unordered(solve_target, range(N_TARGETS))):
            sums[k] = s
            for i, th in enumerate(ths):
                theta[i, k] = th
            print(f"target {k} solved ({n + 1}/{N_TARGETS})", flush=True)
    tmp = OUT + ".tmp.npz"
    np.savez_compressed(tmp, size=SIZE, m=M, lambdas=np.array(LAMBDAS), target_sum=sums, theta=theta[0],
                        theta_lam1=theta[1])
    os.replace(tmp, OUT)


if __name__ == "__main__":
    main()
