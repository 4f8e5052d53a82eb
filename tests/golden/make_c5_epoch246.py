"""Writes c5_epoch246_oracle_theta.txt: the FP64 oracle's minimiser (normal equations by Cholesky
with three refinement steps) for epoch 246 of the seeded 256 x 2048^2, m = 25 batch (chi-squared
with CCD data variance, sigma0 = 8 e-, gain 1.5).  Calls only the oracle and the seeded input
generator; about a minute of CPU.

    python tests/golden/make_c5_epoch246.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synthetic import starfield as sf  # noqa: E402

CONFIG, EPOCH, M, REF, N_STARS = 5, 246, 25, 2048, 40000
GAIN, SIGMA0_E = 1.5, 8.0


def epoch():
    R = sf.star_field(sf.rng_for(CONFIG, 0), REF, REF, N_STARS, 1e2, 1e6, "moffat", 3.0, 500.0).astype(np.float32)
    e = sf._batched_epoch(CONFIG, EPOCH, R.astype(np.float64), M, REF, (REF, REF), True, GAIN, SIGMA0_E)
    return R, e


def main():
    R, e = epoch()
    oo = oracle.Objective(rho="gauss", var="ccd_data", sigma0=SIGMA0_E / GAIN, gain=GAIN)
    th = oracle.solve(R, e.I, M, oo)
    np.savetxt(os.path.join(HERE, "c5_epoch246_oracle_theta.txt"), th, fmt="%.17e",
               header=f"oracle minimiser, epoch {EPOCH} of the seeded {REF}^2, m = {M} batch: K row-major, then B0")


if __name__ == "__main__":
    main()
