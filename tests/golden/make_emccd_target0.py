"""Writes emccd_target0_oracle_theta.txt and emccd_target0_lam1_oracle_theta.txt: the FP64
oracle's minimisers (damped Newton on the exact Hessian) for target 0 of the seeded
many-small-pairs EMCCD workload at full size (482^2 field, m = 19, Huber loss with the EMCCD
model variance and the shared flat), without and with the smoothness penalty at lambda = 1.
Calls only the oracle and the seeded input generator; under a minute of CPU.

    python tests/golden/make_emccd_target0.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synthetic import starfield as sf  # noqa: E402

M, SIZE = 19, 482


def target():
    b = sf.config_emccd(n_epochs=1, size=SIZE, m=25)
    return b, b.epochs[0]


def objective(b, lam=0.0):
    return oracle.Objective(rho="huber", var="emccd_model", gain=b.gain, excess=b.meta["excess"],
                            flat=b.meta["flat"].astype(np.float64), lam=lam)


def main():
    b, e = target()
    for lam, name in ((0.0, "emccd_target0_oracle_theta.txt"), (1.0, "emccd_target0_lam1_oracle_theta.txt")):
        th = oracle.solve(b.R, e.I, M, objective(b, lam))
        L = oracle.loss_grad(b.R, e.I, th, M, objective(b, lam))[0]
        np.savetxt(os.path.join(HERE, name), th, fmt="%.17e",
                   header=f"oracle minimiser, target 0 of the seeded EMCCD workload ({SIZE}^2, m = {M}, "
                          f"lambda = {lam:g}): K row-major, then B0; loss {L:.17e}")


if __name__ == "__main__":
    main()
