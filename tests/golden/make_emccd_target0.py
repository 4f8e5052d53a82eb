"""Writes emccd_target0_oracle_theta.txt: the FP64 oracle's minimiser (damped Newton on the exact
Hessian) for target 0 of the seeded many-small-pairs EMCCD workload at full size (482^2 field,
m = 19, Huber loss with the EMCCD model variance and the shared flat).  Calls only the oracle and
the seeded input generator; a few minutes of CPU.

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


def objective(b):
    return oracle.Objective(rho="huber", var="emccd_model", gain=b.gain, excess=b.meta["excess"],
                            flat=b.meta["flat"].astype(np.float64))


def main():
    b, e = target()
    th = oracle.solve(b.R, e.I, M, objective(b))
    L = oracle.loss_grad(b.R, e.I, th, M, objective(b))[0]
    np.savetxt(os.path.join(HERE, "emccd_target0_oracle_theta.txt"), th, fmt="%.17e",
               header=f"oracle minimiser, target 0 of the seeded EMCCD workload ({SIZE}^2, m = {M}): "
                      f"K row-major, then B0; loss {L:.17e}")


if __name__ == "__main__":
    main()
