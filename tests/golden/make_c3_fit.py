"""Writes c3_chi2_oracle_theta.txt and c3_cauchy_oracle_theta.txt: the FP64 oracle's minimisers
for the seeded 4096^2 CCD-sized pair (80,000 stars, Moffat FWHM 3.5, m = 19) under the
chi-squared and the Cauchy loss (c = 2.3849), both with the CCD variance from the data
(sigma0 = 8 e-, gain 1.5).  Chi-squared: normal equations by Cholesky with three refinement
steps.  Cauchy: damped Newton on the exact Hessian from the chi-squared solution; the header
records whether the Hessian at the minimiser factors (positive definite, so the minimiser is
unique near it).  Calls only the oracle and the seeded input generator; several minutes of CPU.

    python tests/golden/make_c3_fit.py
"""
import os
import sys

import numpy as np
import scipy.linalg

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synthetic import starfield as sf  # noqa: E402

CAUCHY_C = 2.3849


def objective(p, rho):
    return oracle.Objective(rho=rho, var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain,
                            c=CAUCHY_C if rho == "cauchy" else 1.345)


def main():
    p = sf.config3()
    m = p.m
    for rho, name in (("gauss", "c3_chi2_oracle_theta.txt"), ("cauchy", "c3_cauchy_oracle_theta.txt")):
        oo = objective(p, rho)
        th = oracle.solve(p.R, p.I, m, oo, verbose=True)
        L, g = oracle.loss_grad(p.R, p.I, th, m, oo)
        H = oracle.hessian(p.R, p.I, th, m, oo)
        try:
            scipy.linalg.cho_factor(H, lower=True)
            pd = "positive definite"
        except np.linalg.LinAlgError:
            pd = "NOT positive definite"
        np.savetxt(os.path.join(HERE, name), th, fmt="%.17e",
                   header=f"oracle minimiser, seeded 4096^2 CCD-sized pair, m = {m}, rho = {rho}, CCD data "
                          f"variance: K row-major, then B0; loss {L:.17e}; max|grad| {np.max(np.abs(g)):.3e}; "
                          f"Hessian at the minimiser {pd}")
        print(name, "written", flush=True)


if __name__ == "__main__":
    main()
