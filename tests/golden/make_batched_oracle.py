"""Writes batched_oracle_thetas.npz: the FP64 oracle's minimisers (normal equations by Cholesky with
three refinement steps) for every epoch of the seeded 256 x 2048^2, m = 25 batch and for every eighth
epoch of the seeded 64-epoch uneven batch (sides 512..2048, m = 17), both chi-squared with the CCD
variance from the data (sigma0 = 8 e-, gain 1.5).  Each epoch is stored with the FP64 sum of its
target, so a reader can check that its own seeded inputs are the ones solved here.  Calls only the
oracle and the seeded input generator; about 40 s of CPU per 2048^2 epoch (8 cores).  Resumable:
epochs already in the file are kept.

    python tests/golden/make_batched_oracle.py [--only c5|c4]
"""
import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synthetic import starfield as sf  # noqa: E402

OUT = os.path.join(HERE, "batched_oracle_thetas.npz")
GAIN, SIGMA0_E = 1.5, 8.0
# (config, epochs in the batch, kernel size, reference side, stars, side range, epochs solved)
BATCHES = {
    "c5": (5, 256, 25, 2048, 40000, (2048, 2048), list(range(256))),
    "c4": (4, 64, 17, 2048, 30000, (512, 2048), list(range(0, 64, 8))),
}


def load():
    if not os.path.exists(OUT):
        return {}
    z = np.load(OUT)
    return {k: z[k] for k in z.files}


def save(d):
    tmp = OUT + ".tmp.npz"
    np.savez_compressed(tmp, **d)
    os.replace(tmp, OUT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="")
    a = ap.parse_args()
    d = load()
    oo = oracle.Objective(rho="gauss", var="ccd_data", sigma0=SIGMA0_E / GAIN, gain=GAIN)
    for name, (config, n_ep, m, ref, n_stars, sides, todo) in BATCHES.items():
        if a.only and a.only != name:
            continue
        R = sf.star_field(sf.rng_for(config, 0), ref, ref, n_stars, 1e2, 1e6, "moffat", 3.0, 500.0).astype(np.float32)
        R64 = R.astype(np.float64)
        done = list(d.get(f"{name}_epochs", np.zeros(0, np.int64)))
        thetas = list(d.get(f"{name}_theta", np.zeros((0, m * m + 1))))
        sums = list(d.get(f"{name}_target_sum", np.zeros(0)))
        for e in todo:
            if e in done:
                continue
            ep = sf._batched_epoch(config, e, R64, m, ref, sides, True, GAIN, SIGMA0_E)
            Rw = R[ep.row0:ep.row0 + ep.I.shape[0], ep.col0:ep.col0 + ep.I.shape[1]]
            th = oracle.solve(Rw, ep.I, m, oo)
            done.append(e)
            thetas.append(th)
            sums.append(float(np.sum(ep.I, dtype=np.float64)))
            d[f"{name}_epochs"] = np.asarray(done, np.int64)
            d[f"{name}_theta"] = np.asarray(thetas)
            d[f"{name}_target_sum"] = np.asarray(sums)
            d[f"{name}_batch"] = np.asarray([config, n_ep, m, ref, n_stars, sides[0], sides[1]], np.int64)
            save(d)
            print(f"{name} epoch {e} ({len(done)}/{len(todo)})", flush=True)


if __name__ == "__main__":
    main()
