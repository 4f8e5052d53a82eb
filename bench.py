#!/usr/bin/env python
"""Benchmark of the DIA kernel fit on one MI355X.

Workload (default): the CCD-sized pair — 4096 x 4096, 80,000 stars, Moffat PSF
(beta 3, FWHM 3.5 px), fluxes log-uniform 1e2..1e6, sky 500; target = reference
correlated with a 19 x 19 elliptical Gaussian (FWHM 2.2 x 1.8 px, 30 deg,
sum 0.9) plus B0 = -12, read noise 8 e-, gain 1.5.  Objective: chi-squared with
CCD variance from the data.  Inputs are synthetic and seeded; they are
resident in HBM before timing starts.

A step is one complete fit (flat kernel, B0 = median; Adam, then L-BFGS on
the paper's schedule, then the exact-Hessian Newton polish): every optimiser
iteration is one fused forward + objective + backward pass plus the FP64
reduction and the optimiser update.

Printed (one JSON line): fwd+bwd Gtap/s sustained through the timed fits
(value), fits/s, evaluations per fit, the fused kernel's roofline fraction
(its duration measured with HIP events around a captured graph of back-to-back
loss/gradient calls on the launch stream, each call the widening of theta, the
fused pass and the reduction), the FP64 CPU oracle timed on
a bounded sample of the same pair, and ("batched") the split-precision bf16x3
matrix-core form on 256 epochs of 2048^2 against one shared reference (m = 25)
beside the plain form on the first 32 of them: fits/s, evaluations per fit and
the fraction of the BF16 MFMA / FP64 vector peak; and ("many_small_pairs") 158
EMCCD-like targets of one 482^2 field, m = 19, Huber loss with the EMCCD model
variance: per-image solution times (median, 16th and 84th percentiles) from the
box-car and Gaussian starts and the MAP fit, and the batched fits/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DIA kernel fits/s & fwd+bwd Gtap/s at 4096², m=19; % of roofline vs plain"
# The fused pass computes in FP64 (FP32 inputs widened exactly).  MI355X FP64 vector peak:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s.
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_BF16_MFMA_TFLOPS = 2500.0  # dense


def make_batch(args, sf):
    """The batched workload's synthetic inputs, made before anything touches the GPU (the epochs are
    built on threads of this process; each has its own random stream, so the batch is the same)."""
    t0 = time.time()
    workers = min(16, os.cpu_count() or 1)
    if args.batch_workload == "emccd":
        b = sf.config_emccd(n_epochs=args.emccd_epochs, size=max(int(x) for x in args.emccd_sizes.split(",")),
                            m=max(int(x) for x in args.emccd_m.split(",")), workers=workers)
    elif args.batch_workload == "uneven":
        b = sf.config4(n_epochs=args.batch_epochs, workers=workers)
    else:
        b = sf.config5(n_epochs=args.batch_epochs, workers=workers)
    print(f"# generated {len(b.epochs)}-epoch batch in {time.time() - t0:.1f}s ({workers} threads)",
          file=sys.stderr, flush=True)
    return b


def oracle_golden(name, b, np):
    """The oracle's minimisers for this batch's epochs (tests/golden/make_batched_oracle.py), as
    {epoch: theta}, keeping only epochs whose target sums match the stored ones (the same seeded
    inputs); empty when the file is missing."""
    path = os.path.join(ROOT, "tests", "golden", "batched_oracle_thetas.npz")
    if not os.path.exists(path):
        return {}
    z = np.load(path)
    if f"{name}_epochs" not in z.files:
        return {}
    out = {}
    for e, th, sm in zip(z[f"{name}_epochs"], z[f"{name}_theta"], z[f"{name}_target_sum"]):
        e = int(e)
        if e < len(b.epochs) and float(np.sum(b.epochs[e].I, dtype=np.float64)) == float(sm):
            out[e] = th
    return out


def emccd_golden(b, np):
    """The oracle's minimisers for the targets of the many-small-pairs batch
    (tests/golden/make_emccd_oracle.py: 482^2, m = 19, lambda 0 and 1), as ({target: theta},
    {target: theta at lambda = 1}), keeping only targets whose image sums match the stored ones."""
    path = os.path.join(ROOT, "tests", "golden", "emccd_oracle_thetas.npz")
    if not os.path.exists(path):
        return {}, {}
    z = np.load(path)
    if int(z["size"]) != b.R.shape[0]:
        return {}, {}
    g0, g1 = {}, {}
    for k, sm in enumerate(z["target_sum"]):
        if k < len(b.epochs) and float(np.sum(b.epochs[k].I, dtype=np.float64)) == float(sm):
            g0[k], g1[k] = z["theta"][k], z["theta_lam1"][k]
    return g0, g1


def fit_errors(theta, res, gold, m, np):
    """Per-fit error against the oracle's minimiser for the epochs in gold: ||dK||/||K||, |dP|/|P| (P of
    the fit's FP64 iterate), |dB0|/max(|B0|, 1); max and median over those epochs."""
    th = theta.detach().cpu().double().numpy()
    eK, eP, eB = [], [], []
    for e, ref in gold.items():
        if e >= th.shape[0]:
            continue
        Kr = ref[:m * m]
        eK.append(float(np.linalg.norm(th[e, :m * m] - Kr) / np.linalg.norm(Kr)))
        eP.append(abs(res[e].P - Kr.sum()) / abs(Kr.sum()))
        eB.append(abs(res[e].B0 - ref[-1]) / max(abs(ref[-1]), 1.0))
    if not eK:
        return None
    f = lambda x, q: float(f"{np.percentile(x, q):.3g}")
    return {"epochs_checked": len(eK), "K_rel_max": f(eK, 100), "K_rel_median": f(eK, 50), "P_rel_max": f(eP, 100),
            "P_rel_median": f(eP, 50), "B0_rel_max": f(eB, 100), "B0_rel_median": f(eB, 50),
            "within_1e-4": bool(max(eK) <= 1e-4 and max(eP) <= 1e-4 and max(eB) <= 1e-4)}


def batched_section(args, b, dia, torch, dev, np):
    """The batched workload (epochs of 2048^2 against one shared 2048^2 reference, m = 25): one batched fit
    and a burst of batched loss/gradient evaluations in each precision.  The plain form runs on the first
    --batch-plain-epochs epochs of the same batch.  Each fit's error against the oracle's minimiser is
    reported for the epochs that tests/golden/make_batched_oracle.py solved."""
    uneven = args.batch_workload == "uneven"
    m = b.m
    R = torch.from_numpy(b.R).to(dev)
    eps_all = [dia.Epoch(I=torch.from_numpy(e.I).to(dev), ref_row0=e.row0, ref_col0=e.col0) for e in b.epochs]
    obj = dia.Objective(rho="gauss", var="ccd_data", sigma0=b.sigma0_adu, gain=b.gain)
    n_all = len(eps_all)
    side = b.R.shape[0]
    Ps_all = [(e.I.shape[0] - m + 1) * (e.I.shape[1] - m + 1) for e in b.epochs]
    th_all = torch.from_numpy(np.stack([np.r_[e.K_true.ravel(), e.B0_true] for e in b.epochs]).astype(np.float32)).to(dev)
    ws = dia.Workspace(dev)
    if uneven:
        wl = (f"{n_all} epochs of side {min(e.I.shape[0] for e in b.epochs)}..{max(e.I.shape[0] for e in b.epochs)} "
              f"cut from one shared {side}x{side} reference, m={m}, chi2 with CCD data variance")
    else:
        wl = (f"{n_all} epochs x {side}x{side} against one shared {side}x{side} reference, m={m}, "
              f"chi2 with CCD data variance")
    out = {"workload": wl, "epochs": n_all, "valid_pixels": int(sum(Ps_all))}
    gold = oracle_golden("c4" if uneven else "c5", b, np)
    if args.profile_batched:
        for _ in range(args.kernel_reps):
            dia.loss_grad_batched(R, eps_all, th_all, m, obj, precision=args.profile_batched, workspace=ws)
        torch.cuda.synchronize()
        return out
    for prec in [p for p in args.batch_precisions.split(",") if p]:
        n = n_all if prec == "bf16x3" else min(n_all, args.batch_plain_epochs)
        eps, th = eps_all[:n], th_all[:n].contiguous()
        flop = 4.0 * sum(Ps_all[:n]) * m * m  # forward + backward, one FMA (2 FLOP) per tap, every epoch
        for _ in range(2):
            dia.loss_grad_batched(R, eps, th, m, obj, precision=prec, workspace=ws)
        torch.cuda.synchronize()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        a.record()
        for _ in range(reps):
            dia.loss_grad_batched(R, eps, th, m, obj, precision=prec, workspace=ws)
        z.record()
        torch.cuda.synchronize()
        t_eval = a.elapsed_time(z) / 1e3 / reps
        torch.cuda.synchronize()
        a.record()
        theta, res, st = dia.fit_batched(R, eps, m, obj, precision=prec, workspace=ws)
        z.record()
        torch.cuda.synchronize()
        t_fit = a.elapsed_time(z) / 1e3
        ev = [r.n_eval for r in res]
        alg = flop / t_eval / 1e12
        rec = {"epochs": n, "fits_per_s": round(n / t_fit, 3), "fit_s": round(t_fit, 2),
               "evals_per_fit_max": int(max(ev)), "evals_per_fit_mean": round(float(np.mean(ev)), 1),
               "eval_ms": round(1e3 * t_eval, 3), "algorithmic_tflops": round(alg, 2), "status": st,
               "stops": sorted({r.stop for r in res}),
               "first_order_stops": {k: sum(1 for r in res if r.first_order_stop == k)
                                     for k in sorted({r.first_order_stop for r in res})},
               "n_adam_mean": round(float(np.mean([r.n_adam for r in res])), 1),
               "n_lbfgs_mean": round(float(np.mean([r.n_lbfgs for r in res])), 1),
               "n_newton_mean": round(float(np.mean([r.n_newton for r in res])), 2),
               "error_vs_oracle": fit_errors(theta, res, gold, m, np)}
        if prec == "bf16x3":
            rec["mfma_tflops"] = round(3 * alg, 2)
            rec["roofline"] = {"bound": "mfma", "achieved": round(3 * alg, 2), "peak": PEAK_BF16_MFMA_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(3 * alg / PEAK_BF16_MFMA_TFLOPS, 4)}
        else:
            rec["roofline"] = {"bound": "alu", "achieved": round(alg, 2), "peak": PEAK_FP64_VECTOR_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(alg / PEAK_FP64_VECTOR_TFLOPS, 4)}
        out["plain" if prec in ("fp32", "plain") else prec] = rec
        print(f"# batched {prec}: {rec}", file=sys.stderr, flush=True)
    return out


def sf_fwhm_per_sigma():
    import math
    return 2.0 * math.sqrt(2.0 * math.log(2.0))


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x, dtype=np.float64), q)) if len(x) else float("nan")


def emccd_section(args, b, dia, torch, dev, np):
    """Many small aligned pairs shaped like the EMCCD speed test of Section 5.1: n targets of one field
    against the sharpest image as reference, Huber loss with the EMCCD model variance and the flat
    field, central crops of each side in --emccd-sizes, each kernel size in --emccd-m.  Per image:
    the single-pair fit's solution time (median and 16th / 84th percentiles over the targets, the
    paper's statistic) from a flat box-car and from a Gaussian of width sqrt(phi_I^2 - phi_R^2); the
    Spearman rank correlation of solution time with phi_I; then the whole set as one batched fit in
    each precision (fits/s)."""
    from scipy.stats import spearmanr
    full = b.R.shape[0]
    phi_I = np.asarray(b.meta["phi_I"])
    # the Gaussian start's standard deviation from the FWHM difference sqrt(phi_I^2 - phi_R^2)
    phi_K = np.sqrt(np.maximum(phi_I ** 2 - b.meta["phi_R"] ** 2, 0.25)) / sf_fwhm_per_sigma()
    ws = dia.Workspace(dev)
    gold0, gold1 = emccd_golden(b, np)
    gold_m = 19
    out = {"workload": (f"{len(b.epochs)} targets of one {full}x{full} field (2000 stars, Gaussian PSF of FWHM "
                        f"{b.meta['phi_R']}) and the shared flat, Huber loss with EMCCD model variance "
                        f"(E = {b.meta['excess']}, G = {b.gain})"), "cases": []}
    ev = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    for size in [int(x) for x in args.emccd_sizes.split(",")]:
        r0 = (full - size) // 2
        sl = (slice(r0, r0 + size), slice(r0, r0 + size))
        R = torch.from_numpy(np.ascontiguousarray(b.R[sl])).to(dev)
        Fc = torch.from_numpy(np.ascontiguousarray(b.meta["flat"][sl])).to(dev)
        Is = [torch.from_numpy(np.ascontiguousarray(e.I[sl])).to(dev) for e in b.epochs]
        obj = dia.Objective(rho="huber", var="emccd_model", gain=b.gain, excess=b.meta["excess"], flat=Fc)
        objr = dia.Objective(rho="huber", var="emccd_model", gain=b.gain, excess=b.meta["excess"], flat=Fc,
                             lam=args.emccd_lambda)
        for m in [int(x) for x in args.emccd_m.split(",")]:
            case = {"size": size, "m": m}
            # errors against the oracle's minimisers where they exist (the full field at m = 19)
            g0, g1 = (gold0, gold1) if size == full and m == gold_m else ({}, {})
            dia.fit(R, Is[0], m, obj, workspace=ws)  # warm the tile-shape choice and the workspace
            torch.cuda.synchronize()
            case["tile_shape"] = dict(zip(("variant", "rows", "cols"), dia.tile_shape(m, size, size)))
            if args.emccd_lambda > 0:
                # the Laplacian-regularised (MAP) fit of Section 2.7 from the box-car start
                t_ms, n_ev, knorm, rs = [], [], [], []
                for k, I in enumerate(Is):
                    a, z = ev()
                    a.record()
                    r = dia.fit(R, I, m, objr, workspace=ws)
                    z.record()
                    torch.cuda.synchronize()
                    t_ms.append(a.elapsed_time(z))
                    n_ev.append(r.n_eval)
                    knorm.append(float(r.theta[:m * m].norm()))
                    rs.append(r)
                case["single_flat_lambda"] = {"lambda": args.emccd_lambda, "median_ms": round(_pct(t_ms, 50), 2),
                                              "p16_ms": round(_pct(t_ms, 16), 2), "p84_ms": round(_pct(t_ms, 84), 2),
                                              "evals_median": int(_pct(n_ev, 50)),
                                              "kernel_norm_median": round(_pct(knorm, 50), 4)}
                if args.emccd_lambda == 1.0 and g1:
                    case["single_flat_lambda"]["error_vs_oracle"] = fit_errors(
                        torch.stack([r.theta for r in rs]), rs, g1, m, np)
            for init in ("flat", "gauss"):
                t_ms, n_ev, knorm, rs = [], [], [], []
                for k, I in enumerate(Is):
                    a, z = ev()
                    a.record()
                    r = dia.fit(R, I, m, obj, workspace=ws, init=init, init_phi=float(phi_K[k]))
                    z.record()
                    torch.cuda.synchronize()
                    t_ms.append(a.elapsed_time(z))
                    n_ev.append(r.n_eval)
                    knorm.append(float(r.theta[:m * m].norm()))
                    rs.append(r)
                rho_s = spearmanr(t_ms, phi_I).statistic
                case[f"single_{init}"] = {"median_ms": round(_pct(t_ms, 50), 2), "p16_ms": round(_pct(t_ms, 16), 2),
                                          "p84_ms": round(_pct(t_ms, 84), 2),
                                          "evals_median": int(_pct(n_ev, 50)), "evals_p16": int(_pct(n_ev, 16)),
                                          "evals_p84": int(_pct(n_ev, 84)), "spearman_time_phi_I": round(float(rho_s), 2),
                                          "kernel_norm_median": round(_pct(knorm, 50), 4)}
                if g0:
                    case[f"single_{init}"]["error_vs_oracle"] = fit_errors(torch.stack([r.theta for r in rs]), rs,
                                                                           g0, m, np)
            eps = [dia.Epoch(I=I, flat=Fc) for I in Is]
            n = len(eps)
            yy, xx = np.mgrid[:m, :m] - (m - 1) / 2.0
            kg = np.exp(-0.5 * (xx[None] ** 2 + yy[None] ** 2) / phi_K[:, None, None] ** 2)
            kg /= kg.sum(axis=(1, 2), keepdims=True)
            th_g = torch.from_numpy(kg.reshape(n, -1).astype(np.float32)).to(dev)
            th_g = torch.cat([th_g, torch.stack([I.median() for I in Is])[:, None]], 1).contiguous()
            for prec in ("plain", "bf16x3"):
                for init in ("flat", "gauss"):
                    th0 = th_g.clone() if init == "gauss" else None
                    torch.cuda.synchronize()
                    a, z = ev()
                    a.record()
                    th, res, st = dia.fit_batched(R, eps, m, obj, theta=th0, precision=prec, workspace=ws)
                    z.record()
                    torch.cuda.synchronize()
                    t = a.elapsed_time(z) / 1e3
                    e_ = [r.n_eval for r in res]
                    stops = {}
                    for r in res:
                        stops[r.stop] = stops.get(r.stop, 0) + 1
                    case[f"batched_{prec}_{init}"] = {"fits_per_s": round(n / t, 1), "fit_s": round(t, 3),
                                                      "evals_median": int(_pct(e_, 50)), "evals_max": int(max(e_)),
                                                      "status": st, "stops": stops}
                    if g0:
                        case[f"batched_{prec}_{init}"]["error_vs_oracle"] = fit_errors(th, res, g0, m, np)
            out["cases"].append(case)
            print(f"# emccd {case}", file=sys.stderr, flush=True)
    return out


def traffic_from_profile(kernel_sig: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it matches this kernel build."""
    path = os.path.join(ROOT, "profiles", "traffic_fused_eval_4096_m19.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha") != kernel_sig:
        return None
    return rec.get("bytes_per_launch")


def kernel_source_sig() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("dia_common.h", "tile_impl.h"):
        h.update(open(os.path.join(ROOT, "paper_2104_13715_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--init", default="flat", choices=["flat", "gauss"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--newton-schedule", type=int, default=1,
                    help="1: also time the exact-Hessian schedule (Adam to 1e-4, then Newton) on the same pair")
    ap.add_argument("--cpu-rows", type=int, default=1024, help="valid rows of the oracle's timed sample")
    ap.add_argument("--cpu-b08-rows", type=int, default=96,
                    help="valid rows of the band on which the oracle's normal matrix is timed")
    ap.add_argument("--batch-epochs", type=int, default=256,
                    help="epochs of the batched split-precision workload (2048^2 each, m = 25); 0 skips it")
    ap.add_argument("--batch-plain-epochs", type=int, default=32,
                    help="the plain form (FP32 data, FP64 arithmetic on the vector ALUs) of the batched workload "
                         "runs on this many of its epochs")
    ap.add_argument("--batch-precisions", default="bf16x3,plain")
    ap.add_argument("--batch-workload", default="shared", choices=["shared", "uneven", "emccd"],
                    help="shared: epochs of 2048^2 on one shared window (m = 25); uneven: sides 512..2048 cut "
                         "from a shared 2048^2 reference (m = 17, plain form only); emccd: many small aligned "
                         "pairs, Huber loss with the EMCCD noise model (printed alone)")
    ap.add_argument("--emccd-epochs", type=int, default=158)
    ap.add_argument("--small-pairs", type=int, default=1,
                    help="1: add the many-small-pairs section (first of --emccd-sizes / --emccd-m) to the line")
    ap.add_argument("--emccd-sizes", default="482,242", help="central crop sides of the emccd workload")
    ap.add_argument("--emccd-m", default="19,25", help="kernel sizes of the emccd workload")
    ap.add_argument("--emccd-lambda", type=float, default=1.0,
                    help="also time the Laplacian-regularised fit with this lambda (0 skips it)")
    ap.add_argument("--only-batched", action="store_true", help="print the batched section alone")
    ap.add_argument("--profile-batched", default="",
                    help="only run --kernel-reps batched evaluations in this precision (for hardware-counter runs)")
    ap.add_argument("--profile-kernel", action="store_true",
                    help="only run --kernel-reps fused passes and a 256 MiB device copy (for hardware-counter runs; "
                         "the copy calibrates FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path, so --gpus must be 1 "
              "(the value is that GPU's throughput)", file=sys.stderr)
        return 2

    import numpy as np
    from synthetic import starfield as sf

    # the batch first: its worker processes start before this process loads the GPU runtime
    batch = make_batch(args, sf) if args.batch_epochs > 0 and not args.profile_kernel else None
    # the many-small-pairs workload at its first crop and kernel size, as a section of the line
    small = None
    if args.small_pairs and args.batch_workload != "emccd" and not (args.only_batched or args.profile_batched
                                                                      or args.profile_kernel):
        t0 = time.time()
        small = sf.config_emccd(n_epochs=args.emccd_epochs, size=int(args.emccd_sizes.split(",")[0]),
                                m=int(args.emccd_m.split(",")[0]), workers=min(16, os.cpu_count() or 1))
        print(f"# generated the many-small-pairs batch in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    import torch

    import paper_2104_13715_amd as dia

    dev = torch.device("cuda:0")
    if args.batch_workload == "emccd":
        print(json.dumps({"emccd": emccd_section(args, batch, dia, torch, dev, np)}))
        return 0
    if args.only_batched:
        print(json.dumps({"batched": batched_section(args, batch, dia, torch, dev, np)}))
        return 0
    if args.profile_batched:
        batched_section(args, batch, dia, torch, dev, np)
        print(json.dumps({"profile_batched": args.profile_batched, "evaluations": args.kernel_reps}))
        return 0
    t0 = time.time()
    pair = sf.config3(size=args.size)
    m = pair.m
    print(f"# generated {args.size}^2 pair in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    R = torch.from_numpy(pair.R).to(dev)
    I = torch.from_numpy(pair.I).to(dev)
    obj = dia.Objective(rho="gauss", var="ccd_data", sigma0=pair.sigma0_adu, gain=pair.gain)
    H, W = pair.I.shape
    P = (H - m + 1) * (W - m + 1)
    taps_per_eval = 2 * P * m * m  # forward + backward (pixel, tap) products, one FMA each
    ws = dia.Workspace(dev)
    torch.cuda.synchronize()

    if args.profile_kernel:
        th = torch.from_numpy(np.r_[sf.kernel_gaussian(m, 2.2, 1.8, rot_deg=30.0, total=0.9).ravel(),
                                    -12.0].astype(np.float32)).to(dev)
        for _ in range(args.kernel_reps):
            dia.loss_grad(R, I, th, m, obj, ws)
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"profile_kernel": True, "fused_passes": args.kernel_reps, "copy_bytes": 4 * x.numel()}))
        return 0

    fit_kw = dict(init=args.init, init_phi=1.0)
    for _ in range(args.warmup):
        dia.fit(R, I, m, obj, workspace=ws, **fit_kw)
        print("# warmup fit done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    # ------------------------------------------------------------------ timed region: K full fits
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_eval = 0
    results = []
    torch.cuda.synchronize()
    start.record()
    for k in range(args.steps):
        r = dia.fit(R, I, m, obj, workspace=ws, **fit_kw)
        n_eval += r.n_eval
        results.append(r)
    end.record()
    torch.cuda.synchronize()
    t_fit = start.elapsed_time(end) / 1e3
    print(f"# {args.steps} fits in {t_fit:.3f}s, evals {[r.n_eval for r in results]}", file=sys.stderr, flush=True)

    # one more fit from the Gaussian initialisation the paper uses in its speed tests (Section 5): standard
    # deviation sqrt(phi_I^2 - phi_R^2) from the two images' PSF widths (equivalent-circle FWHM of the
    # reference PSF, and of that PSF carried to the target, as a width measurement on the target's stars
    # returns), each converted to a Gaussian standard deviation
    from synthetic.starfield import FWHM_PER_SIGMA, equivalent_fwhm, gaussian_psf, moffat_psf
    psf = moffat_psf(pair.meta["fwhm"]) if pair.meta["psf"] == "moffat" else gaussian_psf(pair.meta["fwhm"])
    phi_R = equivalent_fwhm(psf) / FWHM_PER_SIGMA
    phi_I = equivalent_fwhm(psf, pair.K_true) / FWHM_PER_SIGMA
    phi_k = float(np.sqrt(max(phi_I ** 2 - phi_R ** 2, 0.25)))
    torch.cuda.synchronize()
    gi0 = time.time()
    rg = dia.fit(R, I, m, obj, workspace=ws, init="gauss", init_phi=phi_k)
    torch.cuda.synchronize()
    t_gauss = time.time() - gi0

    # accuracy of the timed fit, and of the same schedule without the Newton polish (the Adam -> L-BFGS
    # point the polish starts from), against the oracle's minimiser of this pair (tests/golden/make_c3_fit.py)
    fit_err = first_order_err = None
    gpath = os.path.join(ROOT, "tests", "golden", "c3_chi2_oracle_theta.txt")
    if args.size == 4096 and os.path.exists(gpath):
        ref = np.loadtxt(gpath)

        def rel_errors(r):
            th = r.theta.cpu().double().numpy()
            Kr = ref[:m * m]
            return {"K_rel": float(f"{np.linalg.norm(th[:m * m] - Kr) / np.linalg.norm(Kr):.3g}"),
                    "P_rel": float(f"{abs(r.P - Kr.sum()) / abs(Kr.sum()):.3g}"),
                    "B0_rel": float(f"{abs(r.B0 - ref[-1]) / max(abs(ref[-1]), 1.0):.3g}")}

        fit_err = rel_errors(results[-1])
        r1 = dia.fit(R, I, m, obj, workspace=ws, max_newton=0, **fit_kw)
        first_order_err = dict(rel_errors(r1), n_adam=r1.n_adam, n_lbfgs=r1.n_lbfgs, stop=r1.stop)
        print(f"# fit error {fit_err}, before the polish {first_order_err}", file=sys.stderr, flush=True)

    # the same pair fitted on the exact-Hessian schedule: Adam to a looser switch (1e-4), no L-BFGS phase,
    # then Newton steps (eq. newtonupdate with the exact FP64 Hessian) to convergence, chi-squared and
    # Cauchy, each against the oracle's minimiser (tests/golden/make_c3_fit.py)
    newton_sched = None
    if args.newton_schedule and args.size == 4096:
        newton_sched = {"options": {"tol_switch": 1e-4, "max_lbfgs": 0, "max_newton": 30, "init": args.init}}
        for rho, gname in (("gauss", "c3_chi2_oracle_theta.txt"), ("cauchy", "c3_cauchy_oracle_theta.txt")):
            o_r = dia.Objective(rho=rho, var="ccd_data", sigma0=pair.sigma0_adu, gain=pair.gain, c=2.3849)
            kw = dict(init=args.init, init_phi=1.0, tol_switch=1e-4, max_lbfgs=0, max_newton=30)
            dia.fit(R, I, m, o_r, workspace=ws, **kw)
            torch.cuda.synchronize()
            reps = 5
            t1 = time.time()
            for _ in range(reps):
                rn = dia.fit(R, I, m, o_r, workspace=ws, **kw)
            torch.cuda.synchronize()
            tn = (time.time() - t1) / reps
            rec = {"fits_per_s": round(1.0 / tn, 3), "evals": rn.n_eval, "n_adam": rn.n_adam, "n_newton": rn.n_newton,
                   "n_hessian": rn.n_hessian, "stop": rn.stop, "status": rn.status}
            gpath = os.path.join(ROOT, "tests", "golden", gname)
            if os.path.exists(gpath):
                ref = np.loadtxt(gpath)
                th = rn.theta.cpu().double().numpy()
                rec["K_rel_err"] = float(f"{np.linalg.norm(th[:m * m] - ref[:m * m]) / np.linalg.norm(ref[:m * m]):.3g}")
                rec["P_rel_err"] = float(f"{abs(rn.P - ref[:m * m].sum()) / abs(ref[:m * m].sum()):.3g}")
                rec["B0_rel_err"] = float(f"{abs(rn.B0 - ref[-1]) / max(abs(ref[-1]), 1.0):.3g}")
            newton_sched["chi2" if rho == "gauss" else "cauchy"] = rec
            print(f"# newton schedule {rho}: {rec}", file=sys.stderr, flush=True)

    # ------------------------------------------------------------------ kernel duration: back-to-back fused passes
    # kernel_reps dia_loss_grad calls (each: the FP64 widening of theta, the fused pass, the reduction) captured
    # in one graph on this stream and replayed, so that no host gap separates the launches (an eager burst is
    # bound by the Python call, and the clock drops in the gaps); every replay is checked against the eager loss
    theta = results[-1].theta.clone()
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty(m * m + 1, dtype=torch.float32, device=dev)
    for _ in range(3):
        dia.loss_grad(R, I, theta, m, obj, ws, loss, grad)
    torch.cuda.synchronize()
    L_eager = loss.item()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(args.kernel_reps):
            dia.loss_grad(R, I, theta, m, obj, ws, loss, grad)
    for _ in range(2):
        loss.zero_()
        graph.replay()
        torch.cuda.synchronize()
        if loss.item() != L_eager:
            raise RuntimeError(f"graph replay of the fused pass gave {loss.item()} instead of {L_eager}")
    kb, ke = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    kb.record()
    graph.replay()
    ke.record()
    torch.cuda.synchronize()
    t_launch = kb.elapsed_time(ke) / 1e3 / args.kernel_reps
    if loss.item() != L_eager:
        raise RuntimeError("timed graph replay of the fused pass disagrees with the eager loss")
    flop_per_launch = 2.0 * taps_per_eval
    achieved_tflops = flop_per_launch / t_launch / 1e12
    traffic = traffic_from_profile(kernel_source_sig())

    # ------------------------------------------------------------------ CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rows = min(args.cpu_rows, H - m + 1) + m - 1
        oobj = oracle.Objective(rho="gauss", var="ccd_data", sigma0=pair.sigma0_adu, gain=pair.gain)
        th = theta.cpu().numpy()
        Rs, Is = pair.R[:rows], pair.I[:rows]
        oracle.loss_grad(Rs[:m + 8], Is[:m + 8], th, m, oobj)  # load the library first
        ps = (rows - m + 1) * (W - m + 1)
        reps, tc = 0, 0.0
        while tc < 10.0 and reps < 50:
            t1 = time.time()
            oracle.loss_grad(Rs, Is, th, m, oobj)
            tc += time.time() - t1
            reps += 1
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        gtaps_cpu = reps * 2 * ps * m * m / tc / 1e9
        # the oracle's B08-style solve (the paper's comparator, Sections 5.1-5.2): the normal matrix
        # X^T W X (linear in the pixel count) timed on a band of rows and scaled to the whole pair, plus
        # its Cholesky factorisation and the three residual-refinement passes at the measured tap rate
        import scipy.linalg
        brows = min(args.cpu_b08_rows, H - m + 1)
        w = oracle.fixed_weights(oobj, pair.I[:brows + m - 1], m)
        t1 = time.time()
        A, _ = oracle.normal_matrix(pair.R[:brows + m - 1], m, w)
        t_nm = time.time() - t1
        t1 = time.time()
        scipy.linalg.cho_factor(A + np.eye(A.shape[0]) * 1e-300, lower=True)
        t_chol = time.time() - t1
        t_b08 = t_nm * P / (brows * (W - m + 1)) + t_chol + 3 * 2.0 * P * m * m / (gtaps_cpu * 1e9)
        model = "unknown"
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        cpu = {"value": round(gtaps_cpu, 4), "unit": "Gtap/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{reps} FP64 loss+gradient evaluations (direct loops) of the top {rows - m + 1} valid rows "
                         f"x {W - m + 1} columns of the same pair, m={m}",
               "cpu_model": model,
               "b08_solve": {"fits_per_s": round(1.0 / t_b08, 5), "seconds_per_fit": round(t_b08, 1),
                             "sample": f"normal matrix of the top {brows} valid rows ({t_nm:.2f} s) scaled to "
                                       f"{P} valid pixels, Cholesky ({t_chol * 1e3:.1f} ms), three refinement "
                                       f"passes at the measured tap rate"}}

    batched = batched_section(args, batch, dia, torch, dev, np) if batch is not None else None
    many_small = None
    if small is not None:
        sa = argparse.Namespace(**vars(args))
        sa.emccd_sizes, sa.emccd_m = args.emccd_sizes.split(",")[0], args.emccd_m.split(",")[0]
        many_small = emccd_section(sa, small, dia, torch, dev, np)

    gtaps = n_eval * taps_per_eval / t_fit / 1e9
    line = {
        "metric": METRIC,
        "value": round(gtaps, 2),
        "unit": "Gtap/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_fit / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded star field, resident in HBM)",
        "config": {"workload": f"single pair {H}x{W}, m={m}, chi2 with CCD data variance, {args.init} init, "
                               f"Adam then L-BFGS on the paper's schedule, then exact-Hessian Newton polish",
                   "H": H, "W": W, "m": m,
                   "valid_pixels": P, "objective": "gauss/ccd_data"},
        "fits_per_s": round(args.steps / t_fit, 3),
        "evals_per_fit": round(n_eval / args.steps, 1),
        "eval_us_in_fit": round(1e6 * t_fit / n_eval, 2),
        "fused_pass_us": round(1e6 * t_launch, 2),
        "kernel_gtaps": round(taps_per_eval / t_launch / 1e9, 1),
        "fit_stop": results[-1].stop,
        "fit_error_vs_oracle": fit_err,
        "first_order_error_vs_oracle": first_order_err,
        "tile_shape": dict(zip(("variant", "rows", "cols"), dia.tile_shape(m, H, W))),
        "fit_counts": {"n_adam": results[-1].n_adam, "n_lbfgs": results[-1].n_lbfgs,
                       "n_newton": results[-1].n_newton, "n_hessian": results[-1].n_hessian,
                       "first_order_stop": results[-1].first_order_stop},
        "gauss_init_fit": {"fits_per_s": round(1.0 / t_gauss, 3), "evals": rg.n_eval, "init_phi": round(phi_k, 4),
                           "phi_R": round(phi_R, 4), "phi_I": round(phi_I, 4), "n_adam": rg.n_adam,
                           "n_lbfgs": rg.n_lbfgs, "n_newton": rg.n_newton, "first_order_stop": rg.first_order_stop,
                           "stop": rg.stop},
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": PEAK_FP64_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_FP64_VECTOR_TFLOPS, 4),
                     "traffic": traffic},
        "newton_schedule": newton_sched,
        "cpu_baseline": cpu,
        "batched": batched,
        "many_small_pairs": many_small,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
