"""Batched split-precision (bf16 x 3) implicit GEMM on the matrix cores, through the C ABI,
against the FP64 oracle epoch by epoch.

Tolerance, derived from the arithmetic (u = 2^-8 is the bf16 unit roundoff; the hi/lo split
represents an FP32 value to 2^-17 relative; the three-product form drops lo*lo, a 2^-18
relative term; MFMA accumulates in FP32, m*m + 1 terms per output):
  model      |dM_p| <= eps_m * Mabs_p,   eps_m = 4 * 2^-17 + (m*m + 1) * 2^-24,   Mabs = |K| (x) |R| + |B0|
  gradient   |d dL/dK_t| <= sum_p (|h_p| |dM_p| + eps_g |g_p|) |R_(p+t)|,  eps_g = 4 * 2^-17 + 256 * 2^-24
             (h = d2l/dM2; g is split like the operands; each tile sums 512 pixels in FP32)
  loss       |dL| <= sum_p (|g_p| |dM_p| + 16 * 2^-24 |l_p|)
             (the FP32 objective uses the hardware reciprocal, rsqrt and log, ~1 ulp each)
The fitted parameters come out of the FP64 Newton polish and meet the usual 1e-4 bar.
"""
import numpy as np
import pytest
import torch

import oracle
from synthetic import starfield as sf

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = torch.device("cuda:0")
U24 = 2.0 ** -24
EPS_SPLIT = 2.0 ** -17


@pytest.fixture(scope="module")
def dia():
    import paper_2104_13715_amd as d
    return d


def gpu(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def shared_batch(n, m, side, seed_cfg):
    # every epoch covers the whole (side x side) reference: the shared-window case of the GEMM path
    return sf.batched(seed_cfg, n, m, side, max(40, side * side // 120), (side, side))


def objs(dia, b, rho="gauss", var="ccd_data"):
    c = 2.3849
    o = dia.Objective(rho=rho, var=var, sigma0=b.sigma0_adu, gain=b.gain, c=c)
    oo = oracle.Objective(rho=rho, var=var, sigma0=b.sigma0_adu, gain=b.gain, c=c)
    return o, oo


def bounds(R, I, th, m, oo):
    th = np.asarray(th, np.float64)
    Mabs = oracle.model(np.abs(R.astype(np.float64)), np.abs(th), m)
    M = oracle.model(R, th, m)
    l, gp, h = oracle.pixel_terms(oo, oracle.valid(I.astype(np.float64), m), M, m)
    eps_m = 4 * EPS_SPLIT + (m * m + 1) * U24
    eps_g = 4 * EPS_SPLIT + 256 * U24
    dM = eps_m * Mabs
    wpix = np.abs(h) * dM + eps_g * np.abs(gp)
    gb = np.concatenate([oracle.grad_kernel(np.abs(R.astype(np.float64)), wpix, m).ravel(), [wpix.sum()]])
    lb = np.sum(np.abs(gp) * dM + 16 * U24 * np.abs(l))
    return gb, lb


@pytest.mark.parametrize("m,side,n,rho", [(9, 130, 40, "gauss"), (17, 150, 7, "cauchy"), (25, 120, 33, "gauss")])
def test_loss_grad_bf16x3_matches_oracle(dia, m, side, n, rho):
    b = shared_batch(n, m, side, 60 + m)
    o, oo = objs(dia, b, rho, "ccd_data" if rho == "gauss" else "ccd_model")
    th = np.stack([oracle.init_theta(e.I, m) * np.r_[np.full(m * m, 1.05), 1.0] for e in b.epochs]).astype(np.float32)
    ep = [dia.Epoch(I=gpu(e.I)) for e in b.epochs]
    loss, grad = dia.loss_grad_batched(gpu(b.R), ep, gpu(th), m, o, precision="bf16x3")
    torch.cuda.synchronize()
    loss = loss.cpu().numpy()
    grad = grad.cpu().double().numpy()
    worst = 0.0
    for k in sorted({0, n // 2, n - 1}):
        e = b.epochs[k]
        L_ref, g_ref = oracle.loss_grad(b.R, e.I, th[k], m, oo)
        gb, lb = bounds(b.R, e.I, th[k], m, oo)
        err = np.abs(grad[k] - g_ref)
        ratio = float(np.max(err / gb))
        worst = max(worst, ratio)
        assert np.all(err <= gb), (k, ratio)
        assert abs(loss[k] - L_ref) <= lb, (k, loss[k], L_ref, lb)
        print(f"epoch {k}: grad rel err {np.linalg.norm(err) / np.linalg.norm(g_ref):.2e}, "
              f"worst err / bound {ratio:.3f}, loss err {abs(loss[k] - L_ref):.3e} (bound {lb:.3e})")
    print(f"m={m} n={n}: worst error / bound {worst:.3f}")


MODES = [(r, v) for r in ("gauss", "huber", "cauchy")
         for v in ("weights", "ccd_data", "ccd_model", "emccd_data", "emccd_model")]


@pytest.mark.parametrize("rho,var", MODES)
def test_loss_grad_bf16x3_every_objective_mode(dia, rho, var):
    # every (rho, sigma source) pair; epoch 0 carries a flat field, epoch 1 a bad-pixel mask,
    # epoch 2 both, epoch 3 neither (null entries beside non-null ones in the same launch)
    m, side, n = 9, 76, 4
    b = shared_batch(n, m, side, 300 + 7 * MODES.index((rho, var)))
    rng = np.random.default_rng(11)
    c = {"gauss": 1.345, "huber": 1.345, "cauchy": 2.3849}[rho]
    th = np.stack([oracle.init_theta(e.I, m) * np.r_[np.full(m * m, 0.97), 1.0] for e in b.epochs]).astype(np.float32)
    L_ref, g_ref, gbs, lbs, ep = [], [], [], [], []
    for k, e in enumerate(b.epochs):
        flat = rng.uniform(0.9, 1.1, e.I.shape).astype(np.float32) if k in (0, 2) else None
        mask = (rng.random(e.I.shape) > 0.1).astype(np.uint8) if k in (1, 2) else None
        w = None
        if var == "weights":
            w = (1.0 / np.maximum(b.sigma0_adu ** 2 + np.maximum(e.I, 0) / b.gain, 1.0)).astype(np.float32)
        oo = oracle.Objective(rho=rho, var=var, sigma0=b.sigma0_adu, gain=b.gain, c=c, weights=w, flat=flat,
                              mask=mask)
        Lr, gr = oracle.loss_grad(b.R, e.I, th[k], m, oo)
        gb, lb = bounds(b.R, e.I, th[k], m, oo)
        L_ref.append(Lr), g_ref.append(gr), gbs.append(gb), lbs.append(lb)
        ep.append(dia.Epoch(I=gpu(e.I), weights=None if w is None else gpu(w),
                            flat=None if flat is None else gpu(flat),
                            mask=None if mask is None else gpu(mask, torch.uint8)))
    o = dia.Objective(rho=rho, var=var, sigma0=b.sigma0_adu, gain=b.gain, c=c)
    loss, grad = dia.loss_grad_batched(gpu(b.R), ep, gpu(th), m, o, precision="bf16x3")
    torch.cuda.synchronize()
    loss, grad = loss.cpu().numpy(), grad.cpu().double().numpy()
    for k in range(n):
        err = np.abs(grad[k] - g_ref[k])
        assert np.all(err <= gbs[k]), (k, float(np.max(err / gbs[k])))
        assert abs(loss[k] - L_ref[k]) <= lbs[k], (k, loss[k], L_ref[k], lbs[k])


def test_bf16x3_agrees_with_fp32_path(dia):
    m, side, n = 17, 140, 9
    b = shared_batch(n, m, side, 91)
    o, oo = objs(dia, b)
    th = np.stack([oracle.init_theta(e.I, m) for e in b.epochs]).astype(np.float32)
    ep = [dia.Epoch(I=gpu(e.I)) for e in b.epochs]
    L1, g1 = dia.loss_grad_batched(gpu(b.R), ep, gpu(th), m, o, precision="bf16x3")
    L2, g2 = dia.loss_grad_batched(gpu(b.R), ep, gpu(th), m, o, precision="fp32")
    g1, g2 = g1.cpu().double().numpy(), g2.cpu().double().numpy()
    for k in range(n):
        gb, _ = bounds(b.R, b.epochs[k].I, th[k], m, oo)
        assert np.all(np.abs(g1[k] - g2[k]) <= gb * 1.01 + 1e-6 * np.abs(g2[k]))


def test_fit_bf16x3_matches_oracle(dia):
    m, side, n = 9, 110, 5
    b = shared_batch(n, m, side, 97)
    o, oo = objs(dia, b)
    ep = [dia.Epoch(I=gpu(e.I)) for e in b.epochs]
    theta, res, st = dia.fit_batched(gpu(b.R), ep, m, o, precision="bf16x3")
    assert st >= 0
    th = theta.cpu().double().numpy()
    for k, e in enumerate(b.epochs):
        ref = oracle.solve(b.R, e.I, m, oo)
        K, Kr = th[k, :-1], ref[:-1]
        eK = np.linalg.norm(K - Kr) / np.linalg.norm(Kr)
        eP = abs(K.sum() - Kr.sum()) / abs(Kr.sum())
        eB = abs(th[k, -1] - ref[-1]) / max(abs(ref[-1]), 1.0)
        print(f"epoch {k}: K {eK:.2e} P {eP:.2e} B0 {eB:.2e} evals {res[k].n_eval} newton {res[k].n_newton} "
              f"stop {res[k].stop}")
        assert res[k].status >= 0
        assert eK <= 1e-4 and eP <= 1e-4 and eB <= 1e-4


def test_fit_bf16x3_more_epochs_than_a_block(dia):
    # 40 epochs: two launches of 32 slots at first; as epochs converge the unconverged ones are
    # gathered into one block (slots then hold arbitrary epoch indices)
    m, side, n = 9, 72, 40
    b = shared_batch(n, m, side, 98)
    o, oo = objs(dia, b)
    ep = [dia.Epoch(I=gpu(e.I)) for e in b.epochs]
    theta, res, st = dia.fit_batched(gpu(b.R), ep, m, o, precision="bf16x3")
    assert st >= 0
    th = theta.cpu().double().numpy()
    evals = [r.n_eval for r in res]
    print(f"evals per epoch: min {min(evals)} max {max(evals)}")
    for k, e in enumerate(b.epochs):
        ref = oracle.solve(b.R, e.I, m, oo)
        K, Kr = th[k, :-1], ref[:-1]
        eK = np.linalg.norm(K - Kr) / np.linalg.norm(Kr)
        eP = abs(K.sum() - Kr.sum()) / abs(Kr.sum())
        eB = abs(th[k, -1] - ref[-1]) / max(abs(ref[-1]), 1.0)
        assert res[k].status >= 0
        assert eK <= 1e-4 and eP <= 1e-4 and eB <= 1e-4, (k, eK, eP, eB)


def test_fit_full_size_epoch_at_gradient_noise_floor(dia):
    # epoch 246 of the seeded 256 x 2048^2, m = 25 batch at full size: its FP64 gradient reaches the
    # rounding floor of the 4.1 M-term sums while the Newton decrement is still above its bar; the
    # polish must declare convergence, and the fit must match the oracle's exact minimiser
    # (tests/golden/make_c5_epoch246.py) to the 1e-4 bar, in both precisions and the single-pair fit
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("c5_epoch246", os.path.join(here, "make_c5_epoch246.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    R, e = mod.epoch()
    ref = np.loadtxt(os.path.join(here, "c5_epoch246_oracle_theta.txt"))
    m = mod.M
    o = dia.Objective(rho="gauss", var="ccd_data", sigma0=mod.SIGMA0_E / mod.GAIN, gain=mod.GAIN)

    def errs(th):
        th = np.asarray(th, np.float64).ravel()
        K, Kr = th[:-1], ref[:-1]
        return (np.linalg.norm(K - Kr) / np.linalg.norm(Kr), abs(K.sum() - Kr.sum()) / abs(Kr.sum()),
                abs(th[-1] - ref[-1]) / max(abs(ref[-1]), 1.0))

    Rg, Ig = gpu(R), gpu(e.I)
    for prec in ("bf16x3", "fp32"):
        theta, res, st = dia.fit_batched(Rg, [dia.Epoch(I=Ig)], m, o, precision=prec)
        eK, eP, eB = errs(theta.cpu().numpy())
        print(f"{prec}: stop {res[0].stop} newton {res[0].n_newton} K {eK:.2e} P {eP:.2e} B0 {eB:.2e}")
        assert st == 0 and res[0].stop == "newton"
        assert eK <= 1e-4 and eP <= 1e-4 and eB <= 1e-4
    f = dia.fit(Rg, Ig, m, o)
    eK, eP, eB = errs(f.theta.cpu().numpy())
    assert f.status == 0 and f.stop == "newton"
    assert eK <= 1e-4 and eP <= 1e-4 and eB <= 1e-4


def test_bf16x3_rejects_unshared_windows_and_sizes(dia):
    b = sf.batched(92, 3, 9, 200, 300, (120, 160))  # different sides and offsets
    o, _ = objs(dia, b)
    ep = [dia.Epoch(I=gpu(e.I), ref_row0=e.row0, ref_col0=e.col0) for e in b.epochs]
    th = torch.zeros((3, 82), dtype=torch.float32, device=DEV)
    with pytest.raises(dia.DIAError) as ex:
        dia.loss_grad_batched(gpu(b.R), ep, th, 9, o, precision="bf16x3")
    assert ex.value.status == dia.E_SIZE
    b2 = shared_batch(2, 11, 60, 93)
    ep2 = [dia.Epoch(I=gpu(e.I)) for e in b2.epochs]
    with pytest.raises(dia.DIAError) as ex:
        dia.loss_grad_batched(gpu(b2.R), ep2, torch.zeros((2, 122), dtype=torch.float32, device=DEV), 11, o,
                              precision="bf16x3")
    assert ex.value.status == dia.E_ARG


def test_loss_grad_bf16x3_full_size_batch_sampled(dia):
    # the benchmarked launch: 32 epochs of 2048^2 against the shared 2048^2 reference, m = 25;
    # the first and last epochs are checked against the oracle (direct loops over 4.1 M pixels)
    b = sf.config5(n_epochs=32)
    m = b.m
    o, oo = objs(dia, b)
    th = np.stack([np.r_[e.K_true.ravel() * 1.02, e.B0_true] for e in b.epochs]).astype(np.float32)
    ep = [dia.Epoch(I=gpu(e.I)) for e in b.epochs]
    loss, grad = dia.loss_grad_batched(gpu(b.R), ep, gpu(th), m, o, precision="bf16x3")
    torch.cuda.synchronize()
    loss = loss.cpu().numpy()
    grad = grad.cpu().double().numpy()
    for k in (0, 31):
        e = b.epochs[k]
        L_ref, g_ref = oracle.loss_grad(b.R, e.I, th[k], m, oo)
        gb, lb = bounds(b.R, e.I, th[k], m, oo)
        err = np.abs(grad[k] - g_ref)
        print(f"epoch {k}: grad rel err {np.linalg.norm(err) / np.linalg.norm(g_ref):.2e}, "
              f"worst err / bound {np.max(err / gb):.3f}, loss err {abs(loss[k] - L_ref):.3e} (bound {lb:.3e})")
        assert np.all(err <= gb)
        assert abs(loss[k] - L_ref) <= lb
