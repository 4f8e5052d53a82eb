"""Exact Hessian (observed Fisher information, Section 2.5) and the Newton polish of a fit,
through the C ABI, against the FP64 oracle.

The Hessian of L is sum_p l''_p x_p x_p^T (M is affine in theta).  The GPU forms l''_p in FP64
from the FP64 model value of FP32 inputs (exactly widened), and the products and sums in FP64,
so it agrees with the oracle to a few FP64 rounding steps per term: the bar is 1e-9 of max |H|.
Fits are held to the spec bar (K, sum K, B0 within 1e-4 relative).
"""
import numpy as np
import pytest
import torch

import oracle
from synthetic import starfield as sf

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def dia():
    import paper_2104_13715_amd as d
    return d


def gpu(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def objs(dia, rho, var, sigma0, gain, weights=None, mask=None):
    c = 1.345 if rho == "huber" else 2.3849
    o_or = oracle.Objective(rho=rho, var=var, sigma0=sigma0, gain=gain, c=c,
                            weights=None if weights is None else weights.astype(np.float64), mask=mask)
    o_gpu = dia.Objective(rho=rho, var=var, sigma0=sigma0, gain=gain, c=c,
                          weights=None if weights is None else gpu(weights),
                          mask=None if mask is None else gpu(mask, torch.uint8))
    return o_or, o_gpu


def check_hessian(dia, R, I, theta, m, o_or, o_gpu, tol=1e-9):
    theta = np.asarray(theta, np.float32)
    H = dia.hessian(gpu(R), gpu(I), gpu(theta), m, o_gpu)
    torch.cuda.synchronize()
    H = H.cpu().numpy()
    Hr = oracle.hessian(R, I, theta.astype(np.float64), m, o_or)
    assert np.array_equal(H, H.T), "assembled Hessian is not exactly symmetric"
    err = np.max(np.abs(H - Hr)) / np.max(np.abs(Hr))
    print(f"hessian m={m} {R.shape}: max rel err {err:.2e}")
    assert err <= tol, f"Hessian max rel err {err:.3e} > {tol}"
    return H, Hr


@pytest.fixture(scope="module")
def c1():
    return sf.config1()


@pytest.mark.parametrize("rho,var", [("gauss", "ccd_data"), ("gauss", "ccd_model"), ("cauchy", "ccd_model"),
                                     ("huber", "ccd_data"), ("gauss", "emccd_model"), ("cauchy", "weights")])
def test_hessian_matches_oracle_config1(dia, c1, rho, var):
    p = c1
    w = None
    if var == "weights":
        w = (1.0 / (p.sigma0_adu ** 2 + np.maximum(p.I, 0.0) / p.gain)).astype(np.float32)
    o_or, o_gpu = objs(dia, rho, var, p.sigma0_adu, p.gain, weights=w)
    theta = oracle.init_theta(p.I, p.m)
    rng = np.random.default_rng(11)
    theta = theta * rng.uniform(0.8, 1.2, theta.size)  # away from any symmetric point
    check_hessian(dia, p.R, p.I, theta, p.m, o_or, o_gpu)


@pytest.mark.parametrize("m,H,W", [(1, 20, 30), (5, 67, 133), (19, 90, 150), (49, 100, 120)])
def test_hessian_kernel_sizes_and_ragged_tiles(dia, m, H, W):
    rng = np.random.default_rng(100 + m)
    R = rng.uniform(50.0, 3000.0, (H, W)).astype(np.float32)
    I = (R + rng.normal(0, 30.0, (H, W))).astype(np.float32)
    theta = rng.uniform(0.0, 2.0 / (m * m), m * m + 1)
    theta[-1] = 3.0
    mask = (rng.uniform(size=(H, W)) > 0.1).astype(np.uint8)
    o_or, o_gpu = objs(dia, "cauchy", "ccd_model", 5.0, 1.3, mask=mask)
    check_hessian(dia, R, I, theta, m, o_or, o_gpu)


def test_hessian_is_fisher_information_at_the_optimum(dia, c1):
    # For the Gaussian NLL with fixed variance the Hessian equals the Fisher information
    # sum_p x_p x_p^T / sigma_p^2 everywhere; at the fit its inverse gives the parameter covariance.
    p = c1
    o_or, o_gpu = objs(dia, "gauss", "ccd_data", p.sigma0_adu, p.gain)
    th = oracle.solve(p.R, p.I, p.m, o_or)
    H, _ = check_hessian(dia, p.R, p.I, th, p.m, o_or, o_gpu)
    Iv = oracle.valid(p.I.astype(np.float64), p.m)
    w = 1.0 / (p.sigma0_adu ** 2 + np.maximum(Iv, 0.0) / p.gain)
    F, _ = oracle.normal_matrix(p.R, p.m, w)
    assert np.max(np.abs(H - F)) <= 1e-9 * np.max(np.abs(F))
    cov = np.linalg.inv(H)
    assert np.all(np.diag(cov) > 0.0)


def check_fit(res, th_ref, m, tol=1e-4):
    th = res.theta.cpu().double().numpy()
    K, Kr = th[:m * m], th_ref[:m * m]
    eK = np.linalg.norm(K - Kr) / np.linalg.norm(Kr)
    eP = abs(K.sum() - Kr.sum()) / abs(Kr.sum())
    eB = abs(th[-1] - th_ref[-1]) / max(abs(th_ref[-1]), 1.0)
    msg = (f"K {eK:.2e} P {eP:.2e} B0 {eB:.2e} evals {res.n_eval} (adam {res.n_adam}, lbfgs {res.n_lbfgs}, "
           f"newton {res.n_newton}, hessians {res.n_hessian}) stop {res.stop}")
    print(msg)
    assert res.status >= 0
    assert eK <= tol and eP <= tol and eB <= tol, msg


def test_newton_finishes_a_capped_fit(dia, c1):
    # three Adam steps, then the polish alone: chi^2 with fixed variance is quadratic, so one exact
    # Newton step lands on the optimum and the next decrement is negligible.
    p = c1
    o_or, o_gpu = objs(dia, "gauss", "ccd_data", p.sigma0_adu, p.gain)
    res = dia.fit(gpu(p.R), gpu(p.I), p.m, o_gpu, max_eval=3, poll_every=1)
    assert res.status == dia.OK and res.stop == "newton" and res.n_hessian == 1
    check_fit(res, oracle.solve(p.R, p.I, p.m, o_or), p.m)


def test_fit_without_newton_reports_the_first_order_result(dia, c1):
    p = c1
    o_or, o_gpu = objs(dia, "gauss", "ccd_data", p.sigma0_adu, p.gain)
    res = dia.fit(gpu(p.R), gpu(p.I), p.m, o_gpu, max_newton=0)
    assert res.n_newton == 0 and res.n_hessian == 0 and res.stop != "newton"
    assert res.status >= 0


@pytest.mark.parametrize("rho,var", [("gauss", "ccd_data"), ("cauchy", "ccd_model")])
def test_fit_m19_crop_of_the_ccd_field(dia, rho, var):
    # m = 19 on a 256^2 crop of the CCD-sized field: the normal matrix has condition ~1e10,
    # where the first-order optimisers alone stop far from the optimum.
    p = sf.crop(sf.config3(size=1024), 256)
    o_or, o_gpu = objs(dia, rho, var, p.sigma0_adu, p.gain)
    res = dia.fit(gpu(p.R), gpu(p.I), p.m, o_gpu)
    check_fit(res, oracle.solve(p.R, p.I, p.m, o_or), p.m)


def test_fit_config2_full_size(dia):
    p = sf.config2()
    o_or, o_gpu = objs(dia, "gauss", "ccd_data", p.sigma0_adu, p.gain)
    res = dia.fit(gpu(p.R), gpu(p.I), p.m, o_gpu)
    check_fit(res, oracle.solve(p.R, p.I, p.m, o_or), p.m)
