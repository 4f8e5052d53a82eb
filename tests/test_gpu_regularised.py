"""Laplacian-regularised (MAP) fits of Section 2.7 through the C ABI, against the FP64 oracle.

The loss gains lambda N_data theta^T L^T L theta (eq. regularised_loss, L of eq. laplacian over
the kernel pixels, N_data the valid-region pixel count).  The GPU adds the penalty's value and
gradient in FP64 in the reduction that follows the fused pass, and 2 lambda N_data L L to the
assembled Hessian; bars as for the unregularised forms: loss 1e-10 and gradient 1e-5 relative,
Hessian 1e-9 of max |H|, fits 1e-4 on K, P and B0.
"""
import numpy as np
import pytest
import torch

import oracle
from synthetic import starfield as sf

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = torch.device("cuda:0")
CASES = [("gauss", "ccd_data", 0.1), ("gauss", "ccd_data", 30.0), ("huber", "emccd_model", 1.0),
         ("cauchy", "ccd_model", 0.5)]


@pytest.fixture(scope="module")
def dia():
    import paper_2104_13715_amd as d
    return d


@pytest.fixture(scope="module")
def c1():
    return sf.config1()


def gpu(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def objs(dia, p, rho, var, lam):
    c = 1.345 if rho == "huber" else 2.3849
    kw = dict(rho=rho, var=var, sigma0=p.sigma0_adu, gain=p.gain, c=c)
    return oracle.Objective(lam=lam, **kw), dia.Objective(lam=lam, **kw)


def theta_off(p, seed):
    th = oracle.init_theta(p.I, p.m)
    return (th * np.random.default_rng(seed).uniform(0.5, 1.5, th.size)).astype(np.float32)


@pytest.mark.parametrize("rho,var,lam", CASES)
def test_regularised_loss_grad_matches_oracle(dia, c1, rho, var, lam):
    p = c1
    o_or, o_gpu = objs(dia, p, rho, var, lam)
    th = theta_off(p, 3)
    L, g = dia.loss_grad(gpu(p.R), gpu(p.I), gpu(th), p.m, o_gpu)
    L, g = float(L.item()), g.cpu().double().numpy()
    Lr, gr = oracle.loss_grad(p.R, p.I, th.astype(np.float64), p.m, o_or)
    pen = oracle.penalty(th.astype(np.float64), p.m, lam, oracle.n_data(*p.I.shape, p.m))
    assert pen[0] > 1e3 * 1e-10 * abs(Lr)  # a missing penalty would fail the loss bar
    assert abs(L - Lr) <= 1e-10 * abs(Lr)
    n = p.m * p.m
    assert np.linalg.norm(g[:n] - gr[:n]) <= 1e-5 * np.linalg.norm(gr[:n])
    assert abs(g[n] - gr[n]) <= 1e-5 * max(abs(gr[n]), 1e-6 * np.abs(gr).max())


@pytest.mark.parametrize("rho,var,lam", CASES)
def test_regularised_hessian_matches_oracle(dia, c1, rho, var, lam):
    p = c1
    o_or, o_gpu = objs(dia, p, rho, var, lam)
    th = theta_off(p, 4)
    H = dia.hessian(gpu(p.R), gpu(p.I), gpu(th), p.m, o_gpu).cpu().numpy()
    Hr = oracle.hessian(p.R, p.I, th.astype(np.float64), p.m, o_or)
    assert np.array_equal(H, H.T)
    assert np.max(np.abs(H - Hr)) <= 1e-9 * np.max(np.abs(Hr))


@pytest.mark.parametrize("rho,var,lam", CASES)
def test_regularised_fit_matches_oracle(dia, c1, rho, var, lam):
    p = c1
    m = p.m
    o_or, o_gpu = objs(dia, p, rho, var, lam)
    ref = oracle.solve(p.R, p.I, m, o_or)
    Lref = oracle.loss_grad(p.R, p.I, ref, m, o_or)[0]
    r = dia.fit(gpu(p.R), gpu(p.I), m, o_gpu)
    th = r.theta.cpu().double().numpy()
    K, Kr = th[:m * m], ref[:m * m]
    eK = np.linalg.norm(K - Kr) / np.linalg.norm(Kr)
    eP = abs(r.P - Kr.sum()) / abs(Kr.sum())
    eB = abs(r.B0 - ref[-1]) / max(abs(ref[-1]), 1.0)
    eL = abs(r.loss - Lref) / abs(Lref)
    print(f"{rho} {var} lambda {lam}: K {eK:.2e} P {eP:.2e} B0 {eB:.2e} loss {eL:.2e} evals {r.n_eval} "
          f"newton {r.n_newton} stop {r.stop}")
    assert r.status >= 0
    assert eK <= 1e-4 and eP <= 1e-4 and eB <= 1e-4 and eL <= 1e-10


def test_regularised_emccd_fit_matches_oracle(dia):
    # the many-small-pairs EMCCD case (Huber loss, EMCCD model variance, flat field): lambda = 1
    # roughens the kernel less (|L K| falls against the maximum-likelihood fit) and the fit lands
    # on the oracle's MAP solution
    m = 9
    b = sf.config_emccd(n_epochs=3, size=90, m=m)
    Fd = gpu(b.meta["flat"])
    R = gpu(b.R)
    Lap = oracle.laplacian(m)
    kw = dict(rho="huber", var="emccd_model", gain=b.gain, excess=b.meta["excess"])
    for e in b.epochs:
        ref0 = oracle.solve(b.R, e.I, m, oracle.Objective(flat=b.meta["flat"].astype(np.float64), **kw))
        o_or = oracle.Objective(flat=b.meta["flat"].astype(np.float64), lam=1.0, **kw)
        ref = oracle.solve(b.R, e.I, m, o_or)
        r = dia.fit(R, gpu(e.I), m, dia.Objective(flat=Fd, lam=1.0, **kw))
        th = r.theta.cpu().double().numpy()
        assert np.linalg.norm(Lap @ ref) < np.linalg.norm(Lap @ ref0)
        assert np.linalg.norm(th[:m * m] - ref[:m * m]) <= 1e-4 * np.linalg.norm(ref[:m * m])
        assert abs(r.P - ref[:m * m].sum()) <= 1e-4 * abs(ref[:m * m].sum())
        assert abs(r.B0 - ref[-1]) <= 1e-4 * max(abs(ref[-1]), 1.0)
        assert r.status >= 0


def test_batched_entry_points_reject_the_penalty(dia, c1):
    p = c1
    o = dia.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain, lam=1.0)
    ep = [dia.Epoch(I=gpu(p.I))]
    th = gpu(oracle.init_theta(p.I, p.m)[None, :])
    with pytest.raises(dia.DIAError):
        dia.loss_grad_batched(gpu(p.R), ep, th, p.m, o)
    with pytest.raises(dia.DIAError):
        dia.fit_batched(gpu(p.R), ep, p.m, o)


def test_map_uncertainty_matches_oracle(dia, c1):
    # Section 2.5 at the MAP fit: the observed information includes the penalty's curvature
    # 2 lambda N_data L L, so the covariance is that of the posterior's Laplace approximation
    p = c1
    m = p.m
    o_or, o_gpu = objs(dia, p, "gauss", "ccd_data", 5.0)
    th = oracle.solve(p.R, p.I, m, o_or)
    F = oracle.hessian(p.R, p.I, th, m, o_or)
    ref = oracle.covariance(F)
    out = dia.uncertainty(gpu(p.R), gpu(p.I), gpu(th), m, o_gpu)
    cov = out.cov.cpu().numpy()
    tol = max(1e-13 * np.linalg.cond(F), 1e-12) + 1e-9  # plus the Hessian's own 1e-9 of max |H|
    assert out.valid and ref["valid"]
    assert np.linalg.norm(cov - ref["cov"]) <= 10 * tol * np.linalg.norm(ref["cov"])
    # the penalty shrinks the kernel's uncertainty against the maximum-likelihood fit
    o0, g0 = objs(dia, p, "gauss", "ccd_data", 0.0)
    th0 = oracle.solve(p.R, p.I, m, o0)
    out0 = dia.uncertainty(gpu(p.R), gpu(p.I), gpu(th0), m, g0)
    assert np.all(out.sigma.cpu().numpy()[:m * m] < out0.sigma.cpu().numpy()[:m * m])


def test_penalty_with_mask_and_one_tap_kernel(dia, c1):
    p = c1
    # a mask leaves N_data (the valid-region count) unchanged
    mask = (np.random.default_rng(9).uniform(size=p.I.shape) > 0.2).astype(np.uint8)
    kw = dict(rho="cauchy", var="ccd_model", sigma0=p.sigma0_adu, gain=p.gain, lam=2.0)
    th = theta_off(p, 6)
    L, g = dia.loss_grad(gpu(p.R), gpu(p.I), gpu(th), p.m, dia.Objective(mask=gpu(mask, torch.uint8), **kw))
    Lr, gr = oracle.loss_grad(p.R, p.I, th.astype(np.float64), p.m, oracle.Objective(mask=mask, **kw))
    assert abs(float(L.item()) - Lr) <= 1e-10 * abs(Lr)
    assert np.linalg.norm(g.cpu().double().numpy() - gr) <= 1e-5 * np.linalg.norm(gr)
    # m = 1: the one-pixel kernel has no neighbours, so the penalty vanishes
    th1 = np.array([1.02, -3.0], np.float32)
    o1 = dia.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain, lam=7.0)
    o0 = dia.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain)
    L1, g1 = dia.loss_grad(gpu(p.R), gpu(p.I), gpu(th1), 1, o1)
    L0, g0 = dia.loss_grad(gpu(p.R), gpu(p.I), gpu(th1), 1, o0)
    assert float(L1.item()) == float(L0.item()) and torch.equal(g1, g0)


def test_regularised_fit_full_size_emccd_target(dia):
    # the MAP fit (lambda = 1) of target 0 of the EMCCD workload at full size (482^2, m = 19)
    # against the oracle's (tests/golden/make_emccd_target0.py)
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("emccd_target0", os.path.join(here, "make_emccd_target0.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    b, e = mod.target()
    m = mod.M
    path = os.path.join(here, "emccd_target0_lam1_oracle_theta.txt")
    ref = np.loadtxt(path)
    with open(path) as f:
        L_ref = float(f.readline().rsplit("loss", 1)[1])
    o = dia.Objective(rho="huber", var="emccd_model", gain=b.gain, excess=b.meta["excess"],
                      flat=gpu(b.meta["flat"]), lam=1.0)
    r = dia.fit(gpu(b.R), gpu(e.I), m, o)
    th = r.theta.cpu().double().numpy()
    K, Kr = th[:m * m], ref[:m * m]
    eK = np.linalg.norm(K - Kr) / np.linalg.norm(Kr)
    eP = abs(r.P - Kr.sum()) / abs(Kr.sum())
    eB = abs(r.B0 - ref[-1]) / max(abs(ref[-1]), 1.0)
    eL = abs(r.loss - L_ref) / abs(L_ref)
    print(f"MAP 482^2: K {eK:.2e} P {eP:.2e} B0 {eB:.2e} loss {eL:.2e} evals {r.n_eval} stop {r.stop}")
    assert r.status >= 0
    assert eK <= 1e-4 and eP <= 1e-4 and eB <= 1e-4 and eL <= 1e-10
