"""The polynomial differential background of Section 2.6 (eq. polybackground in the coordinates of
eq. normcoords) on the GPU, through the C ABI, against the FP64 oracle's ``*_poly`` functions.

Bars: model |dM| <= 2e-6 (sum|K| max|R| + max|B|) (FP32 output); loss 1e-12 relative and gradient
element by element within 1e-10 of each component's summation scale at FP64 parameters
(dia_loss_grad64: both sides sum FP64 products), and the FP32 entry point to the gradient bar of the
fused pass (1e-5 relative plus 1e-9 of the summation scale); Hessian within 1e-9 of max |H|; fits
within 1e-4 (kernel ||dK||/||K||, P, each background coefficient against max(|b|, 1)).
"""
import numpy as np
import pytest
import torch

import oracle
from parity import check_grad_elementwise
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


@pytest.fixture(scope="module")
def vb():
    return sf.config_varying_background()


@pytest.fixture(scope="module")
def vb19():
    return sf.config_varying_background(size=300, m=19)


def objs(dia, rho, var, p, d, lam=0.0):
    kw = dict(rho=rho, var=var, sigma0=p.sigma0_adu, gain=p.gain, c=2.3849 if rho == "cauchy" else 1.345,
              excess=2.0, lam=lam)
    return oracle.Objective(**kw), dia.Objective(bg_degree=d, **kw)


def start(p, d, rng):
    nb = (d + 1) * (d + 2) // 2
    b = np.zeros(nb)
    b[0] = 5.0
    b[1:] = rng.normal(0.0, 8.0, nb - 1)
    return np.concatenate([p.K_true.ravel() * 1.03, b])


def poly_scale(R, I, theta, m, o_or, d):
    """Summation scale S_j = sum_p |g_p| |X_pj| of every gradient component (taps, background terms)."""
    M = oracle.model_poly(R, theta, m, d)
    _, g, _ = oracle.pixel_terms(o_or, oracle.valid(np.asarray(I, np.float64), m), M, m)
    ag = np.abs(g)
    P = np.abs(oracle.poly_columns(*np.shape(R), m, d)).reshape(-1, len(oracle.poly_terms(d)))
    return np.concatenate([oracle.grad_kernel(np.abs(np.asarray(R, np.float64)), ag, m), ag.reshape(-1) @ P])


@pytest.mark.parametrize("d", [1, 2, 4])
def test_model_with_polynomial_background(dia, vb, d):
    p = vb
    th = start(p, d, np.random.default_rng(d)).astype(np.float32)
    M = dia.model(gpu(p.R), gpu(th), p.m, bg_degree=d).cpu().double().numpy()
    ref = oracle.model_poly(p.R, th.astype(np.float64), p.m, d)
    B = oracle.poly_columns(*p.R.shape, p.m, d) @ th[p.m * p.m:].astype(np.float64)
    scale = np.abs(th[:p.m * p.m]).sum() * np.abs(p.R).max() + np.abs(B).max()
    assert np.max(np.abs(M - ref)) <= 2e-6 * scale


@pytest.mark.parametrize("d", [1, 2, 4])
@pytest.mark.parametrize("rho,var", [("gauss", "ccd_data"), ("cauchy", "ccd_model"), ("huber", "emccd_model")])
def test_loss_grad64_with_polynomial_background(dia, vb, rho, var, d):
    p = vb
    m = p.m
    o_or, o_gpu = objs(dia, rho, var, p, d)
    th = start(p, d, np.random.default_rng(10 + d))
    loss, g = dia.loss_grad64(gpu(p.R), gpu(p.I), gpu(th, torch.float64), m, o_gpu)
    L_ref, g_ref = oracle.loss_grad_poly(p.R, p.I, th, m, o_or, d)
    assert abs(loss.item() - L_ref) <= 1e-12 * abs(L_ref)
    scale = poly_scale(p.R, p.I, th, m, o_or, d)
    gg = g.cpu().numpy()
    assert np.all(np.abs(gg - g_ref) <= 1e-10 * scale), np.max(np.abs(gg - g_ref) / scale)


@pytest.mark.parametrize("d", [1, 3])
def test_loss_grad_fp32_with_polynomial_background_ragged_m19(dia, vb19, d):
    # m = 19 on 300^2 (several tiles and a ragged edge), FP32 parameters, with the smoothness penalty
    p = vb19
    m = p.m
    o_or, o_gpu = objs(dia, "cauchy", "ccd_data", p, d, lam=0.5)
    th = start(p, d, np.random.default_rng(20 + d)).astype(np.float32)
    loss, g = dia.loss_grad(gpu(p.R), gpu(p.I), gpu(th), m, o_gpu)
    L_ref, g_ref = oracle.loss_grad_poly(p.R, p.I, th.astype(np.float64), m, o_or, d)
    assert abs(loss.item() - L_ref) <= 1e-10 * abs(L_ref)
    check_grad_elementwise(g.cpu().double().numpy(), g_ref, poly_scale(p.R, p.I, th.astype(np.float64), m, o_or, d))


@pytest.mark.parametrize("d,rho,var,lam", [(2, "gauss", "ccd_data", 0.0), (2, "cauchy", "ccd_model", 0.0),
                                           (1, "huber", "emccd_model", 0.7)])
def test_hessian_with_polynomial_background(dia, vb, d, rho, var, lam):
    p = vb
    m = p.m
    o_or, o_gpu = objs(dia, rho, var, p, d, lam)
    th = start(p, d, np.random.default_rng(30 + d)).astype(np.float32)
    H = dia.hessian(gpu(p.R), gpu(p.I), gpu(th), m, o_gpu).cpu().numpy()
    ref = oracle.hessian_poly(p.R, p.I, th.astype(np.float64), m, o_or, d)
    assert H.shape == ref.shape == (m * m + (d + 1) * (d + 2) // 2,) * 2
    assert np.array_equal(H, H.T)
    assert np.max(np.abs(H - ref)) <= 1e-9 * np.abs(ref).max()


def check_fit_poly(res, ref, m):
    th = res.theta.cpu().double().numpy()
    eK = np.linalg.norm(th[:m * m] - ref[:m * m]) / np.linalg.norm(ref[:m * m])
    eP = abs(res.P - ref[:m * m].sum()) / abs(ref[:m * m].sum())
    eb = np.max(np.abs(th[m * m:] - ref[m * m:]) / np.maximum(np.abs(ref[m * m:]), 1.0))
    print(f"K {eK:.2e} P {eP:.2e} b {eb:.2e} evals {res.n_eval} newton {res.n_newton} stop {res.stop}")
    assert res.status >= 0 and res.stop == "newton"
    assert eK <= 1e-4 and eP <= 1e-4 and eb <= 1e-4
    assert abs(res.B0 - ref[m * m]) <= 1e-4 * max(abs(ref[m * m]), 1.0)


@pytest.mark.parametrize("d,rho,var", [(1, "gauss", "ccd_data"), (2, "gauss", "ccd_data"), (3, "gauss", "ccd_data"),
                                       (2, "cauchy", "ccd_model"), (2, "huber", "emccd_model")])
def test_fit_with_polynomial_background(dia, vb, d, rho, var):
    p = vb
    m = p.m
    o_or, o_gpu = objs(dia, rho, var, p, d)
    res = dia.fit(gpu(p.R), gpu(p.I), m, o_gpu)
    ref = oracle.solve_poly(p.R, p.I, m, o_or, d)
    check_fit_poly(res, ref, m)


def test_fit_with_polynomial_background_m19_regularised(dia, vb19):
    p = vb19
    m = p.m
    o_or, o_gpu = objs(dia, "gauss", "ccd_data", p, 2, lam=1.0)
    res = dia.fit(gpu(p.R), gpu(p.I), m, o_gpu, init="gauss", init_phi=1.0)
    ref = oracle.solve_poly(p.R, p.I, m, o_or, 2)
    check_fit_poly(res, ref, m)


def test_covariance_with_polynomial_background(dia, vb):
    p = vb
    m, d = p.m, 2
    o_or, o_gpu = objs(dia, "gauss", "ccd_data", p, d)
    ref_th = oracle.solve_poly(p.R, p.I, m, o_or, d).astype(np.float32)
    F_ref = oracle.hessian_poly(p.R, p.I, ref_th.astype(np.float64), m, o_or, d)
    cv = dia.uncertainty(gpu(p.R), gpu(p.I), gpu(ref_th), m, o_gpu)
    ref = oracle.covariance(F_ref)
    C = cv.cov.cpu().numpy()
    assert cv.valid
    cond = np.linalg.cond(F_ref)
    assert np.max(np.abs(C - ref["cov"])) <= 1e-14 * cond * np.abs(ref["cov"]).max()
    # sigma_P sums the kernel block only
    sP = np.sqrt(ref["cov"][:m * m, :m * m].sum())
    assert abs(cv.sigma_P - sP) <= 1e-14 * cond * sP


def test_polynomial_background_options_are_checked(dia, vb):
    p = vb
    m = p.m
    R, I = gpu(p.R), gpu(p.I)
    with pytest.raises(dia.DIAError):
        dia.fit(R, I, m, dia.Objective(bg_degree=dia.MAX_BG_DEGREE + 1, sigma0=5.0))
    with pytest.raises(dia.DIAError):  # the reweight/clip loop keeps the scalar background
        dia.fit(R, I, m, dia.Objective(bg_degree=1, sigma0=5.0), max_outer=3, clip_kappa=3.0)
    with pytest.raises(dia.DIAError):  # batched fits have the scalar background
        dia.loss_grad_batched(R, [dia.Epoch(I=I)], torch.zeros((1, m * m + 1), device=DEV), m,
                              dia.Objective(bg_degree=1, sigma0=5.0))


def test_hessian_and_covariance_at_the_largest_parameter_count(dia):
    # m = 49 with a degree-1 background: 2401 taps + 3 background terms, beyond m*m + 1, so the
    # solver's and the inverse's per-parameter arrays must hold the background terms too.  A zero-mean
    # reference keeps the Fisher information well conditioned (about 1e8 here): a positive one makes
    # the constant term and the kernel sum nearly collinear.
    m, d = 49, 1
    rng = np.random.default_rng(49)
    R = rng.normal(0.0, 1000.0, (170, 170)).astype(np.float32)
    K = rng.uniform(0.0, 1.0, (m, m))
    K /= K.sum()
    th = np.concatenate([K.ravel(), [5.0, 3.0, -2.0]])
    M = oracle.model_poly(R, th, m, d)
    I = R.copy()
    h = (m - 1) // 2
    I[h:170 - h, h:170 - h] = M + rng.normal(0.0, 10.0, M.shape)
    kw = dict(rho="gauss", var="ccd_data", sigma0=10.0, gain=1.0)
    o_or, o_gpu = oracle.Objective(**kw), dia.Objective(bg_degree=d, **kw)
    th32 = th.astype(np.float32)
    F_ref = oracle.hessian_poly(R, I, th32.astype(np.float64), m, o_or, d)
    H = dia.hessian(gpu(R), gpu(I), gpu(th32), m, o_gpu).cpu().numpy()
    assert H.shape == (m * m + 3, m * m + 3)
    assert np.max(np.abs(H - F_ref)) <= 1e-9 * np.abs(F_ref).max()
    cv = dia.uncertainty(gpu(R), gpu(I), gpu(th32), m, o_gpu)
    ref = oracle.covariance(F_ref)
    assert cv.valid == ref["valid"]
    C = cv.cov.cpu().numpy()
    cond = np.linalg.cond(F_ref)
    assert np.max(np.abs(C - ref["cov"])) <= 1e-14 * cond * np.abs(ref["cov"]).max()
