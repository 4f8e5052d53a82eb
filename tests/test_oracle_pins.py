"""Pins of the FP64 oracle against things other than itself.

Each test ties one oracle function to a library routine, a closed form, a
finite difference, brute force on tiny inputs, or a value/behaviour the paper
prints (tests/golden/paper_values.json).  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.ndimage
import scipy.signal
import scipy.special
import scipy.stats

import oracle
from synthetic import starfield as sf

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))

RHOS = ["gauss", "huber", "cauchy"]
VARS = ["weights", "ccd_data", "ccd_model", "emccd_data", "emccd_model"]


def tiny_problem(seed=0, H=12, W=11, m=3):
    rng = np.random.default_rng(seed)
    R = rng.uniform(50.0, 400.0, (H, W))
    theta = np.concatenate([rng.uniform(-0.1, 0.4, m * m), [rng.uniform(-5, 5)]])
    I = rng.uniform(20.0, 500.0, (H, W))
    return R, I, theta


def brute_design(R, m):
    """Design matrix by explicit Python loops: row (i, j), column (a, b) -> R[i+a, j+b]; last column 1."""
    H, W = R.shape
    rows = []
    for i in range(H - m + 1):
        for j in range(W - m + 1):
            rows.append([R[i + a, j + b] for a in range(m) for b in range(m)] + [1.0])
    return np.array(rows)


def make_obj(rho, var, H, W, rng, with_mask=False):
    obj = oracle.Objective(rho=rho, var=var, sigma0=3.0, gain=1.7, excess=2.0, var_floor=1.0,
                           c=1.345 if rho == "huber" else 2.3849)
    if var == "weights":
        obj.weights = rng.uniform(0.01, 0.2, (H, W))
    obj.flat = rng.uniform(0.8, 1.2, (H, W))
    if with_mask:
        obj.mask = (rng.uniform(size=(H, W)) > 0.2).astype(np.uint8)
    return obj


# --------------------------------------------------------------------- model / correlation
@pytest.mark.parametrize("m", [1, 3, 5])
def test_model_matches_brute_design_and_scipy(m):
    R, _, theta = tiny_problem(1, 12, 11, m)
    M = oracle.model(R, theta, m)
    X = brute_design(R, m)
    np.testing.assert_allclose(M.ravel(), X @ theta, rtol=1e-13, atol=1e-10)
    K = theta[:m * m].reshape(m, m)
    ref = scipy.signal.correlate2d(R, K, mode="valid") + theta[-1]
    np.testing.assert_allclose(M, ref, rtol=1e-13, atol=1e-10)


def test_valid_pixel_count_matches_paper():
    g = GOLD["valid_pixels_142_m19"]
    assert oracle.n_data(142, 142, 19) == g["value"]
    R = np.zeros((142, 142))
    assert oracle.model(R, np.zeros(19 * 19 + 1), 19).size == g["value"]


def test_correlation_convention_pinned_by_shift():
    # Sec. 3.4 (iii): target = reference shifted by +1 in x and y -> identity kernel at (-1, -1).
    m = 5
    h = 2
    R = np.random.default_rng(3).uniform(0, 100, (20, 20))
    I = np.zeros_like(R)
    I[1:, 1:] = R[:-1, :-1]
    off = GOLD["e2_iii_kernel_offset"]["value"]
    theta = np.zeros(m * m + 1)
    theta[(h + off[0]) * m + (h + off[1])] = 1.0
    M = oracle.model(R, theta, m)
    np.testing.assert_array_equal(M, oracle.valid(I, m))


# --------------------------------------------------------------------- loss shapes
def test_huber_rho_is_scipy_huber():
    z = np.linspace(-6, 6, 1001)
    for c in (0.5, 1.345, 3.0):
        r, p, d = oracle.rho_psi_dpsi("huber", z, c)
        np.testing.assert_allclose(r, scipy.special.huber(c, z), rtol=1e-14, atol=1e-14)


def test_cauchy_rho_is_scaled_cauchy_logpdf():
    z = np.linspace(-30, 30, 1001)
    c = 2.3849
    r, _, _ = oracle.rho_psi_dpsi("cauchy", z, c)
    ref = -(c * c / 2.0) * (scipy.stats.cauchy.logpdf(z, scale=c) + math.log(math.pi * c))
    np.testing.assert_allclose(r, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("rho", RHOS)
def test_psi_and_dpsi_are_derivatives(rho):
    z = np.concatenate([np.linspace(-8, -1.4, 50), np.linspace(-1.3, 1.3, 50), np.linspace(1.4, 8, 50)])
    c = 1.345 if rho == "huber" else 2.3849
    e = 1e-6
    r, p, d = oracle.rho_psi_dpsi(rho, z, c)
    rp, pp, _ = oracle.rho_psi_dpsi(rho, z + e, c)
    rm, pm, _ = oracle.rho_psi_dpsi(rho, z - e, c)
    np.testing.assert_allclose(p, (rp - rm) / (2 * e), rtol=1e-7, atol=1e-7)
    np.testing.assert_allclose(d, (pp - pm) / (2 * e), rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("rho", ["huber", "cauchy"])
def test_robust_losses_reduce_to_gauss_for_large_c(rho):
    z = np.linspace(-5, 5, 101)
    g = oracle.rho_psi_dpsi("gauss", z, 1.0)
    r = oracle.rho_psi_dpsi(rho, z, 1e7)
    for a, b in zip(g, r):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("var", ["ccd_data", "ccd_model", "emccd_data", "emccd_model"])
def test_gauss_loss_is_negative_log_likelihood(var):
    # eq. loglikelihood: -ln p = 1/2 chi^2 + sum ln sigma + N/2 ln 2 pi, checked with scipy's normal logpdf.
    rng = np.random.default_rng(5)
    R, I, theta = tiny_problem(5, 14, 13, 3)
    obj = make_obj("gauss", var, *R.shape, rng)
    Iv = oracle.valid(I, 3)
    M = oracle.model(R, theta, 3)
    X = M if obj.model_sigma else Iv
    F = oracle.valid(obj.flat, 3)
    if var.startswith("ccd"):
        v = obj.sigma0 ** 2 / F ** 2 + np.maximum(X, 0) / (obj.gain * F)
    else:
        v = np.maximum(obj.excess * np.maximum(X, 0) / (obj.gain * F), obj.var_floor)
    nll = -np.sum(scipy.stats.norm.logpdf(Iv, loc=M, scale=np.sqrt(v)))
    L, _ = oracle.loss_grad(R, I, theta, 3, obj)
    const = 0.5 * Iv.size * math.log(2 * math.pi)
    if not obj.model_sigma:
        const += np.sum(0.5 * np.log(v))
    assert abs((L + const) - nll) <= 1e-11 * abs(nll)


def test_ccd_variance_matches_generator_noise():
    # MFV (Sec. 3.2, eq. MFV) at the true parameters is ~1 when the noise model is right.
    p = sf.config1()
    obj = oracle.Objective(rho="gauss", var="ccd_model", sigma0=p.sigma0_adu, gain=p.gain)
    theta = np.concatenate([p.K_true.ravel(), [p.B0_true]])
    M = oracle.model(p.R, theta, 9)
    F = np.ones(M.shape)
    Iv = oracle.valid(p.I.astype(np.float64), 9)
    v, _ = oracle.oracle._variance(obj, M, F)
    z = (Iv - M) / np.sqrt(v)
    assert abs(np.mean(z)) < 4 / math.sqrt(z.size)
    assert abs(np.var(z) - 1.0) < 4 * math.sqrt(2.0 / z.size)


def test_emccd_variance_matches_generator_noise():
    # the many-small-pairs workload: at the true parameters the EMCCD model variance
    # E max(M, 0) / (G F) (eq. EMCCDNM) normalises the residuals to unit variance
    b = sf.config_emccd(n_epochs=2, size=90, m=9)
    F = oracle.valid(b.meta["flat"].astype(np.float64), 9)
    obj = oracle.Objective(rho="gauss", var="emccd_model", gain=b.gain, excess=b.meta["excess"], var_floor=1e-6)
    for e in b.epochs:
        theta = np.concatenate([e.K_true.ravel(), [e.B0_true]])
        M = oracle.model(b.R, theta, 9)
        v, _ = oracle.oracle._variance(obj, M, F)
        z = (oracle.valid(e.I.astype(np.float64), 9) - M) / np.sqrt(v)
        assert abs(np.mean(z)) < 4 / math.sqrt(z.size)
        assert abs(np.var(z) - 1.0) < 4 * math.sqrt(2.0 / z.size)


# --------------------------------------------------------------------- gradient and curvature
@pytest.mark.parametrize("rho", RHOS)
@pytest.mark.parametrize("var", VARS)
def test_grad_matches_central_differences_and_brute_design(rho, var):
    rng = np.random.default_rng(RHOS.index(rho) * 10 + VARS.index(var))
    m = 3
    R, I, theta = tiny_problem(7, 12, 11, m)
    obj = make_obj(rho, var, *R.shape, rng, with_mask=True)
    L, g = oracle.loss_grad(R, I, theta, m, obj)
    e = 1e-6
    fd = np.empty_like(g)
    for k in range(g.size):
        tp = theta.copy(); tp[k] += e
        tm = theta.copy(); tm[k] -= e
        fd[k] = (oracle.loss_grad(R, I, tp, m, obj)[0] - oracle.loss_grad(R, I, tm, m, obj)[0]) / (2 * e)
    np.testing.assert_allclose(g, fd, rtol=2e-6, atol=2e-6 * np.abs(g).max())
    # brute force: grad = X^T l'(M)
    X = brute_design(R, m)
    M = oracle.model(R, theta, m)
    _, gp, _ = oracle.pixel_terms(obj, oracle.valid(I, m), M, m)
    np.testing.assert_allclose(g, X.T @ gp.ravel(), rtol=1e-12, atol=1e-12 * np.abs(g).max())


@pytest.mark.parametrize("rho", RHOS)
@pytest.mark.parametrize("var", VARS)
def test_pixel_curvature_matches_difference_of_slope(rho, var):
    rng = np.random.default_rng(11)
    m = 3
    R, I, theta = tiny_problem(9, 12, 11, m)
    obj = make_obj(rho, var, *R.shape, rng)
    Iv = oracle.valid(I, m)
    M = oracle.model(R, theta, m)
    e = 1e-4
    l, g, h = oracle.pixel_terms(obj, Iv, M, m)
    lp, gp, _ = oracle.pixel_terms(obj, Iv, M + e, m)
    lm, gm, _ = oracle.pixel_terms(obj, Iv, M - e, m)
    np.testing.assert_allclose(g, (lp - lm) / (2 * e), rtol=1e-6, atol=1e-9)
    # skip pixels whose +-e interval straddles a kink (Huber |z| = c)
    smooth = np.abs(((gp - g) - (g - gm)) / e) < 1e-3 * np.maximum(np.abs(h), 1e-6) + 1e-9
    np.testing.assert_allclose(h[smooth], ((gp - gm) / (2 * e))[smooth], rtol=1e-5, atol=1e-12)


def test_constant_reference_couples_kernel_and_background_gradients():
    # R = c0 everywhere: every dL/dK_ab equals c0 * dL/dB0.
    m = 5
    R = np.full((16, 15), 7.25)
    _, I, theta = tiny_problem(2, 16, 15, m)
    obj = oracle.Objective(rho="huber", var="ccd_model", sigma0=4.0, gain=1.2)
    _, g = oracle.loss_grad(R, I, theta, m, obj)
    np.testing.assert_allclose(g[:-1], 7.25 * g[-1], rtol=1e-12)


# --------------------------------------------------------------------- linear solve (B08 step)
def test_normal_matrix_and_cholesky_match_lstsq():
    m = 3
    R, I, _ = tiny_problem(4, 13, 12, m)
    w = np.random.default_rng(4).uniform(0.1, 2.0, (13 - m + 1, 12 - m + 1))
    X = brute_design(R, m)
    A, b = oracle.normal_matrix(R, m, w, oracle.valid(I, m))
    np.testing.assert_allclose(A, X.T @ (w.ravel()[:, None] * X), rtol=1e-12)
    theta = oracle.solve_chi2(R, I, m, w)
    sw = np.sqrt(w.ravel())
    ref = np.linalg.lstsq(sw[:, None] * X, sw * oracle.valid(I, m).ravel(), rcond=None)[0]
    np.testing.assert_allclose(theta, ref, rtol=1e-9, atol=1e-11)


def _recover(R, I, m, B0):
    w = np.ones((R.shape[0] - m + 1, R.shape[1] - m + 1))
    return oracle.solve_chi2(R, I, m, w)


@pytest.fixture(scope="module")
def paper_ref():
    return sf.paper_reference(142, seed=3, phi_R=1.2).astype(np.float32).astype(np.float64)


def _check_recovery(theta, K_true, B0, m):
    K = theta[:m * m]
    assert np.linalg.norm(K - K_true.ravel()) <= 1e-9 * np.linalg.norm(K_true)
    P, Ptrue = K.sum(), K_true.sum()
    assert abs(P - Ptrue) / Ptrue <= 1e-10
    assert abs(theta[-1] - B0) / abs(B0) <= 1e-9


def test_e2_i_self_difference(paper_ref):
    m, B0 = 19, 17.5
    I = paper_ref + B0
    K = np.zeros((m, m)); K[9, 9] = 1.0
    _check_recovery(_recover(paper_ref, I, m, B0), K, B0, m)


def test_e2_ii_gaussian_kernel(paper_ref):
    m, B0 = 19, 17.5
    a = np.arange(m) - 9
    K = np.exp(-0.5 * (a[:, None] ** 2 + a[None, :] ** 2) / 1.5 ** 2)
    K /= K.sum()
    I = np.pad(scipy.signal.correlate2d(paper_ref, K, mode="valid"), 9) + B0
    _check_recovery(_recover(paper_ref, I, m, B0), K, B0, m)


def test_e2_iii_integer_shift(paper_ref):
    m, B0 = 19, 17.5
    I = np.zeros_like(paper_ref)
    I[1:, 1:] = paper_ref[:-1, :-1]
    I += B0
    K = np.zeros((m, m)); K[9 - 1, 9 - 1] = 1.0
    _check_recovery(_recover(paper_ref, I, m, B0), K, B0, m)


def test_e2_iv_half_pixel_cubic_spline_shift(paper_ref):
    m, B0 = 19, 17.5
    I = scipy.ndimage.shift(paper_ref, (0.5, 0.5), order=3, prefilter=False, mode="nearest") + B0
    g = GOLD["e2_iv_bspline_weights_x48"]
    beta = np.array(g["value"], float) / 48.0
    K = np.zeros((m, m))
    for ia, oa in enumerate(g["offsets"]):
        for ib, ob in enumerate(g["offsets"]):
            K[9 + oa, 9 + ob] = beta[ia] * beta[ib]
    _check_recovery(_recover(paper_ref, I, m, B0), K, B0, m)


def test_injected_scale_recovered_on_noiseless_config1():
    p = sf.config1(noise=False)
    obj = oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain)
    theta = oracle.solve(p.R, p.I_noiseless, 9, obj)
    assert abs(oracle.photometric_scale(theta, 9) - 1.1) <= 1e-9
    assert abs(theta[-1] - 5.0) <= 1e-8
    np.testing.assert_allclose(theta[:81], p.K_true.ravel(), atol=1e-10)


def test_reference_offset_invariant():
    # R -> R - s leaves K unchanged and moves B0 to B0 + s * sum K.
    p = sf.config1()
    obj = oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain)
    R = p.R.astype(np.float64)
    t1 = oracle.solve(R, p.I, 9, obj)
    s = 100.0
    t2 = oracle.solve(R - s, p.I, 9, obj)
    np.testing.assert_allclose(t2[:81], t1[:81], rtol=1e-8, atol=1e-11)
    assert abs(t2[81] - (t1[81] + s * t1[:81].sum())) <= 1e-8 * abs(t2[81])


# --------------------------------------------------------------------- non-quadratic solver
@pytest.mark.parametrize("rho", ["huber", "cauchy"])
def test_robust_fit_recovers_noiseless_truth(rho):
    p = sf.config1(noise=False)
    obj = oracle.Objective(rho=rho, var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain,
                           c=1.345 if rho == "huber" else 2.3849)
    theta = oracle.solve(p.R, p.I_noiseless, 9, obj,
                         theta0=oracle.init_theta(p.I_noiseless, 9, "flat"))
    np.testing.assert_allclose(theta[:81], p.K_true.ravel(), atol=1e-9)
    assert abs(theta[81] - 5.0) <= 1e-7


def test_huber_large_c_equals_chi2_solution():
    p = sf.config1()
    base = oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain)
    hub = oracle.Objective(rho="huber", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain, c=1e6)
    t0 = oracle.solve(p.R, p.I, 9, base)
    t1 = oracle.solve(p.R, p.I, 9, hub, theta0=oracle.init_theta(p.I, 9))
    np.testing.assert_allclose(t1, t0, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("rho,var", [("gauss", "ccd_model"), ("huber", "ccd_data"), ("cauchy", "ccd_data"),
                                     ("huber", "emccd_model")])
def test_robust_solution_is_stationary_with_pd_hessian(rho, var):
    p = sf.config1()
    obj = oracle.Objective(rho=rho, var=var, sigma0=p.sigma0_adu, gain=p.gain, excess=2.0,
                           c=1.345 if rho == "huber" else 2.3849)
    theta = oracle.solve(p.R, p.I, 9, obj)
    _, g = oracle.loss_grad(p.R, p.I, theta, 9, obj)
    # gradient scale: sum_p |l'_p| |X_pj| at the flat start
    t0 = oracle.init_theta(p.I, 9)
    _, g0 = oracle.loss_grad(p.R, p.I, t0, 9, obj)
    assert np.abs(g).max() <= 1e-9 * np.abs(g0).max()
    H = oracle.hessian(p.R, p.I, theta, 9, obj)
    assert np.linalg.eigvalsh(H).min() > 0


# --------------------------------------------------------------------- clipping loop
def _design(R, m):
    """Design matrix of the valid region by slicing: column (a, b) is the reference shifted by (a, b)."""
    H, W = R.shape
    Hv, Wv = H - m + 1, W - m + 1
    cols = [R[a:a + Hv, b:b + Wv].ravel() for a in range(m) for b in range(m)]
    return np.stack(cols + [np.ones(Hv * Wv)], axis=1)


def _b08_loop_by_hand(R, I, F, m, s0, G, floor, kappa, n_fits):
    """The reweight-and-clip iteration written out in the test (Sec. 2.1 and 2.4), independent of the
    oracle: fit 1 weighs each pixel by 1/v(I); fit k > 1 by 1/v(M_(k-1)), M from scipy's correlation of
    the previous fit, and drops pixels whose |I - M_(k-1)| / sqrt(v) exceeds kappa (masks accumulate).
    v(X) = max(s0^2 / F^2 + max(X, 0) / (G F), floor), eq. CCDNM.  Each fit is numpy's least squares on
    the square-root-weighted design.  Stops after n_fits or after the first fit whose mask did not change."""
    R = R.astype(np.float64)
    h = (m - 1) // 2
    Iv = I.astype(np.float64)[h:I.shape[0] - h, h:I.shape[1] - h]
    Fv = F[h:F.shape[0] - h, h:F.shape[1] - h]
    X = _design(R, m)

    def var(Xv):
        return np.maximum(s0 * s0 / (Fv * Fv) + np.maximum(Xv, 0.0) / (G * Fv), floor)

    def wls(w, keep):
        sw = np.sqrt(np.where(keep, w, 0.0)).ravel()
        return np.linalg.lstsq(X * sw[:, None], Iv.ravel() * sw, rcond=None)[0]

    keep = np.ones(Iv.shape, bool)
    theta = wls(1.0 / var(Iv), keep)
    fits = 1
    while fits < n_fits:
        M = scipy.signal.correlate(R, theta[:m * m].reshape(m, m), mode="valid") + theta[m * m]
        v = var(M)
        new_keep = keep & (np.abs(Iv - M) / np.sqrt(v) <= kappa)
        changed = not np.array_equal(new_keep, keep)
        keep = new_keep
        theta = wls(1.0 / v, keep)
        fits += 1
        if not changed:
            break
    return theta, keep, fits


@pytest.mark.parametrize("kappa,n_fits", [(3.0, 2), (3.0, 3), (2.0, 4)])
def test_clipped_loop_equals_the_reweighting_written_out(kappa, n_fits):
    # pins fit_clipped's second and later fits: weights 1/v(M_prev) with the flat, the clip threshold on
    # z = (I - M_prev)/sigma, cumulative masks and the stop rule
    p = sf.config1()
    m = p.m
    F = np.random.default_rng(41).uniform(0.9, 1.1, p.R.shape)
    obj = oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain, flat=F, var_floor=1.0)
    th, mask, n = oracle.fit_clipped(p.R, p.I, m, obj, kappa=kappa, max_outer=n_fits)
    ref, keep, n_ref = _b08_loop_by_hand(p.R, p.I, F, m, p.sigma0_adu, p.gain, 1.0, kappa, n_fits)
    assert n == n_ref
    h = oracle.half(m)
    assert np.array_equal(mask[h:-h, h:-h] != 0, keep)
    assert (~keep).sum() > 0  # the clip is active in every case
    np.testing.assert_allclose(th, ref, rtol=1e-10, atol=1e-10 * np.abs(ref[:m * m]).max())


def test_clipping_masks_cosmic_rays_and_recovers_clean_fit():
    p = sf.config1()
    m = p.m
    obj = oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain)
    rng = np.random.default_rng(0)
    I = p.I.astype(np.float64).copy()
    hits = sorted({(int(rng.integers(10, 118)), int(rng.integers(10, 118))) for _ in range(12)})
    for (i, j) in hits:
        I[i, j] += 50.0 * math.sqrt(p.sigma0_adu ** 2 + max(I[i, j], 0) / p.gain)
    theta3, mask3, n3 = oracle.fit_clipped(p.R, I, m, obj, kappa=3.0, max_outer=3)
    assert n3 == 3 and all(mask3[i, j] == 0 for (i, j) in hits)
    # one reweight: the hits are masked after the first fit.  The same loop on the clean image, started
    # with that mask, clips nothing more and also refits once, so the two second fits see the same pixels
    # with weights from first fits that differ only by the hits' pull on the contaminated one
    theta, mask, n = oracle.fit_clipped(p.R, I, m, obj, kappa=3.0, max_outer=2)
    assert n == 2 and all(mask[i, j] == 0 for (i, j) in hits)
    clean_obj = oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain, mask=mask)
    clean, cmask, nc = oracle.fit_clipped(p.R, p.I, m, clean_obj, kappa=3.0, max_outer=2)
    assert nc == 2 and np.array_equal(cmask, mask)
    K, K0 = theta[:m * m], clean[:m * m]
    # the photometric scale and background agree to 1e-5; the kernel's poorly constrained modes carry
    # the weight difference at about 1e-4 (one more reweight alone moves them by 1e-3)
    assert abs(K.sum() - K0.sum()) / abs(K0.sum()) < 1e-5
    assert abs(theta[m * m] - clean[m * m]) / max(abs(clean[m * m]), 1.0) < 1e-4
    assert np.linalg.norm(K - K0) / np.linalg.norm(K0) < 2e-4


# --------------------------------------------------------------------- optimiser pieces and init
def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(1)
    g = rng.normal(size=20) * 10 ** rng.uniform(-3, 3, 20)
    th = rng.normal(size=20)
    lr = np.full(20, 1e-3)
    t1, m1, v1 = oracle.adam_step(th, g, np.zeros(20), np.zeros(20), 1, lr, eps=0.0)
    np.testing.assert_allclose(t1 - th, -lr * np.sign(g), rtol=1e-12)
    # constant gradient: every bias-corrected step has size lr
    for t in range(2, 30):
        t2, m1, v1 = oracle.adam_step(t1, g, m1, v1, t, lr, eps=0.0)
        np.testing.assert_allclose(t2 - t1, -lr * np.sign(g), rtol=1e-12)
        t1 = t2


def test_lbfgs_direction_is_the_bfgs_inverse_hessian_update():
    # the two-loop recursion applies the inverse-Hessian estimate built by the BFGS update
    #   H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T,  rho = 1 / s.y,
    # from H_0 = gamma I, pair by pair (oldest first), written out here as dense matrices
    rng = np.random.default_rng(12)
    n = 7
    A = rng.normal(size=(n, n))
    A = A @ A.T + n * np.eye(n)  # a convex quadratic: y = A s gives s.y > 0
    pairs = []
    for _ in range(4):
        s = rng.normal(size=n)
        pairs.append((s, A @ s))
    g = rng.normal(size=n)
    s_n, y_n = pairs[-1]
    H = (s_n @ y_n) / (y_n @ y_n) * np.eye(n)
    for s, y in pairs:
        rho = 1.0 / (s @ y)
        E = np.eye(n) - rho * np.outer(s, y)
        H = E @ H @ E.T + rho * np.outer(s, s)
    np.testing.assert_allclose(oracle.lbfgs_direction(g, pairs), -H @ g, rtol=1e-12, atol=1e-12)
    # no pairs: steepest descent; n A-conjugate pairs of a quadratic (the eigenvectors of A) give the
    # exact Newton step (the BFGS update keeps the secant condition of every earlier conjugate pair)
    np.testing.assert_allclose(oracle.lbfgs_direction(g, []), -g, rtol=0, atol=0)
    full = [(e, A @ e) for e in np.linalg.eigh(A)[1].T]
    np.testing.assert_allclose(oracle.lbfgs_direction(g, full), -np.linalg.solve(A, g), rtol=1e-10, atol=1e-12)


def test_init_theta():
    I = np.arange(1.0, 101.0).reshape(10, 10)
    t = oracle.init_theta(I, 5, "flat")
    assert abs(t[:25].sum() - 1.0) < 1e-15 and np.all(t[:25] == t[0])
    assert t[25] == 50.5
    t = oracle.init_theta(I, 5, "gauss", 1.3)
    assert abs(t[:25].sum() - 1.0) < 1e-15 and np.argmax(t[:25]) == 12


@pytest.mark.parametrize("phi,m", [(1.0, 15), (1.5, 19), (2.2, 25)])
def test_gaussian_init_width_is_a_standard_deviation(phi, m):
    # Sec. 2.9 parameterises the Gaussian start by its standard deviation: the sampled kernel's second
    # moment along each axis is phi^2 (the grid sum of a sampled Gaussian reproduces it to e^(-2 pi^2
    # phi^2) while the truncation at the kernel edge is far in the tail); a FWHM reading would give
    # (phi / 2.355)^2.  Centred, symmetric and separable.
    I = np.full((40, 40), 3.0)
    K = oracle.init_theta(I, m, "gauss", phi)[:m * m].reshape(m, m)
    h = oracle.half(m)
    a = np.arange(m) - h
    assert abs(K.sum() - 1.0) < 1e-14
    assert abs(np.sum(K * a[:, None])) < 1e-14 and abs(np.sum(K * a[None, :])) < 1e-14
    assert np.sum(K * a[:, None] ** 2) == pytest.approx(phi * phi, rel=1e-6)
    assert np.sum(K * a[None, :] ** 2) == pytest.approx(phi * phi, rel=1e-6)
    np.testing.assert_allclose(K, np.outer(K.sum(1), K.sum(0)), rtol=1e-12, atol=1e-16)


def test_huber_constant_large_c_limit():
    # Sec. 2.4: for large c, Q -> (N/2) ln 2 pi
    n = 15376
    assert abs(oracle.huber_constant(40.0, n) - 0.5 * n * math.log(2 * math.pi)) < 1e-9 * n


def test_generator_gaussian_width_rule():
    # eq. truetargetPSF: a Gaussian PSF of sd phi_R correlated with a Gaussian kernel of sd phi_K
    # is a Gaussian of sd sqrt(phi_R^2 + phi_K^2) (second moments add).
    phi_R, phi_K = 1.3, 1.5
    R = sf.render_stars((61, 61), np.array([30.0]), np.array([30.0]), np.array([1.0]),
                        sf.gaussian_psf(phi_R * sf.FWHM_PER_SIGMA), 25)
    K = sf.kernel_gaussian(21, phi_K * sf.FWHM_PER_SIGMA)
    T = sf.correlate_target(R, K, 0.0)
    y, x = np.mgrid[0:61, 0:61]
    var = np.sum(T * (x - 30.0) ** 2) / np.sum(T)
    assert abs(var - (phi_R ** 2 + phi_K ** 2)) < 1e-3


def _mfv(obj, I, M, m):
    F = np.ones(M.shape) if obj.flat is None else oracle.valid(obj.flat, m)
    v, _ = oracle.oracle._variance(obj, M, F)
    z = (oracle.valid(I, m) - M) / np.sqrt(v)
    return np.mean(z), np.var(z), z.size


def test_ccd_flat_field_variance_by_simulation():
    # eq. CCDNM: a detector that sees F*S with read noise sigma0 (ADU) and gain G, divided by the flat,
    # has variance sigma0^2/F^2 + S/(G F).  Simulated here pixel by pixel.
    rng = np.random.default_rng(21)
    H = W = 160
    m = 3
    S = rng.uniform(50, 3000, (H, W))
    F = rng.uniform(0.6, 1.4, (H, W))
    G, s0 = 1.7, 6.0
    raw = rng.poisson(F * S * G) / G + rng.normal(0, s0, (H, W))
    I = raw / F
    theta = np.zeros(m * m + 1); theta[4] = 1.0
    obj = oracle.Objective(var="ccd_model", sigma0=s0, gain=G, flat=F, var_floor=0.0)
    mu, var, n = _mfv(obj, I, oracle.model(S, theta, m), m)
    assert abs(mu) < 4 / math.sqrt(n) and abs(var - 1) < 4 * math.sqrt(2 / n)


def test_emccd_variance_by_simulation():
    # eq. EMCCDNM with E = 2, G_Total = 25.8/300: photo-electrons ~ Poisson, the EM register multiplies
    # each by an exponential gain (mean 300), 25.8 EM-electrons per ADU, then the flat is divided out.
    rng = np.random.default_rng(22)
    H = W = 160
    m = 3
    S = rng.uniform(200, 5000, (H, W))
    F = rng.uniform(0.7, 1.3, (H, W))
    gt = GOLD["emccd_gain_total"]["value"]
    n_phot = rng.poisson(F * S * gt)
    em = rng.gamma(np.maximum(n_phot, 1), 300.0) * (n_phot > 0)
    I = em / 25.8 / F
    theta = np.zeros(m * m + 1); theta[4] = 1.0
    obj = oracle.Objective(var="emccd_model", gain=gt, excess=GOLD["emccd_excess_E"]["value"], flat=F,
                           var_floor=0.0)
    mu, var, n = _mfv(obj, I, oracle.model(S, theta, m), m)
    assert abs(mu) < 4 / math.sqrt(n) and abs(var - 1) < 0.05


def test_mask_equals_zero_weight():
    rng = np.random.default_rng(8)
    m = 3
    R, I, theta = tiny_problem(8, 12, 11, m)
    w = rng.uniform(0.01, 0.2, R.shape)
    mask = (rng.uniform(size=R.shape) > 0.3).astype(np.uint8)
    for rho in RHOS:
        a = oracle.loss_grad(R, I, theta, m, oracle.Objective(rho=rho, var="weights", weights=w, mask=mask))
        b = oracle.loss_grad(R, I, theta, m, oracle.Objective(rho=rho, var="weights", weights=w * mask))
        assert abs(a[0] - b[0]) <= 1e-12 * abs(a[0])
        np.testing.assert_allclose(a[1], b[1], rtol=1e-12, atol=1e-12 * np.abs(a[1]).max())


# ------------------------------------------------------------------ Fisher information and covariance (Sec. 2.5)
def test_covariance_of_one_tap_fit_is_the_closed_form_inverse():
    # m = 1, fixed weights: F = sum_p w_p (R_p, 1)(R_p, 1)^T is the 2 x 2 matrix [[a, b], [b, c]]
    # with a = sum w R^2, b = sum w R, c = sum w, whose inverse is [[c, -b], [-b, a]] / (ac - b^2)
    rng = np.random.default_rng(31)
    R = rng.uniform(10.0, 500.0, (23, 19))
    w = rng.uniform(0.5, 2.0, R.shape)
    I = 0.8 * R + 3.0 + rng.normal(0.0, 1.0, R.shape) / np.sqrt(w)
    oo = oracle.Objective(rho="gauss", var="weights", weights=w)
    F = oracle.hessian(R, I, np.array([0.8, 3.0]), 1, oo)
    a, b, c = np.sum(w * R * R), np.sum(w * R), np.sum(w)
    np.testing.assert_allclose(F, [[a, b], [b, c]], rtol=1e-13)
    out = oracle.covariance(F)
    det = a * c - b * b
    np.testing.assert_allclose(out["cov"], np.array([[c, -b], [-b, a]]) / det, rtol=1e-10)
    np.testing.assert_allclose(out["sigma"], np.sqrt([c / det, a / det]), rtol=1e-10)
    assert math.isclose(out["sigma_P"], math.sqrt(c / det), rel_tol=1e-10)  # P = K for m = 1
    assert out["valid"] and math.isclose(out["logdet"], -math.log(det), rel_tol=1e-10)


def test_covariance_validity_tests():
    # a matrix with a negative eigenvalue fails (its inverse has a negative eigenvalue too);
    # one with an even number of negative eigenvalues has a positive determinant but still fails
    good = np.array([[4.0, 1.0, 0.0], [1.0, 3.0, 0.5], [0.0, 0.5, 2.0]])
    assert oracle.covariance(good)["valid"]
    assert not oracle.covariance(np.diag([2.0, -1.0, 3.0]))["valid"]
    two_neg = oracle.covariance(np.diag([-2.0, -1.0, 3.0]))
    assert not two_neg["valid"] and np.linalg.det(two_neg["cov"]) > 0


def test_covariance_is_the_scatter_of_refitted_parameters():
    # Cramer-Rao for the Gaussian chi-squared with the true weights: the minimiser is linear in the
    # data, so over repeated noise draws its covariance is exactly F^-1.  400 draws: the sample
    # standard deviations agree within 15 % (each estimate has ~3.5 % standard error)
    rng = np.random.default_rng(32)
    m = 3
    R = rng.uniform(50.0, 800.0, (30, 28))
    theta = np.r_[rng.uniform(0.0, 0.3, m * m), 7.0]
    M = oracle.model(R, theta, m)
    s = rng.uniform(2.0, 6.0, M.shape)
    wfull = np.zeros(R.shape)
    h = oracle.half(m)
    wfull[h:R.shape[0] - h, h:R.shape[1] - h] = 1.0 / s ** 2
    oo = oracle.Objective(rho="gauss", var="weights", weights=wfull)
    out = oracle.covariance(oracle.hessian(R, np.zeros(R.shape), theta, m, oo))
    fits = []
    for _ in range(400):
        I = np.zeros(R.shape)
        I[h:R.shape[0] - h, h:R.shape[1] - h] = M + s * rng.standard_normal(M.shape)
        fits.append(oracle.solve(R, I, m, oo))
    fits = np.array(fits)
    sd = fits.std(axis=0, ddof=1)
    np.testing.assert_allclose(sd, out["sigma"], rtol=0.15)
    sdP = fits[:, :m * m].sum(axis=1).std(ddof=1)
    assert abs(sdP / out["sigma_P"] - 1.0) < 0.15


# --------------------------------------------------------------------- kernel regulariser (Sec. 2.7)
@pytest.mark.parametrize("m", [1, 3, 5, 9])
def test_laplacian_spectrum_is_the_grid_graph_closed_form(m):
    # eq. laplacian on the m x m grid with side-sharing adjacency is the Kronecker sum of two path
    # graphs, whose Laplacian eigenvalues are 2 - 2 cos(pi j / m), j = 0 .. m-1
    L = oracle.laplacian(m)
    n = m * m
    assert L.shape == (n + 1, n + 1)
    assert np.array_equal(L, L.T)
    assert not L[n].any() and not L[:, n].any()
    assert np.allclose(L[:n, :n].sum(axis=1), 0.0)
    deg = np.diag(L)[:n].reshape(m, m)
    if m > 1:
        assert deg[0, 0] == 2 and deg[-1, -1] == 2
        if m > 2:
            assert deg[0, 1] == 3 and deg[1, 1] == 4
    path = 2.0 - 2.0 * np.cos(np.pi * np.arange(m) / m)
    want = np.sort((path[:, None] + path[None, :]).ravel())
    got = np.linalg.eigvalsh(L[:n, :n])
    assert np.allclose(got, want, atol=1e-12)


def test_penalty_of_a_single_pixel_and_a_constant_kernel():
    m, lam, N = 5, 0.7, 123
    th = np.zeros(m * m + 1)
    th[m * m] = 42.0  # B0 is not penalised
    assert oracle.penalty(th, m, lam, N)[0] == 0.0
    th[:m * m] = 0.3  # constant kernel: the null space of L
    assert abs(oracle.penalty(th, m, lam, N)[0]) < 1e-12
    for (a, b), deg in (((2, 2), 4), ((0, 0), 2), ((0, 2), 3)):
        th = np.zeros(m * m + 1)
        th[a * m + b] = 1.0
        # L e_u has deg at u and -1 at each of the deg neighbours: |L e_u|^2 = deg^2 + deg
        assert oracle.penalty(th, m, lam, N)[0] == pytest.approx(lam * N * (deg * deg + deg), rel=1e-14)


def test_penalty_gradient_and_hessian_are_derivatives():
    rng = np.random.default_rng(5)
    m, lam, N = 5, 2.5, 77
    th = rng.normal(size=m * m + 1)
    p, g, H = oracle.penalty(th, m, lam, N)
    h = 1e-3
    for k in (0, 7, 12, 24, 25):
        e = np.zeros_like(th)
        e[k] = h
        fd = (oracle.penalty(th + e, m, lam, N)[0] - oracle.penalty(th - e, m, lam, N)[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-9, abs=1e-9)  # exact for a quadratic up to rounding
        assert np.allclose((oracle.penalty(th + e, m, lam, N)[1] - oracle.penalty(th - e, m, lam, N)[1]) / (2 * h),
                           H[:, k], rtol=1e-9, atol=1e-9)
    assert p == pytest.approx(0.5 * th @ H @ th, rel=1e-12)


@pytest.fixture(scope="module")
def c1_pair():
    return sf.config1()


def test_regularised_solve_limits(c1_pair):
    p = c1_pair
    m = p.m
    obj = oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain)
    t0 = oracle.solve(p.R, p.I, m, obj)
    # lambda = 0 is the maximum-likelihood fit
    obj0 = oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain, lam=0.0)
    assert np.array_equal(oracle.solve(p.R, p.I, m, obj0), t0)
    # lambda -> infinity: the kernel is forced into the null space of L (a constant), and the fit
    # tends, as 1/lambda, to the two-parameter weighted least squares of I on (box sum of R, 1)
    w = oracle.fixed_weights(obj, p.I, m).ravel()
    box = scipy.signal.correlate(p.R.astype(np.float64), np.ones((m, m)), mode="valid").ravel()
    A = np.stack([box, np.ones_like(box)], 1) * np.sqrt(w)[:, None]
    y = oracle.valid(p.I.astype(np.float64), m).ravel() * np.sqrt(w)
    c, B0 = np.linalg.lstsq(A, y, rcond=None)[0]
    dev = []
    for lam in (1e8, 1e10):
        tL = oracle.solve(p.R, p.I, m, oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu,
                                                         gain=p.gain, lam=lam))
        K = tL[:m * m]
        dev.append((np.ptp(K) / abs(K.mean()), abs(K.mean() / c - 1.0), abs(tL[m * m] / B0 - 1.0)))
    assert dev[1][0] <= 1e-4 and dev[1][1] <= 1e-5 and dev[1][2] <= 1e-6
    for a, b in zip(dev[0], dev[1]):
        assert 50.0 <= a / b <= 200.0
    # in between, the penalty trades smoothness for fit: |L K| falls and the data loss rises with lambda
    Lap = oracle.laplacian(m)
    prev_s, prev_d = np.inf, -np.inf
    for lam in (1e-3, 1e-1, 10.0):
        t = oracle.solve(p.R, p.I, m, oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu,
                                                        gain=p.gain, lam=lam))
        s = np.linalg.norm(Lap @ t)
        d = oracle.loss_grad(p.R, p.I, t, m, obj)[0]
        assert s < prev_s and d > prev_d
        prev_s, prev_d = s, d


@pytest.mark.parametrize("rho,var", [("gauss", "ccd_data"), ("huber", "emccd_model")])
def test_regularised_solution_is_stationary(c1_pair, rho, var):
    p = c1_pair
    m = p.m
    obj = oracle.Objective(rho=rho, var=var, sigma0=p.sigma0_adu, gain=p.gain, lam=0.5)
    th = oracle.solve(p.R, p.I, m, obj)
    L, g = oracle.loss_grad(p.R, p.I, th, m, obj)
    # the gradient of the regularised loss vanishes against the size of its two parts
    obj0 = oracle.Objective(rho=rho, var=var, sigma0=p.sigma0_adu, gain=p.gain)
    g0 = oracle.loss_grad(p.R, p.I, th, m, obj0)[1]
    gp = oracle.penalty(th, m, obj.lam, oracle.n_data(*p.I.shape, m))[1]
    assert np.max(np.abs(g)) <= 1e-7 * (np.max(np.abs(g0)) + np.max(np.abs(gp)))
    assert np.max(np.abs(gp)) > 1e-3 * np.max(np.abs(g0))  # the penalty is active


# --------------------------------------------------------------------- spatially varying background (Sec. 2.6)
def test_poly_terms_and_normalised_coordinates():
    assert oracle.poly_terms(0) == [(0, 0)]
    assert len(oracle.poly_terms(3)) == 10  # (d + 1)(d + 2) / 2
    assert all(a + b <= 3 for a, b in oracle.poly_terms(3))
    rows, cols, m = 41, 60, 5
    eta, xi = oracle.norm_coords(rows, cols, m)
    assert eta.shape == (rows - m + 1, cols - m + 1)
    # centred on the image centre (the valid region is symmetric about it), steps of 1/N
    assert abs(eta.sum()) < 1e-12 and abs(xi.sum()) < 1e-12
    assert np.allclose(np.diff(eta[0]), 1.0 / cols) and np.allclose(np.diff(xi[:, 0]), 1.0 / rows)
    assert np.all(np.abs(eta) < 0.5) and np.all(np.abs(xi) < 0.5)


def test_poly_background_of_degree_zero_is_the_constant_background(c1_pair):
    p = c1_pair
    th = oracle.init_theta(p.I, p.m)
    assert np.array_equal(oracle.model_poly(p.R, th, p.m, 0), oracle.model(p.R, th, p.m))
    obj = oracle.Objective(rho="huber", var="ccd_model", sigma0=p.sigma0_adu, gain=p.gain)
    L0, g0 = oracle.loss_grad(p.R, p.I, th, p.m, obj)
    L1, g1 = oracle.loss_grad_poly(p.R, p.I, th, p.m, obj, 0)
    assert L0 == pytest.approx(L1, rel=1e-14) and np.allclose(g0, g1, rtol=1e-12, atol=0)


def _tilted_target(p, coeffs, d):
    # the noiseless target with a background written out pixel by pixel from eq. polybackground
    # and eq. normcoords on the full target grid (independent of the oracle's design columns)
    H, W = p.R.shape
    I = sf.correlate_target(p.R.astype(np.float64), p.K_true, 0.0)
    xc, yc = (W - 1) / 2.0, (H - 1) / 2.0
    B = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            eta, xi = (x - xc) / W, (y - yc) / H
            B[y, x] = sum(c * eta ** a * xi ** b for c, (a, b) in zip(coeffs, oracle.poly_terms(d)))
    return I + B


def test_poly_background_noiseless_recovery(c1_pair):
    p = c1_pair
    m, d = p.m, 2
    coeffs = [40.0, 25.0, -60.0, -35.0, 80.0, 15.0]
    I = _tilted_target(p, coeffs, d)
    w = np.ones((p.R.shape[0] - m + 1, p.R.shape[1] - m + 1))
    th = oracle.solve_chi2_poly(p.R, I, m, w, d)
    assert np.allclose(th[:m * m], p.K_true.ravel(), rtol=0, atol=1e-9 * np.abs(p.K_true).max())
    assert np.allclose(th[m * m:], coeffs, rtol=1e-7, atol=1e-7)
    # a constant background cannot absorb the tilt: the fit is biased and leaves a residual
    th0 = oracle.solve_chi2(p.R, I, m, w)
    assert np.max(np.abs(th0[:m * m] - p.K_true.ravel())) > 1e-4 * np.abs(p.K_true).max()


def test_normalised_coordinates_condition_the_background_terms():
    # the paper's reason for eq. normcoords: the terms are closer to orthogonal than in raw pixel
    # coordinates (the normal matrix of the background columns is far better conditioned)
    rows, cols, m, d = 200, 300, 9, 3
    P = oracle.poly_columns(rows, cols, m, d).reshape(-1, len(oracle.poly_terms(d)))
    h = oracle.half(m)
    y, x = np.mgrid[h:rows - h, h:cols - h].astype(np.float64)
    Q = np.stack([x.ravel() ** a * y.ravel() ** b for a, b in oracle.poly_terms(d)], axis=1)
    assert np.linalg.cond(P.T @ P) < 1e-6 * np.linalg.cond(Q.T @ Q)


@pytest.mark.parametrize("rho,var", [("gauss", "ccd_data"), ("huber", "ccd_model")])
def test_poly_background_gradient_is_the_derivative(c1_pair, rho, var):
    p = c1_pair
    m, d = p.m, 2
    obj = oracle.Objective(rho=rho, var=var, sigma0=p.sigma0_adu, gain=p.gain)
    th = np.concatenate([p.K_true.ravel(), [5.0, 3.0, -2.0, 4.0, 1.0, -6.0]])
    _, g = oracle.loss_grad_poly(p.R, p.I, th, m, obj, d)
    for k in range(m * m, m * m + 6):
        e = np.zeros_like(th)
        e[k] = 1e-3
        fd = (oracle.loss_grad_poly(p.R, p.I, th + e, m, obj, d)[0]
              - oracle.loss_grad_poly(p.R, p.I, th - e, m, obj, d)[0]) / 2e-3
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-6 * np.abs(g).max())


def test_poly_hessian_is_the_jacobian_of_the_gradient(c1_pair):
    # every column of hessian_poly against central differences of loss_grad_poly's gradient (Cauchy loss,
    # model variance, degree 2), and the kernel block's penalty term with lambda > 0
    p = c1_pair
    m, d = p.m, 2
    th = np.concatenate([p.K_true.ravel() * 1.02, [5.0, 3.0, -2.0, 4.0, 1.0, -6.0]])
    for lam in (0.0, 0.3):
        obj = oracle.Objective(rho="cauchy", var="ccd_model", sigma0=p.sigma0_adu, gain=p.gain, c=2.3849, lam=lam)
        H = oracle.hessian_poly(p.R, p.I, th, m, obj, d)
        assert np.allclose(H, H.T, rtol=1e-12, atol=1e-13 * np.abs(H).max())
        cols = list(range(0, m * m, 7)) + list(range(m * m, m * m + 6))
        for k in cols:
            hk = 1e-6 if k < m * m else 1e-4
            e = np.zeros_like(th)
            e[k] = hk
            fd = (oracle.loss_grad_poly(p.R, p.I, th + e, m, obj, d)[1]
                  - oracle.loss_grad_poly(p.R, p.I, th - e, m, obj, d)[1]) / (2 * hk)
            assert np.allclose(fd, H[:, k], rtol=1e-5, atol=1e-6 * np.abs(H[:, k]).max()), k


def test_poly_hessian_of_degree_zero_is_the_hessian(c1_pair):
    p = c1_pair
    th = np.r_[p.K_true.ravel(), p.B0_true]
    obj = oracle.Objective(rho="huber", var="emccd_model", gain=p.gain, excess=2.0, lam=0.5)
    assert np.allclose(oracle.hessian_poly(p.R, p.I, th, p.m, obj, 0), oracle.hessian(p.R, p.I, th, p.m, obj),
                       rtol=1e-12, atol=0)


def test_solve_poly_chi2_is_the_normal_equations_solution(c1_pair):
    p = c1_pair
    m, d = p.m, 2
    obj = oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain)
    I = _tilted_target(p, [40.0, 25.0, -60.0, -35.0, 80.0, 15.0], d) + sf.rng_for(0, 77).normal(0, 3.0, p.R.shape)
    th = oracle.solve_poly(p.R, I, m, obj, d)
    ref = oracle.solve_chi2_poly(p.R, I, m, oracle.fixed_weights(obj, I, m), d)
    assert np.allclose(th, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_solve_poly_robust_loss_recovers_a_noiseless_background(c1_pair):
    # noiseless target with a degree-2 background: every residual vanishes at the truth, where the
    # Cauchy loss with fixed sigma takes its minimum
    p = c1_pair
    m, d = p.m, 2
    coeffs = [40.0, 25.0, -60.0, -35.0, 80.0, 15.0]
    I = _tilted_target(p, coeffs, d)
    obj = oracle.Objective(rho="cauchy", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain, c=2.3849)
    th = oracle.solve_poly(p.R, I, m, obj, d)
    assert np.allclose(th[:m * m], p.K_true.ravel(), rtol=0, atol=1e-8 * np.abs(p.K_true).max())
    assert np.allclose(th[m * m:], coeffs, rtol=1e-7, atol=1e-7)


def test_solve_poly_is_stationary_and_reduces_to_solve(c1_pair):
    p = c1_pair
    m = p.m
    obj = oracle.Objective(rho="cauchy", var="ccd_model", sigma0=p.sigma0_adu, gain=p.gain, c=2.3849)
    th0 = oracle.solve_poly(p.R, p.I, m, obj, 0)
    assert np.allclose(th0, oracle.solve(p.R, p.I, m, obj), rtol=1e-9, atol=1e-9 * np.abs(th0).max())
    I = _tilted_target(p, [10.0, 5.0, -8.0], 1) + (p.I - p.I_noiseless)
    th = oracle.solve_poly(p.R, I, m, obj, 1)
    _, g = oracle.loss_grad_poly(p.R, I, th, m, obj, 1)
    Iv = oracle.valid(I.astype(np.float64), m)
    _, gp, _ = oracle.pixel_terms(obj, Iv, oracle.model_poly(p.R, th, m, 1), m)
    scale = np.concatenate([oracle.grad_kernel(np.abs(p.R.astype(np.float64)), np.abs(gp), m),
                            np.abs(gp).reshape(-1) @ np.abs(oracle.poly_columns(*p.R.shape, m, 1)).reshape(-1, 3)])
    assert np.all(np.abs(g) <= 1e-10 * scale)
    np.linalg.cholesky(oracle.hessian_poly(p.R, I, th, m, obj, 1))
