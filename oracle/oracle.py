"""FP64 CPU oracle for the DIA kernel fit of Hitchcock et al. (PyTorchDIA).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library: the two correlations are plain C loops (``dia_oracle.c``),
everything else is numpy in float64.

What it computes, with the passage each part follows:

* ``model``          M = R (x) K + B0 on the valid region   (Sec. 2.1, eq. model_image_delta_basis)
* ``pixel_terms``    per-pixel loss l, dl/dM, d2l/dM2 for
                       - rho = z^2/2 (eq. chi_squared / eq. loss),
                       - Huber rho (eq. huber_loss, eq. huber_nll),
                       - Cauchy rho (c^2/2) ln(1 + z^2/c^2) (a wide-tailed drop-in, Sec. 2.4),
                     with sigma from explicit weights, from the data, or from the
                     model through the CCD (eq. CCDNM) or EMCCD (eq. EMCCDNM) noise
                     model; the + sum ln sigma term of eq. loss / eq. huber_nll is kept
                     only when sigma depends on the model.
* ``loss_grad``      L(theta) and its gradient (dL/dK = sum g R-shifted, dL/dB0 = sum g)
* ``normal_matrix``  X^T diag(w) X with X the (N_data x (m^2+1)) design matrix of eq. 2
                     (the B08 linear step of Sec. 1 / Sec. 2.1)
* ``solve_chi2``     the exact minimiser of 1/2 sum w r^2 by Cholesky
* ``solve``          stationary point of the non-quadratic objectives by damped Newton
                     (exact Hessian X^T diag(l'') X, since M is affine in theta)
* ``fit_clipped``    the B08 outer loop: refit with sigma from the previous model and
                     cumulative |z| > kappa clipping (Sec. 2.1 / Sec. 2.4)
* ``adam_step``      one bias-corrected Adam update (Sec. 2.3, Kingma & Ba defaults)
* ``lbfgs_direction`` the L-BFGS search direction by the two-loop recursion (Sec. 2.3)
* ``init_theta``     B0 = median(I), flat or Gaussian K (Sec. 2.9)
* ``photometric_scale``  P = sum K (eq. photometric_scale_factor)
* ``covariance``     Sec. 2.5: Sigma = F^-1 of the observed Fisher information F (eq. covmatrix),
                     standard errors sqrt(Sigma_pp) (eq. deltatheta), the error of P, and the
                     paper's validity tests of Sigma (determinant and eigenvalues positive)
* ``poly_terms``, ``norm_coords``, ``model_poly``, ``loss_grad_poly``, ``solve_chi2_poly``,
  ``hessian_poly``, ``solve_poly``
                     Sec. 2.6: the background B(x, y) = sum b_ab eta^a xi^b of degree d
                     (eq. polybackground) in the normalised coordinates of eq. normcoords,
                     replacing the constant B0 (the coefficient b_00 sits where B0 did)
* ``laplacian``, ``penalty``  Sec. 2.7: the kernel-pixel Laplacian L (eq. laplacian) and the MAP
                     penalty lambda N_data theta^T L^T L theta added to the loss (eq. regularised_loss);
                     ``loss_grad``, ``hessian``, ``solve`` and ``solve_chi2`` include it when
                     Objective.lam > 0

Where the paper is silent or ambiguous, the reading taken is stated where it is used.
Parity pins for every function live in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.linalg

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dia_oracle.c")
_LIB = os.path.join(_HERE, "libdia_oracle.so")


def build_oracle(force: bool = False) -> str:
    """Compile the C loops with gcc (IEEE double, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
                               "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _clib():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_oracle())
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_model.argtypes = [dp, i64, i64, i64, dp, i64, ctypes.c_double, dp]
        lib.oracle_model.restype = ctypes.c_int
        lib.oracle_grad_kernel.argtypes = [dp, i64, i64, i64, dp, i64, dp]
        lib.oracle_grad_kernel.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ----------------------------------------------------------------------------- geometry
def half(m: int) -> int:
    if m < 1 or m % 2 == 0:
        raise ValueError("kernel size must be odd and >= 1")
    return (m - 1) // 2


def valid(a: np.ndarray, m: int) -> np.ndarray:
    """The valid-region view of an array on the target grid (Sec. 2.1: N_data = (N - 2n)^2)."""
    h = half(m)
    return a[h:a.shape[0] - h, h:a.shape[1] - h]


def n_data(rows: int, cols: int, m: int) -> int:
    """Pixels of the valid region; also N_data of eq. regularised_loss (the reading of "number of
    target image pixels" consistent with the data term the penalty is weighed against)."""
    return (rows - m + 1) * (cols - m + 1)


def split_theta(theta, m):
    theta = np.asarray(theta, dtype=np.float64)
    return theta[:m * m].reshape(m, m), float(theta[m * m])


def photometric_scale(theta, m) -> float:
    """P = sum_lm K_lm, eq. photometric_scale_factor."""
    return float(np.sum(np.asarray(theta, dtype=np.float64)[:m * m]))


# ----------------------------------------------------------------------------- model
def model(R, theta, m) -> np.ndarray:
    """Valid model image, eq. model_image_delta_basis (direct loops in C)."""
    R = _f64(R)
    K, B0 = split_theta(theta, m)
    K = _f64(K)
    H, W = R.shape
    M = np.empty((H - m + 1, W - m + 1))
    if _clib().oracle_model(_ptr(R), H, W, W, _ptr(K), m, B0, _ptr(M)) != 0:
        raise ValueError("bad sizes")
    return M


def grad_kernel(R, g, m) -> np.ndarray:
    """dL/dK_ab = sum_ij g_ij R_(i+a)(j+b) over the valid region (direct loops in C)."""
    R = _f64(R)
    g = _f64(g)
    H, W = R.shape
    assert g.shape == (H - m + 1, W - m + 1)
    dK = np.empty(m * m)
    if _clib().oracle_grad_kernel(_ptr(R), H, W, W, _ptr(g), m, _ptr(dK)) != 0:
        raise ValueError("bad sizes")
    return dK


# ----------------------------------------------------------------------------- objective
@dataclass
class Objective:
    """A scalar objective: rho in {'gauss', 'huber', 'cauchy'} and the source of sigma.

    var: 'weights'     sigma^2 = 1 / weights (fixed)
         'ccd_data'    sigma^2 = max(sigma0^2/F^2 + max(I,0)/(G F), var_floor)       (eq. CCDNM on I, fixed)
         'ccd_model'   sigma^2 = max(sigma0^2/F^2 + max(M,0)/(G F), var_floor)       (eq. CCDNM on M)
         'emccd_data'  sigma^2 = max(E max(I,0)/(G F), var_floor)                    (eq. EMCCDNM on I, fixed)
         'emccd_model' sigma^2 = max(E max(M,0)/(G F), var_floor)                    (eq. EMCCDNM on M)
    weights / flat / mask are arrays on the target's full grid (mask: nonzero = use)."""
    rho: str = "gauss"
    var: str = "ccd_data"
    sigma0: float = 0.0
    gain: float = 1.0
    excess: float = 2.0
    var_floor: float = 1.0
    c: float = 1.345
    weights: Optional[np.ndarray] = None
    flat: Optional[np.ndarray] = None
    mask: Optional[np.ndarray] = None
    lam: float = 0.0  # lambda of eq. regularised_loss (0 = the maximum-likelihood fit)

    @property
    def model_sigma(self) -> bool:
        return self.var in ("ccd_model", "emccd_model")


def rho_psi_dpsi(rho: str, z: np.ndarray, c: float):
    """rho(z), psi = rho'(z) and psi'(z) for the three loss shapes."""
    if rho == "gauss":
        return 0.5 * z * z, z, np.ones_like(z)
    if rho == "huber":  # eq. huber_loss
        inner = np.abs(z) <= c
        r = np.where(inner, 0.5 * z * z, c * (np.abs(z) - 0.5 * c))
        p = np.where(inner, z, c * np.sign(z))
        d = np.where(inner, 1.0, 0.0)
        return r, p, d
    if rho == "cauchy":
        q = 1.0 + (z / c) ** 2
        return 0.5 * c * c * np.log1p((z / c) ** 2), z / q, (2.0 - q) / (q * q)
    raise ValueError(rho)


def _variance(obj: Objective, X: np.ndarray, F: np.ndarray):
    """sigma^2 as a function of X (I or M) and its derivative d sigma^2 / dX."""
    if obj.var.startswith("ccd"):
        raw = obj.sigma0 ** 2 / (F * F) + np.maximum(X, 0.0) / (obj.gain * F)
        slope = 1.0 / (obj.gain * F)
    elif obj.var.startswith("emccd"):
        raw = obj.excess * np.maximum(X, 0.0) / (obj.gain * F)
        slope = obj.excess / (obj.gain * F)
    else:
        raise ValueError(obj.var)
    v = np.maximum(raw, obj.var_floor)
    dv = np.where((X > 0.0) & (raw > obj.var_floor), slope, 0.0)
    return v, dv


def pixel_terms(obj: Objective, Iv: np.ndarray, M: np.ndarray, m: int):
    """Per valid pixel: loss l, g = dl/dM and h = d2l/dM2 (masked pixels give zeros).

    Fixed sigma:  l = rho(z), z = (I - M)/sigma, g = -psi(z)/sigma, h = psi'(z)/sigma^2.
    Model sigma:  l = rho(z) + ln sigma (eq. loss / eq. huber_nll), sigma^2 = v(M), v' = dv/dM,
                  z' = -v^-1/2 - r v' / (2 v^3/2),  z'' = v' / v^3/2 + 3 r v'^2 / (4 v^5/2),
                  g = psi z' + v'/(2v),  h = psi' z'^2 + psi z'' - v'^2/(2 v^2)."""
    shape = M.shape
    F = np.ones(shape) if obj.flat is None else _f64(valid(obj.flat, m))
    r = Iv - M
    if obj.var == "weights":
        w = _f64(valid(obj.weights, m))
        sw = np.sqrt(w)
        z = r * sw
        rr, p, dp = rho_psi_dpsi(obj.rho, z, obj.c)
        l, g, h = rr, -p * sw, dp * w
    elif not obj.model_sigma:
        v, _ = _variance(obj, Iv, F)
        s = np.sqrt(v)
        z = r / s
        rr, p, dp = rho_psi_dpsi(obj.rho, z, obj.c)
        l, g, h = rr, -p / s, dp / v
    else:
        v, dv = _variance(obj, M, F)
        s = np.sqrt(v)
        z = r / s
        rr, p, dp = rho_psi_dpsi(obj.rho, z, obj.c)
        z1 = -1.0 / s - r * dv / (2.0 * v * s)
        z2 = dv / (v * s) + 0.75 * r * dv * dv / (v * v * s)
        l = rr + 0.5 * np.log(v)
        g = p * z1 + dv / (2.0 * v)
        h = dp * z1 * z1 + p * z2 - dv * dv / (2.0 * v * v)
    if obj.mask is not None:
        use = valid(obj.mask, m) != 0
        l, g, h = np.where(use, l, 0.0), np.where(use, g, 0.0), np.where(use, h, 0.0)
    return l, g, h


def loss_grad(R, I, theta, m, obj: Objective):
    """L(theta) = sum over valid unmasked pixels of l, and its gradient [dL/dK (m*m), dL/dB0];
    plus the penalty of eq. regularised_loss when obj.lam > 0."""
    R = _f64(R)
    Iv = _f64(valid(_f64(I), m))
    M = model(R, theta, m)
    l, g, _ = pixel_terms(obj, Iv, M, m)
    grad = np.empty(m * m + 1)
    grad[:m * m] = grad_kernel(R, g, m)
    grad[m * m] = np.sum(g)
    L = float(np.sum(l))
    if obj.lam > 0.0:
        p, pg, _ = penalty(theta, m, obj.lam, n_data(*np.shape(I), m))
        L += p
        grad += pg
    return L, grad


# ----------------------------------------------------------------------------- spatially varying background
def poly_terms(d: int):
    """Exponents (a, b) of the terms eta^a xi^b of eq. polybackground, in its summation order
    (a = 0..d outer, b = 0..d-a inner); b_00 is the constant background B0."""
    if d < 0:
        raise ValueError("degree must be >= 0")
    return [(a, b) for a in range(d + 1) for b in range(d - a + 1)]


def norm_coords(rows: int, cols: int, m: int):
    """eq. normcoords on the valid region: eta = (x - x_c) / N_x along the columns, xi = (y - y_c) / N_y
    along the rows, (x, y) the pixel's coordinates on the target grid and (x_c, y_c) = ((N_x - 1)/2,
    (N_y - 1)/2) its centre (the reading of "image centre" for pixel-centred integer coordinates)."""
    h = half(m)
    x = np.arange(h, cols - h, dtype=np.float64)
    y = np.arange(h, rows - h, dtype=np.float64)
    eta = (x - (cols - 1) / 2.0) / cols
    xi = (y - (rows - 1) / 2.0) / rows
    return (np.broadcast_to(eta[None, :], (y.size, x.size)).copy(),
            np.broadcast_to(xi[:, None], (y.size, x.size)).copy())


def poly_columns(rows: int, cols: int, m: int, d: int) -> np.ndarray:
    """The background's design columns on the valid region, (Hv, Wv, n_b): eta^a xi^b per term."""
    eta, xi = norm_coords(rows, cols, m)
    return np.stack([eta ** a * xi ** b for a, b in poly_terms(d)], axis=-1)


def model_poly(R, theta, m, d):
    """M = R (x) K + B(x, y) on the valid region (eq. model_image with eq. polybackground);
    theta = [K (m*m, a-major), b in poly_terms(d) order]."""
    theta = _f64(theta)
    nb = len(poly_terms(d))
    if theta.size != m * m + nb:
        raise ValueError("theta must hold m*m kernel values and the background coefficients")
    M = model(R, np.concatenate([theta[:m * m], [0.0]]), m)
    return M + poly_columns(*np.shape(R), m, d) @ theta[m * m:]


def loss_grad_poly(R, I, theta, m, obj: Objective, d):
    """L(theta) and [dL/dK, dL/db] with the polynomial background; the penalty of eq.
    regularised_loss acts on the kernel only (L is zero on every background coefficient)."""
    theta = _f64(theta)
    Iv = _f64(valid(_f64(I), m))
    M = model_poly(R, theta, m, d)
    l, g, _ = pixel_terms(obj, Iv, M, m)
    P = poly_columns(*np.shape(R), m, d)
    grad = np.concatenate([grad_kernel(R, g, m), np.tensordot(g, P, axes=([0, 1], [0, 1]))])
    L = float(np.sum(l))
    if obj.lam > 0.0:
        p, pg, _ = penalty(np.concatenate([theta[:m * m], [0.0]]), m, obj.lam, n_data(*np.shape(I), m))
        L += p
        grad[:m * m] += pg[:m * m]
    return L, grad


def normal_matrix_poly(R, m, d, w, y=None):
    """X^T diag(w) X and X^T (w y) for the design [R windows (m*m), background terms (n_b)]."""
    R = _f64(R)
    Hv, Wv = R.shape[0] - m + 1, R.shape[1] - m + 1
    P = poly_columns(*R.shape, m, d).reshape(Hv * Wv, -1)
    win = np.lib.stride_tricks.sliding_window_view(R, (m, m)).reshape(Hv * Wv, m * m)
    X = np.concatenate([win, P], axis=1)
    WX = X * w.reshape(-1)[:, None]
    return X.T @ WX, (None if y is None else WX.T @ y.reshape(-1))


def solve_chi2_poly(R, I, m, w, d, refine: int = 3) -> np.ndarray:
    """Exact minimiser of 1/2 sum w (I - M)^2 with the polynomial background, by Cholesky with
    residual refinement (each refinement an exact Newton step on the quadratic)."""
    Iv = _f64(valid(_f64(I), m))
    A, b = normal_matrix_poly(R, m, d, w, Iv)
    cf = scipy.linalg.cho_factor(A, lower=True)
    theta = scipy.linalg.cho_solve(cf, b)
    P = poly_columns(*np.shape(R), m, d)
    for _ in range(refine):
        gv = w * (model_poly(R, theta, m, d) - Iv)
        g = np.concatenate([grad_kernel(R, gv, m), np.tensordot(gv, P, axes=([0, 1], [0, 1]))])
        theta = theta - scipy.linalg.cho_solve(cf, g)
    return theta


def _penalty_poly(theta, m, d, lam, N):
    """The penalty of eq. regularised_loss with a polynomial background: it acts on the kernel only,
    so (value, gradient, Hessian) are those of the kernel block with every coefficient free."""
    nb = len(poly_terms(d))
    p, pg, ph = penalty(np.concatenate([_f64(theta)[:m * m], [0.0]]), m, lam, N)
    g = np.zeros(m * m + nb)
    g[:m * m] = pg[:m * m]
    H = np.zeros((m * m + nb, m * m + nb))
    H[:m * m, :m * m] = ph[:m * m, :m * m]
    return p, g, H


def hessian_poly(R, I, theta, m, obj: Objective, d):
    """X^T diag(l'') X for the design [R windows, background terms] (Sec. 2.5 with Sec. 2.6), plus the
    penalty's Hessian on the kernel block when obj.lam > 0."""
    Iv = _f64(valid(_f64(I), m))
    M = model_poly(R, theta, m, d)
    _, _, h = pixel_terms(obj, Iv, M, m)
    A, _ = normal_matrix_poly(R, m, d, h)
    if obj.lam > 0.0:
        A = A + _penalty_poly(theta, m, d, obj.lam, n_data(*np.shape(I), m))[2]
    return A


def solve_poly(R, I, m, obj: Objective, d, max_iter: int = 100):
    """Stationary point of L(theta) with the degree-d background: the steps of ``solve`` (damped Newton
    on the exact Hessian, the IRLS surrogate where it is not positive definite, Armijo backtracking)
    on the design [R windows, background terms].  Starts from the chi-squared solution with sigma from
    the data (for rho = gauss with fixed sigma that solution is the answer, refined by Newton steps)."""
    Iv = _f64(valid(_f64(I), m))
    N = n_data(*np.shape(I), m)
    start = Objective(rho="gauss", var=obj.var.replace("model", "data"), sigma0=obj.sigma0, gain=obj.gain,
                      excess=obj.excess, var_floor=obj.var_floor, weights=obj.weights, flat=obj.flat, mask=obj.mask)
    theta = solve_chi2_poly(R, I, m, fixed_weights(start, I, m), d)
    L, g = loss_grad_poly(R, I, theta, m, obj, d)
    for _ in range(max_iter):
        M = model_poly(R, theta, m, d)
        A = hessian_poly(R, I, theta, m, obj, d)
        try:
            step = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(A, lower=True), g)
        except np.linalg.LinAlgError:
            A, _ = normal_matrix_poly(R, m, d, _irls_weights(obj, Iv, M, m))
            if obj.lam > 0.0:
                A = A + _penalty_poly(theta, m, d, obj.lam, N)[2]
            step = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(A, lower=True), g)
        slope = float(g @ step)
        t = 1.0
        while True:
            cand = theta + t * step
            Lc, gc = loss_grad_poly(R, I, cand, m, obj, d)
            if Lc <= L + 1e-4 * t * slope or t < 1e-10:
                break
            t *= 0.5
        done = np.linalg.norm(t * step) <= 1e-13 * max(1.0, np.linalg.norm(theta)) or Lc >= L
        if Lc <= L:
            theta, L, g = cand, Lc, gc
        if done:
            break
    return theta


# ----------------------------------------------------------------------------- kernel regulariser
def laplacian(m) -> np.ndarray:
    """Sec. 2.7, eq. laplacian: the (m*m + 1)^2 Laplacian of the graph whose nodes are the kernel
    pixels (a-major order, as in theta) and whose edges join pixels sharing a side (the reading
    of "adjacent": 4-neighbours).  Diagonal = number of neighbours, -1 for each adjacent pair,
    and a zero row and column for B0."""
    n = m * m
    L = np.zeros((n + 1, n + 1))
    for a in range(m):
        for b in range(m):
            u = a * m + b
            for da, db in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                if 0 <= a + da < m and 0 <= b + db < m:
                    L[u, (a + da) * m + (b + db)] = -1.0
                    L[u, u] += 1.0
    return L


def penalty(theta, m, lam, N):
    """lambda N theta^T L^T L theta, its gradient 2 lambda N L^T L theta and Hessian 2 lambda N L^T L."""
    L = laplacian(m)
    theta = _f64(theta)
    Lt = L @ theta
    Hp = 2.0 * lam * N * (L.T @ L)
    return float(lam * N * (Lt @ Lt)), Hp @ theta, Hp


# ----------------------------------------------------------------------------- normal matrix
def design_rows(R, m, i0, i1):
    """Rows of the design matrix X for valid rows i0..i1-1: columns R_(i+a)(j+b) (a-major), then 1."""
    R = _f64(R)
    Wv = R.shape[1] - m + 1
    win = np.lib.stride_tricks.sliding_window_view(R[i0:i1 + m - 1], (m, m))  # (i1-i0, Wv, m, m)
    X = np.empty(((i1 - i0) * Wv, m * m + 1))
    X[:, :m * m] = win.reshape(-1, m * m)
    X[:, m * m] = 1.0
    return X


def normal_matrix(R, m, w, y=None, chunk_px: int = 1 << 16):
    """A = X^T diag(w) X and b = X^T (w * y) over the valid region (w, y valid-shaped)."""
    R = _f64(R)
    Hv, Wv = R.shape[0] - m + 1, R.shape[1] - m + 1
    n = m * m + 1
    A = np.zeros((n, n))
    b = np.zeros(n)
    rows = max(1, chunk_px // Wv)
    for i0 in range(0, Hv, rows):
        i1 = min(Hv, i0 + rows)
        X = design_rows(R, m, i0, i1)
        wc = w[i0:i1].reshape(-1)
        WX = X * wc[:, None]
        A += X.T @ WX
        if y is not None:
            b += WX.T @ y[i0:i1].reshape(-1)
    return A, b


def fixed_weights(obj: Objective, I, m) -> np.ndarray:
    """w = 1/sigma^2 on the valid region for a fixed-sigma objective (zero where masked)."""
    Iv = _f64(valid(_f64(I), m))
    F = np.ones(Iv.shape) if obj.flat is None else _f64(valid(obj.flat, m))
    if obj.var == "weights":
        w = _f64(valid(obj.weights, m)).copy()
    elif not obj.model_sigma:
        v, _ = _variance(obj, Iv, F)
        w = 1.0 / v
    else:
        raise ValueError("sigma depends on the model")
    if obj.mask is not None:
        w = np.where(valid(obj.mask, m) != 0, w, 0.0)
    return w


def solve_chi2(R, I, m, w, refine: int = 3, lam: float = 0.0) -> np.ndarray:
    """Exact minimiser of 1/2 sum w (I - M)^2 [+ lambda N_data theta^T L^T L theta]:
    (X^T W X + 2 lambda N_data L^T L) theta = X^T W I, by Cholesky (Sec. 2.7 for the penalty).

    The normal equations square the condition number of X, so the Cholesky solution is refined
    with the residual gradient X^T W (X theta - I) taken from the direct loops (each refinement
    is one exact Newton step on the quadratic)."""
    Iv = _f64(valid(_f64(I), m))
    A, b = normal_matrix(R, m, w, Iv)
    Hp = penalty(np.zeros(m * m + 1), m, lam, n_data(*np.shape(I), m))[2] if lam > 0.0 else None
    if Hp is not None:
        A = A + Hp
    cf = scipy.linalg.cho_factor(A, lower=True)
    theta = scipy.linalg.cho_solve(cf, b)
    for _ in range(refine):
        gv = w * (model(R, theta, m) - Iv)
        g = np.concatenate([grad_kernel(R, gv, m), [np.sum(gv)]])
        if Hp is not None:
            g = g + Hp @ theta
        theta = theta - scipy.linalg.cho_solve(cf, g)
    return theta


def hessian(R, I, theta, m, obj: Objective):
    """X^T diag(l'') X, plus 2 lambda N_data L^T L when obj.lam > 0 (Sec. 2.5, Sec. 2.7)."""
    Iv = _f64(valid(_f64(I), m))
    M = model(R, theta, m)
    _, _, h = pixel_terms(obj, Iv, M, m)
    A, _ = normal_matrix(R, m, h)
    if obj.lam > 0.0:
        A = A + penalty(theta, m, obj.lam, n_data(*np.shape(I), m))[2]
    return A


def covariance(F) -> dict:
    """Sec. 2.5 for a Fisher information F (n x n, the last parameter B0, the first n - 1 the kernel):
      cov     = F^-1                                   (eq. covmatrix)
      sigma   = sqrt(cov_pp)                           (eq. deltatheta, the Cramer-Rao bound)
      sigma_P = sqrt(1^T cov_KK 1), the error of P = sum K (eq. photometric_scale_factor)
      valid   = the paper's two tests of cov: its determinant is positive, and after
                diagonalisation every eigenvalue is positive
      logdet  = ln det cov (NaN when the determinant is not positive)"""
    F = _f64(F)
    n = F.shape[0]
    cov = np.linalg.inv(F)
    cov = 0.5 * (cov + cov.T)
    ev = np.linalg.eigvalsh(cov)
    sign, logdet = np.linalg.slogdet(cov)
    d = np.diag(cov)
    sP2 = float(cov[:n - 1, :n - 1].sum())
    return dict(cov=cov, sigma=np.sqrt(np.where(d > 0, d, np.nan)),
                sigma_P=float(np.sqrt(sP2)) if sP2 > 0 else float("nan"),
                valid=bool(sign > 0 and np.all(ev > 0)), logdet=float(logdet) if sign > 0 else float("nan"),
                eigvals=ev)


def _irls_weights(obj: Objective, Iv, M, m):
    """A positive surrogate curvature psi(z)/(z sigma^2) at the current sigma (majorises rho)."""
    F = np.ones(M.shape) if obj.flat is None else _f64(valid(obj.flat, m))
    if obj.var == "weights":
        v = 1.0 / np.maximum(_f64(valid(obj.weights, m)), 1e-300)
    else:
        v, _ = _variance(obj, M if obj.model_sigma else Iv, F)
    z = (Iv - M) / np.sqrt(v)
    _, p, _ = rho_psi_dpsi(obj.rho, z, obj.c)
    ratio = np.where(np.abs(z) > 1e-12, p / np.where(np.abs(z) > 1e-12, z, 1.0), 1.0)
    w = ratio / v
    if obj.var == "weights":
        w = np.where(_f64(valid(obj.weights, m)) > 0, w, 0.0)
    if obj.mask is not None:
        w = np.where(valid(obj.mask, m) != 0, w, 0.0)
    return w


def solve(R, I, m, obj: Objective, theta0=None, max_iter: int = 100, verbose: bool = False):
    """Stationary point of L(theta) (eq. loss / eq. huber_nll / Cauchy).

    rho = gauss with fixed sigma is quadratic: one Cholesky solve.  Otherwise damped Newton on the
    FP64 loss: Hessian X^T diag(l'') X (exact, M is affine in theta); where it is not positive
    definite the IRLS surrogate X^T diag(psi/(z sigma^2)) X is used; Armijo backtracking.  Stops when
    the step is below 1e-13 of |theta| or the loss stops decreasing."""
    if obj.rho == "gauss" and not obj.model_sigma:
        return solve_chi2(R, I, m, fixed_weights(obj, I, m), lam=obj.lam)
    Iv = _f64(valid(_f64(I), m))
    Hp = penalty(np.zeros(m * m + 1), m, obj.lam, n_data(*np.shape(I), m))[2] if obj.lam > 0.0 else 0.0
    if theta0 is None:
        if obj.model_sigma:
            start = Objective(rho="gauss", var=obj.var.replace("model", "data"), sigma0=obj.sigma0,
                              gain=obj.gain, excess=obj.excess, var_floor=obj.var_floor,
                              flat=obj.flat, mask=obj.mask)
        else:
            start = Objective(rho="gauss", var=obj.var, sigma0=obj.sigma0, gain=obj.gain,
                              excess=obj.excess, var_floor=obj.var_floor, weights=obj.weights,
                              flat=obj.flat, mask=obj.mask)
        theta = solve_chi2(R, I, m, fixed_weights(start, I, m), lam=obj.lam)
    else:
        theta = _f64(theta0).copy()
    L, g = loss_grad(R, I, theta, m, obj)
    for it in range(max_iter):
        M = model(R, theta, m)
        _, _, h = pixel_terms(obj, Iv, M, m)
        A, _ = normal_matrix(R, m, h)
        try:
            step = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(A + Hp, lower=True), g)
        except np.linalg.LinAlgError:
            A, _ = normal_matrix(R, m, _irls_weights(obj, Iv, M, m))
            step = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(A + Hp, lower=True), g)
        slope = float(g @ step)
        t = 1.0
        while True:
            cand = theta + t * step
            Lc, gc = loss_grad(R, I, cand, m, obj)
            if Lc <= L + 1e-4 * t * slope or t < 1e-10:
                break
            t *= 0.5
        if verbose:
            print(f"newton {it}: L={Lc:.17g} t={t:g} |step|={np.linalg.norm(t * step):.3e}")
        done = np.linalg.norm(t * step) <= 1e-13 * max(1.0, np.linalg.norm(theta)) or Lc >= L
        if Lc <= L:
            theta, L, g = cand, Lc, gc
        if done:
            break
    return theta


# ----------------------------------------------------------------------------- B08 outer loop
def fit_clipped(R, I, m, obj: Objective, kappa: float = 3.0, max_outer: int = 3):
    """B08-style iteration (Sec. 2.1 and 2.4): fit 1 with sigma from the data, then refit with
    sigma^2 = v(M_prev) held fixed (eq. CCDNM) and the pixels with |z| > kappa clipped
    (z = (I - M_prev)/sigma, cumulative masks), until max_outer fits or the mask stops changing.
    Returns (theta, mask on the full grid (1 = used), number of fits)."""
    I64 = _f64(I)
    H, W = I64.shape
    Iv = valid(I64, m)
    h = half(m)
    base_mask = np.ones((H, W), np.uint8) if obj.mask is None else (np.asarray(obj.mask) != 0).astype(np.uint8)
    mask = base_mask.copy()
    cur = Objective(rho="gauss", var=obj.var.replace("model", "data"), sigma0=obj.sigma0, gain=obj.gain,
                    excess=obj.excess, var_floor=obj.var_floor, flat=obj.flat, mask=mask)
    theta = solve_chi2(R, I64, m, fixed_weights(cur, I64, m))
    n_fit = 1
    while n_fit < max_outer:
        M = model(R, theta, m)
        F = np.ones(M.shape) if obj.flat is None else _f64(valid(obj.flat, m))
        v, _ = _variance(Objective(var=obj.var.replace("data", "model"), sigma0=obj.sigma0, gain=obj.gain,
                                   excess=obj.excess, var_floor=obj.var_floor), M, F)
        z = (Iv - M) / np.sqrt(v)
        new_mask = mask.copy()
        new_mask[h:H - h, h:W - h] &= (np.abs(z) <= kappa).astype(np.uint8)
        wfull = np.zeros((H, W))
        wfull[h:H - h, h:W - h] = 1.0 / v
        changed = not np.array_equal(new_mask, mask)
        mask = new_mask
        cur = Objective(rho="gauss", var="weights", weights=wfull, mask=mask)
        theta = solve_chi2(R, I64, m, fixed_weights(cur, I64, m))
        n_fit += 1
        if not changed:
            break
    return theta, mask, n_fit


# ----------------------------------------------------------------------------- optimiser pieces
def adam_step(theta, grad, m1, v1, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, cited in Sec. 2.3), bias-corrected; lr may be per-parameter.
    Returns (theta', m1', v1'); t is the 1-based step number."""
    m1 = beta1 * np.asarray(m1, np.float64) + (1.0 - beta1) * grad
    v1 = beta2 * np.asarray(v1, np.float64) + (1.0 - beta2) * grad * grad
    mhat = m1 / (1.0 - beta1 ** t)
    vhat = v1 / (1.0 - beta2 ** t)
    return np.asarray(theta, np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m1, v1


def lbfgs_direction(g, pairs):
    """The L-BFGS search direction d = -H g of Sec. 2.3 (eq. newtonupdate with H the quasi-Newton
    inverse-Hessian estimate), by the two-loop recursion of Nocedal & Wright (Numerical Optimization,
    Algorithm 7.4): pairs = [(s_i, y_i)] oldest first, each with s_i . y_i > 0; the initial estimate
    is gamma I with gamma = s.y / y.y of the newest pair (1 when there is none).  Returns d."""
    q = np.array(g, np.float64)
    alphas = []
    for s, y in reversed(pairs):
        a = float(s @ q) / float(s @ y)
        q = q - a * y
        alphas.append(a)
    gamma = float(pairs[-1][0] @ pairs[-1][1]) / float(pairs[-1][1] @ pairs[-1][1]) if pairs else 1.0
    r = gamma * q
    for (s, y), a in zip(pairs, reversed(alphas)):
        b = float(y @ r) / float(s @ y)
        r = r + (a - b) * s
    return -r


def init_theta(I, m, kind: str = "flat", phi_K: float = 1.0):
    """Sec. 2.9: B0 = median of the target image; K flat at 1/N_K, or a symmetric Gaussian with
    standard deviation phi_K normalised to sum 1.  An even count takes the mean of the two middle values."""
    theta = np.empty(m * m + 1)
    if kind == "flat":
        theta[:m * m] = 1.0 / (m * m)
    elif kind == "gauss":
        h = half(m)
        a, b = np.meshgrid(np.arange(m) - h, np.arange(m) - h, indexing="ij")
        k = np.exp(-0.5 * (a * a + b * b) / (phi_K * phi_K))
        theta[:m * m] = (k / k.sum()).ravel()
    else:
        raise ValueError(kind)
    theta[m * m] = float(np.median(_f64(I)))
    return theta


def huber_constant(c: float, n: int) -> float:
    """Normalising constant Q of eq. huber_nll (Sec. 2.4): N ln(sqrt(2 pi) erf(c/sqrt 2) + 2 exp(-c^2/2)/c)."""
    from math import erf, exp, log, pi, sqrt
    return n * log(sqrt(2.0 * pi) * erf(c / sqrt(2.0)) + 2.0 * exp(-c * c / 2.0) / c)
