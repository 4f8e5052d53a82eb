"""Shared parity measures of the GPU tests (no GPU work here).

Gradient, element by element: component j of the GPU gradient passes when
    |g_j - g_ref_j| <= tol * |g_ref_j| + floor * S_j,
S_j = sum_p |g_p X_pj| the summation scale of that component (X_pj = R_(p+j) for a kernel tap,
1 for B0), evaluated with the oracle's per-pixel derivative at the same parameters.  The relative
term is the spec bar; the floor term covers components that cancel to near zero, where a
relative error is undefined.  With FP64 sums on both sides the achieved error is about 1e-13 S_j,
so the default floor of 1e-9 S_j still fails any dropped, misplaced or wrongly signed term.
"""
import numpy as np

import oracle


def summation_scale(R, I, theta, m, o_or):
    """S_j = sum_p |g_p| |X_pj| for every parameter (kernel taps, then B0)."""
    R = np.asarray(R, np.float64)
    M = oracle.model(R, np.asarray(theta, np.float64), m)
    _, g, _ = oracle.pixel_terms(o_or, oracle.valid(np.asarray(I, np.float64), m), M, m)
    ag = np.abs(g)
    return np.concatenate([oracle.grad_kernel(np.abs(R), ag, m), [ag.sum()]])


def check_grad_elementwise(g, g_ref, scale, tol=1e-5, floor=1e-9):
    g = np.asarray(g, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    err = np.abs(g - g_ref)
    bound = tol * np.abs(g_ref) + floor * np.asarray(scale, np.float64)
    worst = int(np.argmax(err / np.maximum(bound, 1e-300)))
    assert np.all(err <= bound), (f"gradient component {worst}: |d| {err[worst]:.3e} > bound {bound[worst]:.3e} "
                                  f"(g_ref {g_ref[worst]:.3e}, scale {scale[worst]:.3e})")
    return float(np.max(err / np.maximum(scale, 1e-300)))
