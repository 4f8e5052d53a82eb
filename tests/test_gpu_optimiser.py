"""The device optimiser's arithmetic (Sec. 2.3 eqs. update and newtonupdate, Sec. 2.9 schedule)
against the oracle's Adam step and L-BFGS two-loop direction, step by step.

The device works in the coordinates u = (c K, B0 + s sum K), s the mean and c the RMS spread of
the reference (the same optimum as the raw parameters).  The replica below maps every point
the same way, evaluates the oracle's FP64 loss and gradient at the FP32 rounding of each point
(the values the fused pass reads), moves with ``oracle.adam_step`` (learning rate lr_K c for the
kernel coordinates, lr_B0 for the background) and, after the switch, with
``oracle.lbfgs_direction`` over the curvature pairs the Adam steps produced.  The device's
points are read back through ``max_eval`` caps with the Newton polish off.  Agreement is to a
few FP32 spacings of theta: both sides round the same FP64 values, which differ only by the
order of FP64 sums.  A wrong bias correction, learning-rate scale, sign or curvature pair moves
a step by O(1) of itself.
"""
import numpy as np
import pytest
import torch

import oracle
from synthetic import starfield as sf

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = torch.device("cuda:0")
LR_K, LR_B0 = 1e-3, 10.0


@pytest.fixture(scope="module")
def dia():
    import paper_2104_13715_amd as d
    return d


def gpu(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


class Replica:
    """The optimiser's path in u, written with the oracle's pieces."""

    def __init__(self, p, m, o_or):
        self.p, self.m, self.o = p, m, o_or
        R = p.R.astype(np.float64)
        self.s = R.mean()
        self.c = np.sqrt((R * R).mean() - self.s * self.s)
        th0 = oracle.init_theta(p.I, m, "flat")
        self.u = self.to_u(th0)

    def to_u(self, th):
        m2 = self.m * self.m
        return np.r_[self.c * th[:m2], th[m2] + self.s * th[:m2].sum()]

    def theta32(self, u):
        m2 = self.m * self.m
        k = u[:m2] / self.c
        return np.r_[k.astype(np.float32), np.float32(u[m2] - self.s * k.sum())].astype(np.float32)

    def eval(self, u):
        """(loss, gradient in u) at the FP32 rounding of the point u."""
        m2 = self.m * self.m
        L, g = oracle.loss_grad(self.p.R, self.p.I, self.theta32(u).astype(np.float64), self.m, self.o)
        gu = np.r_[(g[:m2] - self.s * g[m2]) / self.c, g[m2]]
        return L, gu

    def lr(self):
        m2 = self.m * self.m
        return np.r_[np.full(m2, LR_K * self.c), LR_B0]


def push(pairs, s, y, H=10):
    sy, ss, yy = s @ y, s @ s, y @ y
    if sy > 1e-12 * np.sqrt(ss * yy) and sy > 0:
        pairs.append((s, y))
        del pairs[:-H]


def spacing(th):
    return np.spacing(np.abs(th).astype(np.float32)).astype(np.float64)


@pytest.fixture(scope="module")
def setup(dia):
    p = sf.config1()
    m = p.m
    o_or = oracle.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain)
    o_gpu = dia.Objective(rho="gauss", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain)
    return p, m, o_or, o_gpu, gpu(p.R), gpu(p.I)


def device_point(dia, setup, max_eval, max_adam=5000):
    p, m, _, o_gpu, R, I = setup
    return dia.fit(R, I, m, o_gpu, max_eval=max_eval, max_adam=max_adam, poll_every=1, max_newton=0)


def test_device_adam_steps_match_oracle_adam_step(dia, setup):
    p, m, o_or, _, _, _ = setup
    rep = Replica(p, m, o_or)
    u = rep.u.copy()
    m1 = np.zeros_like(u)
    v1 = np.zeros_like(u)
    for t in range(1, 5):
        L, g = rep.eval(u)
        u, m1, v1 = oracle.adam_step(u, g, m1, v1, t, rep.lr())
        # t evaluations, t Adam updates: the device's point after its t-th update
        res = device_point(dia, setup, max_eval=t)
        assert res.n_adam == t and res.n_lbfgs == 0 and res.n_eval == t
        th_dev = res.theta.cpu().double().numpy()
        th_rep = rep.theta32(u).astype(np.float64)
        err = np.abs(th_dev - th_rep)
        assert np.all(err <= 4.0 * spacing(th_rep)), (t, int(np.argmax(err / spacing(th_rep))), err.max())
    # the first step is lr times the gradient's sign in every coordinate (bias-corrected moments)
    _, g0 = rep.eval(rep.u)
    step1 = oracle.adam_step(rep.u, g0, np.zeros_like(u), np.zeros_like(u), 1, rep.lr())[0] - rep.u
    np.testing.assert_allclose(step1, -rep.lr() * np.sign(g0), rtol=1e-6)


def test_device_lbfgs_direction_matches_oracle_two_loop(dia, setup):
    # three Adam steps, the switch (max_adam) and the first L-BFGS trial at step length 1: the
    # device's history holds the three Adam curvature pairs, so its direction is the oracle's
    # two-loop direction over the same pairs
    p, m, o_or, _, _, _ = setup
    A = 3
    rep = Replica(p, m, o_or)
    u = rep.u.copy()
    m1 = np.zeros_like(u)
    v1 = np.zeros_like(u)
    pairs = []
    L, g = rep.eval(u)
    for t in range(1, A + 1):
        u_new, m1, v1 = oracle.adam_step(u, g, m1, v1, t, rep.lr())
        L_new, g_new = rep.eval(u_new)
        push(pairs, u_new - u, g_new - g)
        u, L, g = u_new, L_new, g_new
    d = oracle.lbfgs_direction(g, pairs)
    gtd = float(g @ d)
    assert gtd < 0
    L_t, g_t = rep.eval(u + d)
    dll = L_t - L
    dL = dll if abs(dll) > 1e-5 * abs(L) else 0.5 * float((g + g_t) @ d)
    accepted = dL <= 1e-4 * gtd
    assert accepted, "the replica's first L-BFGS trial should be accepted at step length 1"
    res = device_point(dia, setup, max_eval=A + 2, max_adam=A)
    assert res.n_adam == A and res.n_lbfgs == 1, (res.n_adam, res.n_lbfgs)
    th_dev = res.theta.cpu().double().numpy()
    th_rep = rep.theta32(u + d).astype(np.float64)
    th_from = rep.theta32(u).astype(np.float64)
    err = np.abs(th_dev - th_rep)
    assert np.all(err <= 4.0 * spacing(th_rep) + 1e-9 * np.abs(th_rep - th_from)), \
        (int(np.argmax(err)), err.max())
    # the accepted L-BFGS step lowered the loss; the device reports the FP64 loss of that point
    assert L_t < L
    assert abs(res.loss - L_t) <= 1e-12 * abs(L_t)


def test_fit_without_polish_lowers_the_loss_and_reports_its_stop(dia, setup):
    p, m, o_or, o_gpu, R, I = setup
    res = dia.fit(R, I, m, o_gpu, max_newton=0)
    L0 = oracle.loss_grad(p.R, p.I, oracle.init_theta(p.I, m, "flat").astype(np.float32).astype(np.float64), m,
                          o_or)[0]
    L1 = oracle.loss_grad(p.R, p.I, res.theta.cpu().double().numpy(), m, o_or)[0]
    assert res.n_newton == 0 and res.stop == res.first_order_stop and res.stop != "newton"
    assert res.n_adam > 0 and res.n_lbfgs > 0
    assert L1 < L0 and abs(res.loss - L1) <= 1e-6 * abs(L1)


def test_first_order_cap_is_reported_beside_a_converged_polish(dia, setup):
    p, m, o_or, o_gpu, R, I = setup
    res = dia.fit(R, I, m, o_gpu, max_adam=2, max_lbfgs=2)
    assert res.status == dia.OK and res.stop == "newton"
    assert res.first_order_stop == "cap" and res.n_lbfgs == 2


@pytest.mark.parametrize("rho,var", [("gauss", "ccd_data"), ("cauchy", "ccd_model")])
def test_no_lbfgs_phase_hands_over_to_newton(dia, rho, var):
    # max_lbfgs = 0: the first-order part ends at the Adam switch and the exact-Hessian Newton steps take
    # the fit to the oracle's minimiser (the eq. newtonupdate form with the exact Hessian)
    p = sf.config1()
    m = p.m
    o_or = oracle.Objective(rho=rho, var=var, sigma0=p.sigma0_adu, gain=p.gain, c=2.3849)
    o_gpu = dia.Objective(rho=rho, var=var, sigma0=p.sigma0_adu, gain=p.gain, c=2.3849)
    res = dia.fit(gpu(p.R), gpu(p.I), m, o_gpu, tol_switch=1e-4, max_lbfgs=0, max_newton=30)
    ref = oracle.solve(p.R, p.I, m, o_or)
    th = res.theta.cpu().double().numpy()
    eK = np.linalg.norm(th[:m * m] - ref[:m * m]) / np.linalg.norm(ref[:m * m])
    eP = abs(res.P - ref[:m * m].sum()) / abs(ref[:m * m].sum())
    eB = abs(res.B0 - ref[-1]) / max(abs(ref[-1]), 1.0)
    assert res.n_lbfgs == 0 and res.n_newton >= 1 and res.stop == "newton", res
    assert res.first_order_stop in ("rel_change", "cap"), res.first_order_stop
    assert eK <= 1e-4 and eP <= 1e-4 and eB <= 1e-4, (eK, eP, eB)
    # the Adam phase ended on the switch rule, not on its cap
    assert res.n_adam < 5000


def test_step_lds_and_l2_paths_agree_bitwise(dia, monkeypatch):
    # the step kernels run the L-BFGS two-loop recursion on an LDS copy of the history when it fits
    # (the default) or on the history in global memory (DIA_STEP_LDS=0, and any history too large for
    # LDS): the same arithmetic in the same order, so whole fits agree to the bit, single and batched
    p = sf.config1()
    o = dia.Objective(rho="cauchy", var="ccd_data", sigma0=p.sigma0_adu, gain=p.gain, c=2.3849)
    b = sf.batched(40, 4, 9, 256, 600, (120, 200))
    Rb = gpu(b.R)
    eps = [dia.Epoch(I=gpu(e.I), ref_row0=e.row0, ref_col0=e.col0) for e in b.epochs]
    runs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("DIA_STEP_LDS", flag)
        r = dia.fit(gpu(p.R), gpu(p.I), p.m, o, max_newton=0)
        th, res, st = dia.fit_batched(Rb, eps, b.m, o, max_newton=0)
        runs.append((r.theta.cpu().numpy().tobytes(), th.cpu().numpy().tobytes(), r.n_eval, r.n_lbfgs,
                     [x.n_lbfgs for x in res]))
    assert runs[0][3] > 0 and min(runs[0][4]) > 0, "the fits should reach the L-BFGS phase"
    assert runs[0] == runs[1]
