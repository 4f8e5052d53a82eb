"""dia_loss_grad_noalloc (the entry point that allocates nothing: its workspace is the library's static
device scratch) against dia_loss_grad on the same inputs: two calls in a row, the second on a smaller
image and kernel, each to the parity bar of the fused pass (loss to 1e-12 relative, gradient element
by element within 1e-5 relative plus 1e-9 of each component's summation scale), and the size check
that rejects a call whose workspace would exceed the scratch."""
import numpy as np
import pytest
import torch

import oracle
from parity import check_grad_elementwise, summation_scale
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


def _compare(dia, R, I, theta, m, rho, var, sigma0, gain):
    c = 2.3849 if rho == "cauchy" else 1.345
    obj = dia.Objective(rho=rho, var=var, sigma0=sigma0, gain=gain, c=c)
    o_or = oracle.Objective(rho=rho, var=var, sigma0=sigma0, gain=gain, c=c)
    Rg, Ig, tg = gpu(R), gpu(I), gpu(theta)
    L_ws, g_ws = dia.loss_grad(Rg, Ig, tg, m, obj)
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    grad = torch.full((m * m + 1,), float("nan"), dtype=torch.float32, device=DEV)
    dia.loss_grad_noalloc(Rg, Ig, tg, m, obj, loss=loss, grad=grad)
    torch.cuda.synchronize()
    L0, L1 = L_ws.item(), loss.item()
    assert abs(L1 - L0) <= 1e-12 * abs(L0), (L0, L1)
    g0 = g_ws.cpu().double().numpy()
    g1 = grad.cpu().double().numpy()
    scale = summation_scale(R, I, theta.astype(np.float64), m, o_or)
    check_grad_elementwise(g1, g0, scale)
    # and against the oracle at the same point
    L_ref, g_ref = oracle.loss_grad(R, I, theta.astype(np.float64), m, o_or)
    assert abs(L1 - L_ref) <= 1e-9 * abs(L_ref)
    check_grad_elementwise(g1, g_ref, scale)


def test_noalloc_matches_loss_grad_two_calls_second_smaller(dia):
    big = sf.crop(sf.config3(size=512), 300)
    th_big = np.r_[big.K_true.ravel() * 1.02, big.B0_true + 1.5].astype(np.float32)
    _compare(dia, big.R, big.I, th_big, big.m, "cauchy", "ccd_model", big.sigma0_adu, big.gain)
    small = sf.config1()
    th_small = np.r_[small.K_true.ravel() * 0.97, small.B0_true - 0.5].astype(np.float32)
    _compare(dia, small.R, small.I, th_small, small.m, "gauss", "ccd_data", small.sigma0_adu, small.gain)


def test_noalloc_rejects_a_call_beyond_its_scratch(dia):
    # m = 49 on 2048^2 needs more partial rows than the static scratch holds: rejected before anything
    # is enqueued, outputs untouched
    m, n = 49, 2048
    need = dia.workspace_size(dia.OP_LOSS_GRAD, n, n, n, m)
    assert need > dia.NOALLOC_SCRATCH_BYTES
    R = torch.ones((n, n), dtype=torch.float32, device=DEV)
    theta = torch.zeros(m * m + 1, dtype=torch.float32, device=DEV)
    loss = torch.full((1,), -7.0, dtype=torch.float64, device=DEV)
    grad = torch.full((m * m + 1,), -7.0, dtype=torch.float32, device=DEV)
    obj = dia.Objective(rho="gauss", var="ccd_data", sigma0=5.0, gain=1.0)
    with pytest.raises(dia.DIAError) as e:
        dia.loss_grad_noalloc(R, R, theta, m, obj, loss=loss, grad=grad)
    assert e.value.status == dia.E_SCRATCH
    torch.cuda.synchronize()
    assert loss.item() == -7.0 and bool(torch.all(grad == -7.0))
