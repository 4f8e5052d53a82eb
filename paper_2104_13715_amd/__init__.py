"""MI355X DIA kernel fit: Python binding of libdia.so (argument marshalling only).

Every numerical step runs in the library's HIP kernels; torch supplies device
memory and the current stream.  The names follow the C ABI in include/dia.h:

* ``model(R, theta, m)``                       eq. model_image_delta_basis on the valid region
* ``loss_grad(R, I, theta, m, objective)``     fused forward + objective + backward
* ``loss_grad64(R, I, theta, m, objective)``   the same at FP64 parameters, FP64 gradient
* ``loss_grad_noalloc(R, I, theta, m, objective)``  loss_grad on the library's static scratch
* ``fit(R, I, m, objective, **opts)``           Adam then L-BFGS on the device
* ``DIALoss.apply(theta, R, I, m, objective)``  autograd wrapper around ``loss_grad``
* ``hessian(R, I, theta, m, objective)``         observed Fisher information (Section 2.5)
* ``covariance(F, m)``                          its inverse, standard errors, validity flag

If libdia.so has not been built this module raises ImportError: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# DIA_LIBRARY names another build of the same library (the host-sanitizer build of the CPU checks)
LIB_PATH = os.environ.get("DIA_LIBRARY") or os.path.join(_HERE, "libdia.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libdia.so not found at {LIB_PATH}; build it with `python -m paper_2104_13715_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

# ----------------------------------------------------------------------------- constants (dia.h)
MAX_M = 49
MAX_BG_DEGREE = 4
OK, W_NOT_CONVERGED = 0, 1
E_ARG, E_SIZE, E_WORKSPACE, E_HIP, E_NONFINITE, E_SCRATCH = -1, -2, -3, -4, -5, -6
NOALLOC_SCRATCH_BYTES = 16 << 20
RHO = {"gauss": 0, "huber": 1, "cauchy": 2}
VAR = {"weights": 0, "ccd_data": 1, "ccd_model": 2, "emccd_data": 3, "emccd_model": 4}
OP_MODEL, OP_LOSS_GRAD, OP_FIT, OP_FIT_CLIPPED, OP_HESSIAN, OP_COVARIANCE = 0, 1, 2, 3, 4, 5
INIT = {"flat": 0, "gauss": 1, "user": 2}
STOP = {0: "none", 1: "rel_change", 2: "gradient", 3: "line_search", 4: "cap", 5: "newton"}


class _Image(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("ld", ctypes.c_int64)]


class _Objective(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_int32), ("var", ctypes.c_int32), ("sigma0", ctypes.c_double),
                ("gain", ctypes.c_double), ("excess", ctypes.c_double), ("var_floor", ctypes.c_double),
                ("c", ctypes.c_double), ("weights", ctypes.c_void_p), ("flat", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("lam", ctypes.c_double), ("bg_degree", ctypes.c_int32)]


class _Epoch(ctypes.Structure):
    _fields_ = [("I", ctypes.c_void_p), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("ld", ctypes.c_int64),
                ("ref_row0", ctypes.c_int32), ("ref_col0", ctypes.c_int32), ("weights", ctypes.c_void_p),
                ("flat", ctypes.c_void_p), ("mask", ctypes.c_void_p)]


class _FitOpts(ctypes.Structure):
    _fields_ = [("init", ctypes.c_int32), ("init_phi", ctypes.c_double), ("lr_K", ctypes.c_double),
                ("lr_B0", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("tol_switch", ctypes.c_double), ("tol_change", ctypes.c_double),
                ("tol_grad", ctypes.c_double), ("history", ctypes.c_int32), ("max_adam", ctypes.c_int32),
                ("max_lbfgs", ctypes.c_int32), ("max_eval", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("clip_kappa", ctypes.c_double), ("poll_every", ctypes.c_int32), ("max_newton", ctypes.c_int32)]


class _FitResult(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_double), ("P", ctypes.c_double), ("B0", ctypes.c_double),
                ("n_eval", ctypes.c_int32), ("n_adam", ctypes.c_int32), ("n_lbfgs", ctypes.c_int32),
                ("n_outer", ctypes.c_int32), ("n_masked", ctypes.c_int64), ("stop", ctypes.c_int32),
                ("status", ctypes.c_int32), ("n_newton", ctypes.c_int32), ("n_hessian", ctypes.c_int32),
                ("first_order_stop", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_lib.dia_version.restype = ctypes.c_int
_lib.dia_status_string.argtypes = [ctypes.c_int]
_lib.dia_status_string.restype = ctypes.c_char_p
_lib.dia_workspace_size.argtypes = [_i32, _i32, _i32, _i64, _i32, ctypes.POINTER(_sz)]
_lib.dia_model.argtypes = [_Image, _vp, _i32, _vp, _i64, _vp]
_lib.dia_model_bg.argtypes = [_Image, _vp, _i32, _i32, _vp, _i64, _vp]
_lib.dia_loss_grad.argtypes = [_Image, _Image, ctypes.POINTER(_Objective), _vp, _i32, _vp, _vp, _vp, _sz, _vp]
_lib.dia_loss_grad64.argtypes = [_Image, _Image, ctypes.POINTER(_Objective), _vp, _i32, _vp, _vp, _vp, _sz, _vp]
_lib.dia_loss_grad_noalloc.argtypes = [_Image, _Image, ctypes.POINTER(_Objective), _vp, _i32, _vp, _vp, _vp]
_lib.dia_tile_shape.argtypes = [_i32, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
_lib.dia_hessian.argtypes = [_Image, _Image, ctypes.POINTER(_Objective), _vp, _i32, _vp, _vp, _sz, _vp]
_lib.dia_covariance.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.dia_covariance_bg.argtypes = [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.dia_fit_opts_default.argtypes = [ctypes.POINTER(_FitOpts)]
_lib.dia_fit_opts_default.restype = None
_lib.dia_fit.argtypes = [_Image, _Image, ctypes.POINTER(_Objective), _i32, ctypes.POINTER(_FitOpts), _vp,
                         ctypes.POINTER(_FitResult), _vp, _sz, _vp]
_lib.dia_batched_workspace_size.argtypes = [_Image, ctypes.POINTER(_Epoch), _i32, _i32, _i32, _i32,
                                            ctypes.POINTER(_sz)]
_lib.dia_loss_grad_batched.argtypes = [_Image, ctypes.POINTER(_Epoch), _i32, _i32, ctypes.POINTER(_Objective), _i32,
                                       _vp, _vp, _vp, _vp, _sz, _vp]
_lib.dia_fit_batched.argtypes = [_Image, ctypes.POINTER(_Epoch), _i32, _i32, ctypes.POINTER(_Objective),
                                 ctypes.POINTER(_FitOpts), _i32, _vp, ctypes.POINTER(_FitResult), _vp, _sz, _vp]
for _f in ("dia_workspace_size", "dia_model", "dia_model_bg", "dia_loss_grad", "dia_loss_grad64",
           "dia_loss_grad_noalloc", "dia_hessian", "dia_covariance_bg", "dia_tile_shape", "dia_covariance", "dia_fit",
           "dia_batched_workspace_size", "dia_loss_grad_batched", "dia_fit_batched"):
    getattr(_lib, _f).restype = ctypes.c_int

# "fp32" (the C enum's name) and "plain" name the same form: FP32 data, FP64 arithmetic on the vector ALUs
PREC = {"fp32": 0, "plain": 0, "bf16x3": 1}

EXPORTS = ("dia_version", "dia_status_string", "dia_workspace_size", "dia_model", "dia_model_bg", "dia_loss_grad",
           "dia_loss_grad64", "dia_loss_grad_noalloc", "dia_hessian", "dia_covariance_bg", "dia_tile_shape",
           "dia_covariance", "dia_fit_opts_default", "dia_fit", "dia_batched_workspace_size",
           "dia_loss_grad_batched", "dia_fit_batched")


class DIAError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


def version() -> int:
    return _lib.dia_version()


def status_string(status: int) -> str:
    return _lib.dia_status_string(int(status)).decode()


def _check(status: int, where: str) -> int:
    if status < 0:
        raise DIAError(status, where)
    return status


# ----------------------------------------------------------------------------- marshalling helpers
def _image(t: torch.Tensor, name: str) -> _Image:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.dim() != 2 or not t.is_cuda:
        raise TypeError(f"{name} must be a 2-D float32 CUDA tensor")
    if t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return _Image(t.data_ptr(), t.shape[0], t.shape[1], t.stride(0))


def _like_target(t: Optional[torch.Tensor], I: torch.Tensor, dtype, name: str):
    if t is None:
        return None
    if t.dtype != dtype or t.shape != I.shape or t.stride() != I.stride() or t.device != I.device:
        raise ValueError(f"{name} must be a {dtype} tensor laid out like the target (same shape and strides)")
    return t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


@dataclass
class Objective:
    """rho in {'gauss', 'huber', 'cauchy'}; var in {'weights', 'ccd_data', 'ccd_model', 'emccd_data',
    'emccd_model'} (see include/dia.h).  weights / flat / mask are tensors laid out like the target.
    lam: lambda of the kernel-smoothness penalty (single-pair calls only; 0 = none).
    bg_degree: degree d of the polynomial background of Section 2.6 (0 = the scalar B0); theta then has
    m*m + (d+1)(d+2)/2 entries (single-pair calls only)."""
    rho: str = "gauss"
    var: str = "ccd_data"
    sigma0: float = 0.0
    gain: float = 1.0
    excess: float = 2.0
    var_floor: float = 1.0
    c: float = 1.345
    weights: Optional[torch.Tensor] = None
    flat: Optional[torch.Tensor] = None
    mask: Optional[torch.Tensor] = None
    lam: float = 0.0
    bg_degree: int = 0

    def n_params(self, m: int) -> int:
        d = int(self.bg_degree)
        return m * m + (d + 1) * (d + 2) // 2

    def _c(self, I: torch.Tensor) -> _Objective:
        return _Objective(RHO[self.rho], VAR[self.var], float(self.sigma0), float(self.gain), float(self.excess),
                          float(self.var_floor), float(self.c),
                          _like_target(self.weights, I, torch.float32, "weights"),
                          _like_target(self.flat, I, torch.float32, "flat"),
                          _like_target(self.mask, I, torch.uint8, "mask"), float(self.lam), int(self.bg_degree))


def workspace_size(op: int, rows: int, cols: int, ld: int, m: int) -> int:
    n = _sz(0)
    _check(_lib.dia_workspace_size(op, rows, cols, ld, m, ctypes.byref(n)), "dia_workspace_size")
    return int(n.value)


class Workspace:
    """A 256-byte aligned device buffer (torch-owned) reused across calls of one size or less."""

    def __init__(self, device):
        self.device = torch.device(device)
        self.buf = None
        self.nbytes = 0

    def get(self, nbytes: int):
        if nbytes == 0:
            return None, 0
        if self.buf is None or self.nbytes < nbytes:
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.nbytes = nbytes
        p = self.buf.data_ptr()
        return p + (-p) % 256, nbytes


def _theta(theta: torch.Tensor, m: int, device, n: Optional[int] = None) -> torch.Tensor:
    n = m * m + 1 if n is None else n
    if theta.dtype != torch.float32 or theta.numel() != n or not theta.is_contiguous():
        raise ValueError(f"theta must be a contiguous float32 tensor of {n} values (the kernel, then the background)")
    if theta.device != device:
        raise ValueError("theta must live on the images' device")
    return theta


# ----------------------------------------------------------------------------- entry points
def model(R: torch.Tensor, theta: torch.Tensor, m: int, out: Optional[torch.Tensor] = None,
          bg_degree: int = 0) -> torch.Tensor:
    """Valid model image (rows-m+1, cols-m+1), eq. model_image_delta_basis (with the polynomial background
    of eq. polybackground when bg_degree > 0)."""
    Ri = _image(R, "R")
    theta = _theta(theta, m, R.device, Objective(bg_degree=bg_degree).n_params(m))
    if out is None:
        out = torch.empty((max(R.shape[0] - m + 1, 1), max(R.shape[1] - m + 1, 1)), dtype=torch.float32,
                          device=R.device)
    _check(_lib.dia_model_bg(Ri, theta.data_ptr(), m, int(bg_degree), out.data_ptr(), out.stride(0),
                             _stream(R.device)), "dia_model_bg")
    return out


def loss_grad(R: torch.Tensor, I: torch.Tensor, theta: torch.Tensor, m: int, objective: Objective,
              workspace: Optional[Workspace] = None, loss: Optional[torch.Tensor] = None,
              grad: Optional[torch.Tensor] = None):
    """(loss float64[1], grad float32[n]) of the objective at theta, one fused pass (n = objective.n_params(m))."""
    Ri, Ii = _image(R, "R"), _image(I, "I")
    n = objective.n_params(m)
    theta = _theta(theta, m, R.device, n)
    obj = objective._c(I)
    ws = workspace or Workspace(R.device)
    nbytes = workspace_size(OP_LOSS_GRAD, I.shape[0], I.shape[1], I.stride(0), m)
    p, nb = ws.get(nbytes)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=R.device)
    if grad is None:
        grad = torch.empty(n, dtype=torch.float32, device=R.device)
    _check(_lib.dia_loss_grad(Ri, Ii, ctypes.byref(obj), theta.data_ptr(), m, loss.data_ptr(), grad.data_ptr(),
                              p, nb, _stream(R.device)), "dia_loss_grad")
    return loss, grad


def loss_grad64(R: torch.Tensor, I: torch.Tensor, theta: torch.Tensor, m: int, objective: Objective,
                workspace: Optional[Workspace] = None, loss: Optional[torch.Tensor] = None,
                grad: Optional[torch.Tensor] = None):
    """(loss float64[1], grad float64[n]) at FP64 parameters theta, one fused pass (dia_loss_grad64)."""
    Ri, Ii = _image(R, "R"), _image(I, "I")
    n = objective.n_params(m)
    if theta.dtype != torch.float64 or theta.numel() != n or not theta.is_contiguous():
        raise ValueError(f"theta must be a contiguous float64 tensor of {n} values")
    if theta.device != R.device:
        raise ValueError("theta must live on the images' device")
    obj = objective._c(I)
    ws = workspace or Workspace(R.device)
    p, nb = ws.get(workspace_size(OP_LOSS_GRAD, I.shape[0], I.shape[1], I.stride(0), m))
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=R.device)
    if grad is None:
        grad = torch.empty(n, dtype=torch.float64, device=R.device)
    _check(_lib.dia_loss_grad64(Ri, Ii, ctypes.byref(obj), theta.data_ptr(), m, loss.data_ptr(), grad.data_ptr(),
                                p, nb, _stream(R.device)), "dia_loss_grad64")
    return loss, grad


def tile_shape(m: int, rows: int, cols: int):
    """(variant, tile rows, tile cols) that single-pair calls use for this kernel and image size (the
    autotuner's choice once made, else the default)."""
    v, ty, tx = _i32(0), _i32(0), _i32(0)
    _check(_lib.dia_tile_shape(m, rows, cols, ctypes.byref(v), ctypes.byref(ty), ctypes.byref(tx)), "dia_tile_shape")
    return v.value, ty.value, tx.value


def loss_grad_noalloc(R: torch.Tensor, I: torch.Tensor, theta: torch.Tensor, m: int, objective: Objective,
                      loss: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None):
    """loss_grad without a workspace (dia_loss_grad_noalloc): the library's static device scratch holds
    the partial sums.  Pass preallocated loss (float64[1]) and grad (float32[m*m+1]) to allocate
    nothing at all."""
    Ri, Ii = _image(R, "R"), _image(I, "I")
    n = objective.n_params(m)
    theta = _theta(theta, m, R.device, n)
    obj = objective._c(I)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=R.device)
    if grad is None:
        grad = torch.empty(n, dtype=torch.float32, device=R.device)
    _check(_lib.dia_loss_grad_noalloc(Ri, Ii, ctypes.byref(obj), theta.data_ptr(), m, loss.data_ptr(),
                                      grad.data_ptr(), _stream(R.device)), "dia_loss_grad_noalloc")
    return loss, grad


def hessian(R: torch.Tensor, I: torch.Tensor, theta: torch.Tensor, m: int, objective: Objective,
            workspace: Optional[Workspace] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Observed Fisher information: the exact FP64 Hessian d2L/dtheta2, n x n (n = objective.n_params(m))."""
    Ri, Ii = _image(R, "R"), _image(I, "I")
    n = objective.n_params(m)
    theta = _theta(theta, m, R.device, n)
    obj = objective._c(I)
    if out is None:
        out = torch.empty((n, n), dtype=torch.float64, device=R.device)
    if out.dtype != torch.float64 or tuple(out.shape) != (n, n) or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of shape (n, n)")
    ws = workspace or Workspace(R.device)
    p, nb = ws.get(workspace_size(OP_HESSIAN, I.shape[0], I.shape[1], I.stride(0), m))
    _check(_lib.dia_hessian(Ri, Ii, ctypes.byref(obj), theta.data_ptr(), m, out.data_ptr(), p, nb,
                            _stream(R.device)), "dia_hessian")
    return out


@dataclass
class Covariance:
    """Section 2.5 at a fit: cov = F^-1, sigma = sqrt(diag cov), sigma_P = the error of P = sum K;
    valid is the positive-definiteness test of cov (logdet = ln det cov, min_pivot = the smallest
    Cholesky pivot of F); the tensors are NaN when valid is False."""
    cov: torch.Tensor
    sigma: torch.Tensor
    sigma_P: float
    valid: bool
    logdet: float
    min_pivot: float


def covariance(F: torch.Tensor, m: int, workspace: Optional[Workspace] = None, bg_degree: int = 0) -> Covariance:
    """Covariance estimate and validity test from an observed Fisher information F (float64, n x n,
    n = m*m + (d+1)(d+2)/2 for a background of degree d)."""
    n = Objective(bg_degree=bg_degree).n_params(m)
    if F.dtype != torch.float64 or tuple(F.shape) != (n, n) or not F.is_contiguous() or F.device.type != "cuda":
        raise ValueError(f"F must be a contiguous float64 device tensor of shape ({n}, {n})")
    cov = torch.empty((n, n), dtype=torch.float64, device=F.device)
    sigma = torch.empty(n, dtype=torch.float64, device=F.device)
    sP = torch.empty(1, dtype=torch.float64, device=F.device)
    info = torch.empty(3, dtype=torch.float64, device=F.device)
    ws = workspace or Workspace(F.device)
    p, nb = ws.get(workspace_size(OP_COVARIANCE, 1, 1, 1, m))
    _check(_lib.dia_covariance_bg(F.data_ptr(), m, int(bg_degree), cov.data_ptr(), sigma.data_ptr(), sP.data_ptr(),
                                  info.data_ptr(), p, nb, _stream(F.device)), "dia_covariance_bg")
    h = info.cpu().tolist()
    return Covariance(cov=cov, sigma=sigma, sigma_P=float(sP.item()), valid=h[0] == 1.0, logdet=h[1],
                      min_pivot=h[2])


def uncertainty(R: torch.Tensor, I: torch.Tensor, theta: torch.Tensor, m: int, objective: Objective,
                workspace: Optional[Workspace] = None) -> Covariance:
    """Section 2.5 at theta: the covariance of the observed Fisher information (the exact Hessian)."""
    return covariance(hessian(R, I, theta, m, objective, workspace), m, workspace, objective.bg_degree)


@dataclass
class FitResult:
    theta: torch.Tensor
    loss: float
    P: float
    B0: float
    n_eval: int
    n_adam: int
    n_lbfgs: int
    n_outer: int
    n_masked: int
    stop: str
    status: int
    n_newton: int = 0
    n_hessian: int = 0
    first_order_stop: str = "none"
    extra: dict = field(default_factory=dict)

    m: int = 0

    @property
    def K(self) -> torch.Tensor:
        return self.theta[:self.m * self.m].view(self.m, self.m)


def fit_options(**kw) -> _FitOpts:
    o = _FitOpts()
    _lib.dia_fit_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "init":
            v = INIT[v] if isinstance(v, str) else int(v)
        if not hasattr(o, k):
            raise TypeError(f"unknown fit option {k}")
        setattr(o, k, v)
    return o


def fit(R: torch.Tensor, I: torch.Tensor, m: int, objective: Objective, theta: Optional[torch.Tensor] = None,
        workspace: Optional[Workspace] = None, **opts) -> FitResult:
    """Fit K and the background (Adam then L-BFGS on the device, then the Newton polish); returns after the
    fit has finished."""
    Ri, Ii = _image(R, "R"), _image(I, "I")
    n = objective.n_params(m)
    if theta is not None:
        opts.setdefault("init", "user")
        theta = _theta(theta, m, R.device, n)
    else:
        theta = torch.empty(n, dtype=torch.float32, device=R.device)
    o = fit_options(**opts)
    obj = objective._c(I)
    ws = workspace or Workspace(R.device)
    op = OP_FIT_CLIPPED if o.max_outer > 1 else OP_FIT
    p, nb = ws.get(workspace_size(op, I.shape[0], I.shape[1], I.stride(0), m))
    res = _FitResult()
    st = _lib.dia_fit(Ri, Ii, ctypes.byref(obj), m, ctypes.byref(o), theta.data_ptr(), ctypes.byref(res), p, nb,
                      _stream(R.device))
    _check(st, "dia_fit")
    return FitResult(theta=theta, loss=res.loss, P=res.P, B0=res.B0, n_eval=res.n_eval, n_adam=res.n_adam,
                     n_lbfgs=res.n_lbfgs, n_outer=res.n_outer, n_masked=int(res.n_masked),
                     stop=STOP.get(res.stop, str(res.stop)), status=st, n_newton=res.n_newton,
                     n_hessian=res.n_hessian, first_order_stop=STOP.get(res.first_order_stop, str(res.first_order_stop)),
                     m=m)


class DIALoss(torch.autograd.Function):
    """L(theta) as a 0-d float64 tensor whose backward is the fused hand-written gradient.

    forward runs one fused pass and keeps the gradient; backward scales it by the incoming
    gradient, so no second pass over the images is needed.  A float64 theta goes through
    ``dia_loss_grad64`` unrounded (FP64 gradient); any other dtype through ``dia_loss_grad``
    at FP32."""

    @staticmethod
    def forward(ctx, theta, R, I, m, objective, workspace=None):
        if theta.dtype == torch.float64:
            loss, grad = loss_grad64(R, I, theta.detach().contiguous(), m, objective, workspace)
        else:
            loss, grad = loss_grad(R, I, theta.detach().to(torch.float32).contiguous(), m, objective, workspace)
        ctx.save_for_backward(grad)
        ctx.theta_dtype = theta.dtype
        return loss.reshape(())

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        g = (grad.to(torch.float64) * gout.to(torch.float64)).to(ctx.theta_dtype)
        return g, None, None, None, None, None


# ----------------------------------------------------------------------------- batched epochs
@dataclass
class Epoch:
    """A target and the reference pixel under its pixel (0, 0); optional arrays laid out like I."""
    I: torch.Tensor
    ref_row0: int = 0
    ref_col0: int = 0
    weights: Optional[torch.Tensor] = None
    flat: Optional[torch.Tensor] = None
    mask: Optional[torch.Tensor] = None

    def _c(self) -> _Epoch:
        im = _image(self.I, "epoch I")
        return _Epoch(im.data, im.rows, im.cols, im.ld, int(self.ref_row0), int(self.ref_col0),
                      _like_target(self.weights, self.I, torch.float32, "weights"),
                      _like_target(self.flat, self.I, torch.float32, "flat"),
                      _like_target(self.mask, self.I, torch.uint8, "mask"))


def _epochs(epochs):
    arr = (_Epoch * len(epochs))()
    for k, e in enumerate(epochs):
        arr[k] = e._c()
    return arr


def batched_workspace_size(R: torch.Tensor, epochs, m: int, precision: str = "fp32", fit: bool = False) -> int:
    n = _sz(0)
    _check(_lib.dia_batched_workspace_size(_image(R, "R"), _epochs(epochs), len(epochs), m, PREC[precision],
                                           int(fit), ctypes.byref(n)), "dia_batched_workspace_size")
    return int(n.value)


def loss_grad_batched(R: torch.Tensor, epochs, theta: torch.Tensor, m: int, objective: Objective,
                      precision: str = "fp32", workspace: Optional[Workspace] = None):
    """Per-epoch (loss float64[n], grad float32[n, m*m+1]) at theta[n, m*m+1]."""
    n = len(epochs)
    Ri = _image(R, "R")
    if theta.dtype != torch.float32 or theta.shape != (n, m * m + 1) or not theta.is_contiguous():
        raise ValueError("theta must be a contiguous float32 tensor of shape (n_epochs, m*m + 1)")
    ep = _epochs(epochs)
    obj = objective._c(R)
    ws = workspace or Workspace(R.device)
    p, nb = ws.get(batched_workspace_size(R, epochs, m, precision, False))
    loss = torch.empty(n, dtype=torch.float64, device=R.device)
    grad = torch.empty((n, m * m + 1), dtype=torch.float32, device=R.device)
    _check(_lib.dia_loss_grad_batched(Ri, ep, n, m, ctypes.byref(obj), PREC[precision], theta.data_ptr(),
                                      loss.data_ptr(), grad.data_ptr(), p, nb, _stream(R.device)),
           "dia_loss_grad_batched")
    return loss, grad


def fit_batched(R: torch.Tensor, epochs, m: int, objective: Objective, theta: Optional[torch.Tensor] = None,
                precision: str = "fp32", workspace: Optional[Workspace] = None, **opts):
    """Fit every epoch; returns (theta float32[n, m*m+1], list of per-epoch FitResult, overall status)."""
    n = len(epochs)
    Ri = _image(R, "R")
    if theta is not None:
        opts.setdefault("init", "user")
        if theta.dtype != torch.float32 or theta.shape != (n, m * m + 1) or not theta.is_contiguous():
            raise ValueError("theta must be a contiguous float32 tensor of shape (n_epochs, m*m + 1)")
    else:
        theta = torch.empty((n, m * m + 1), dtype=torch.float32, device=R.device)
    o = fit_options(**opts)
    ep = _epochs(epochs)
    obj = objective._c(R)
    ws = workspace or Workspace(R.device)
    p, nb = ws.get(batched_workspace_size(R, epochs, m, precision, True))
    res = (_FitResult * n)()
    st = _lib.dia_fit_batched(Ri, ep, n, m, ctypes.byref(obj), ctypes.byref(o), PREC[precision], theta.data_ptr(),
                              res, p, nb, _stream(R.device))
    _check(st, "dia_fit_batched")
    out = [FitResult(theta=theta[k], loss=r.loss, P=r.P, B0=r.B0, n_eval=r.n_eval, n_adam=r.n_adam,
                     n_lbfgs=r.n_lbfgs, n_outer=r.n_outer, n_masked=int(r.n_masked),
                     stop=STOP.get(r.stop, str(r.stop)), status=r.status, n_newton=r.n_newton,
                     n_hessian=r.n_hessian, first_order_stop=STOP.get(r.first_order_stop, str(r.first_order_stop)),
                     m=m)
           for k, r in enumerate(res)]
    return theta, out, st
