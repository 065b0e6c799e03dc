"""Binding of the LPV state-space surrogate kernels (``lpv_*`` in slosh.h).

Argument marshalling only: simulation, loss and gradient, Adam, L-BFGS and
the closed-loop simulation all run in ``libslosh.so``.  Parameters are FP64
device tensors [R, 141] in the packed order of the C ABI (A0, B0, C0, A1, B1,
C1, W1, b1, W2, b2, W3, b3, x0, row-major); data are scaled FP64 device
tensors [n, 3].
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import torch

from ._lib import LpvOpts, check, load

N_THETA = 137
N_PARAM = 141


@dataclasses.dataclass
class Options:
    sigma2: float = 1e-4
    sigmax: float = 1e-6
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    c1: float = 1e-4
    gtol: float = 1e-10
    ftol: float = 1e-13
    max_backtracks: int = 40
    lti_only: bool = False

    def c(self) -> LpvOpts:
        return LpvOpts(self.sigma2, self.sigmax, self.lr, self.beta1, self.beta2, self.eps, self.c1, self.gtol,
                       self.ftol, int(self.max_backtracks), 1 if self.lti_only else 0)


def _p(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _f64(t, device) -> torch.Tensor:
    return torch.as_tensor(t, dtype=torch.float64).to(device).contiguous()


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace(n_models: int, n_samples: int, device) -> torch.Tensor:
    L = load()
    b = C.c_size_t()
    check(L.lpv_workspace_bytes(int(n_models), int(n_samples), C.byref(b)), "lpv_workspace_bytes")
    return torch.empty(max(1, b.value), dtype=torch.uint8, device=device)


def simulate(params: torch.Tensor, u: torch.Tensor, with_p: bool = False):
    """yhat [R, n, 3] (and p [R, n]) from u [n, 3] or [R, n, 3]."""
    L = load()
    dev = params.device
    params = _f64(params, dev).reshape(-1, N_PARAM)
    u = _f64(u, dev)
    R = params.shape[0]
    per = 1 if u.dim() == 3 else 0
    n = u.shape[-2]
    y = torch.empty(R, n, 3, dtype=torch.float64, device=dev)
    p = torch.empty(R, n, dtype=torch.float64, device=dev) if with_p else None
    check(L.lpv_simulate(_p(params), R, _p(u), per, n, _p(y), _p(p), _stream(dev)), "lpv_simulate")
    return (y, p) if with_p else y


def loss_grad(params: torch.Tensor, u: torch.Tensor, y: torch.Tensor, opts: Options = Options(),
              grad: bool = True, ws: Optional[torch.Tensor] = None):
    """(loss [R], grad [R, 141] or None)."""
    L = load()
    dev = params.device
    params = _f64(params, dev).reshape(-1, N_PARAM)
    u, y = _f64(u, dev), _f64(y, dev)
    R, n = params.shape[0], u.shape[0]
    loss = torch.empty(R, dtype=torch.float64, device=dev)
    g = torch.empty(R, N_PARAM, dtype=torch.float64, device=dev) if grad else None
    if ws is None:
        ws = workspace(R, n, dev)
    o = opts.c()
    check(L.lpv_loss_grad(_p(params), R, _p(u), _p(y), n, C.byref(o), _p(loss), _p(g), _p(ws), ws.numel(),
                          _stream(dev)), "lpv_loss_grad")
    return loss, g


def loss_grad_noalloc(params: torch.Tensor, u: torch.Tensor, y: torch.Tensor, opts: Options = Options(),
                      grad: bool = True):
    """loss_grad through lpv_loss_grad_noalloc: no workspace; the library's
    fixed per-GPU array holds the reverse sweep's record.  Only the outputs
    are allocated here (by torch, before the call)."""
    L = load()
    dev = params.device
    params = _f64(params, dev).reshape(-1, N_PARAM)
    u, y = _f64(u, dev), _f64(y, dev)
    R, n = params.shape[0], u.shape[0]
    loss = torch.empty(R, dtype=torch.float64, device=dev)
    g = torch.empty(R, N_PARAM, dtype=torch.float64, device=dev) if grad else None
    o = opts.c()
    check(L.lpv_loss_grad_noalloc(_p(params), R, _p(u), _p(y), n, C.byref(o), _p(loss), _p(g), _stream(dev)),
          "lpv_loss_grad_noalloc")
    return loss, g


def adam(params: torch.Tensor, u: torch.Tensor, y: torch.Tensor, iters: int, opts: Options = Options(),
         ws: Optional[torch.Tensor] = None):
    """Runs `iters` Adam steps in place on params [R, 141]; returns the loss [R]
    at the last evaluated point."""
    L = load()
    dev = params.device
    assert params.dtype == torch.float64 and params.is_contiguous()
    u, y = _f64(u, dev), _f64(y, dev)
    R, n = params.shape[0], u.shape[0]
    loss = torch.empty(R, dtype=torch.float64, device=dev)
    if ws is None:
        ws = workspace(R, n, dev)
    o = opts.c()
    check(L.lpv_adam(_p(params), R, _p(u), _p(y), n, C.byref(o), int(iters), _p(loss), _p(ws), ws.numel(),
                     _stream(dev)), "lpv_adam")
    return loss


def lbfgs(params: torch.Tensor, u: torch.Tensor, y: torch.Tensor, max_iter: int, opts: Options = Options(),
          ws: Optional[torch.Tensor] = None):
    """L-BFGS in place on params [R, 141]; returns (loss [R], status [R], iters [R])."""
    L = load()
    dev = params.device
    assert params.dtype == torch.float64 and params.is_contiguous()
    u, y = _f64(u, dev), _f64(y, dev)
    R, n = params.shape[0], u.shape[0]
    loss = torch.empty(R, dtype=torch.float64, device=dev)
    status = torch.empty(R, dtype=torch.int32, device=dev)
    iters = torch.empty(R, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(R, n, dev)
    o = opts.c()
    check(L.lpv_lbfgs(_p(params), R, _p(u), _p(y), n, C.byref(o), int(max_iter), _p(loss), _p(status), _p(iters),
                      _p(ws), ws.numel(), _stream(dev)), "lpv_lbfgs")
    return loss, status, iters


def closed_loop(params: torch.Tensor, force: torch.Tensor, ref: torch.Tensor, ts: float, kp: float, kd: float,
                u_scale, y_scale, x0: Optional[torch.Tensor] = None, with_tau: bool = False):
    """Augmented model under the sampled attitude law: y [R, n, 6] (r_x, r_y,
    theta, rdot_x, rdot_y, thetadot) and optionally tau [R, n].  force [n, 2]
    or [R, n, 2] world forces, ref [n] or [R, n] (physical units)."""
    L = load()
    dev = params.device
    params = _f64(params, dev).reshape(-1, N_PARAM)
    force, ref = _f64(force, dev), _f64(ref, dev)
    R = params.shape[0]
    n = force.shape[-2]
    y = torch.empty(R, n, 6, dtype=torch.float64, device=dev)
    tau = torch.empty(R, n, dtype=torch.float64, device=dev) if with_tau else None
    x0d = None if x0 is None else _f64(x0, dev).reshape(R, 4)
    sc = (C.c_double * 6)(*[float(v) for v in list(u_scale) + list(y_scale)])
    check(L.lpv_closed_loop(_p(params), R, _p(x0d), _p(force), 1 if force.dim() == 3 else 0, _p(ref),
                            1 if ref.dim() == 2 else 0, n, float(ts), float(kp), float(kd), sc, _p(y), _p(tau),
                            _stream(dev)), "lpv_closed_loop")
    return (y, tau) if with_tau else y
