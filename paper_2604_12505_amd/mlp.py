"""Python binding of the surrogate-network part of libslosh.so (marshalling only)."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from ._lib import check, load

N_PARAMS = 231171
DIMS = (128, 256, 256, 256, 256, 3)


def pack(params) -> np.ndarray:
    """[(W [out, in], b [out]), ...] -> the packed FP32 vector of the C ABI."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unpack(vec) -> list:
    v = np.asarray(vec, np.float64)
    out, o = [], 0
    for i in range(len(DIMS) - 1):
        n_in, n_out = DIMS[i], DIMS[i + 1]
        W = v[o:o + n_in * n_out].reshape(n_out, n_in); o += n_in * n_out
        b = v[o:o + n_out]; o += n_out
        out.append((W, b))
    return out


class Mlp:
    """``mlp_init`` on construction; forward / train_step / params."""

    def __init__(self, params_vec, max_batch: int, device="cuda:0",
                 stream: Optional[torch.cuda.Stream] = None):
        self.L = load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        p = torch.as_tensor(np.asarray(params_vec, np.float32), device=self.device).contiguous()
        assert p.numel() == N_PARAMS
        nbytes = C.c_size_t()
        check(self.L.mlp_workspace_bytes(int(max_batch), C.byref(nbytes)), "mlp_workspace_bytes")
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + nbytes.value]
        self.max_batch = int(max_batch)
        h = C.c_void_p()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        check(self.L.mlp_init(C.c_void_p(p.data_ptr()), int(max_batch), C.c_void_p(self.ws.data_ptr()),
                              C.c_size_t(nbytes.value), C.c_void_p(self.stream.cuda_stream), C.byref(h)),
              "mlp_init")
        self.h = h
        self._keep = []

    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def forward(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        x = x.to(self.device, torch.float32).contiguous()
        B = x.shape[0]
        y = out if out is not None else torch.empty(B, 3, device=self.device)
        self._enter()
        check(self.L.mlp_forward(self.h, C.c_void_p(x.data_ptr()), int(B), C.c_void_p(y.data_ptr())),
              "mlp_forward")
        self._keep = [x]
        self._leave()
        return y

    def launch(self, x: torch.Tensor, out: torch.Tensor) -> None:
        """forward() without the hand-over between the caller's stream and the
        network's: enqueues the inference launch on the network's stream only.
        x (float32, contiguous, on the device) and out must already be ordered
        on that stream (for example by a previous forward() or a device
        synchronize); for back-to-back launches on resident data, each of
        which forward() would bracket with two cross-stream event waits."""
        B = x.shape[0]
        if x.dtype != torch.float32 or not x.is_contiguous() or tuple(out.shape) != (B, 3):
            raise ValueError("launch: x must be contiguous float32 and out of shape (B, 3)")
        check(self.L.mlp_forward(self.h, C.c_void_p(x.data_ptr()), int(B), C.c_void_p(out.data_ptr())),
              "mlp_forward")

    def train_step(self, x, target, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, want_grad=False):
        x = x.to(self.device, torch.float32).contiguous()
        t = target.to(self.device, torch.float32).contiguous()
        loss = torch.empty(1, device=self.device)
        grad = torch.empty(N_PARAMS, device=self.device) if want_grad else None
        self._enter()
        check(self.L.mlp_train_step(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                    int(x.shape[0]), float(lr), float(beta1), float(beta2), float(eps),
                                    None if grad is None else C.c_void_p(grad.data_ptr()),
                                    C.c_void_p(loss.data_ptr())), "mlp_train_step")
        self._keep = [x, t]
        self._leave()
        return loss, grad

    def backward(self, x, dy) -> torch.Tensor:
        """dL/dparams [231171] for the output gradient dy [B, 3] at inputs x."""
        x = x.to(self.device, torch.float32).contiguous()
        dy = dy.to(self.device, torch.float32).contiguous()
        grad = torch.empty(N_PARAMS, device=self.device)
        self._enter()
        check(self.L.mlp_backward(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(dy.data_ptr()), int(x.shape[0]),
                                  C.c_void_p(grad.data_ptr())), "mlp_backward")
        self._keep = [x, dy]
        self._leave()
        return grad

    def adam_step(self, grad, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step from grad [231171] with bias correction for step t."""
        g = grad.to(self.device, torch.float32).contiguous()
        self._enter()
        check(self.L.mlp_adam_step(self.h, C.c_void_p(g.data_ptr()), float(lr), float(beta1), float(beta2),
                                   float(eps), int(t)), "mlp_adam_step")
        self._keep = [g]
        self._leave()

    def coupled_rollout(self, norm, static, feat0, rigid0, u_seq, body, log_stride: int, z_max: float = 6.0,
                        window: int = 32):
        """mlp_coupled_rollout: the rigid body driven by this network's wrench
        instead of SPH.  static [R, n_static], feat0 [R, window, 3] (theta,
        thetadot, input torque of the first window's samples), rigid0 [R, 6]
        (r, theta, rdot, thetadot at sample window - 1), u_seq [R, n_steps, 3],
        body [R, 3] (mass, inertia, dt).  Returns dict(y [R, T, 6] and wrench
        [R, T, 3] (NaN where not computed), feat [R, T, 3], rigid [R, 6]
        float64 after the last step, flags [R] int32)."""
        dev = self.device
        u = torch.as_tensor(u_seq, device=dev, dtype=torch.float32).contiguous()
        R, n_steps, _ = u.shape
        T = -(-n_steps // int(log_stride))
        st = torch.as_tensor(static, device=dev, dtype=torch.float32).contiguous()
        feat = torch.zeros(R, T, 3, device=dev)
        feat[:, :window] = torch.as_tensor(feat0, device=dev, dtype=torch.float32)
        rigid = torch.as_tensor(rigid0, device=dev, dtype=torch.float64).contiguous().clone()
        bd = torch.as_tensor(body, device=dev, dtype=torch.float64).contiguous()
        y = torch.full((R, T, 6), float("nan"), device=dev)
        w = torch.full((R, T, 3), float("nan"), device=dev)
        flags = torch.empty(R, dtype=torch.int32, device=dev)
        nv = np.asarray(norm, np.float32)
        nm = (C.c_float * len(nv))(*[float(v) for v in nv])
        self._enter()
        check(self.L.mlp_coupled_rollout(self.h, int(R), int(n_steps), int(log_stride), int(window),
                                         C.c_void_p(bd.data_ptr()), C.c_void_p(u.data_ptr()),
                                         C.c_void_p(st.data_ptr()), int(st.shape[1]), nm, float(z_max),
                                         C.c_void_p(rigid.data_ptr()), C.c_void_p(feat.data_ptr()),
                                         C.c_void_p(y.data_ptr()), C.c_void_p(w.data_ptr()),
                                         C.c_void_p(flags.data_ptr())),
              "mlp_coupled_rollout")
        self._keep = [u, st, feat, rigid, bd, y, w, flags]
        self._leave()
        return dict(y=y, wrench=w, feat=feat, rigid=rigid, flags=flags)

    def params(self) -> torch.Tensor:
        p = torch.empty(N_PARAMS, device=self.device)
        self._enter()
        check(self.L.mlp_get_params(self.h, C.c_void_p(p.data_ptr())), "mlp_get_params")
        self._leave()
        return p

    def close(self):
        if getattr(self, "h", None):
            self.stream.synchronize()
            check(self.L.mlp_destroy(self.h), "mlp_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
