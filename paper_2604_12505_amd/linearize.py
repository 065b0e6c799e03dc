"""Differentiable rollouts on top of the tangent-linear step.

``FinalWrench`` is a ``torch.autograd.Function``: the slosh wrench (body
frame) of the last step of an n-step rollout, as a function of the applied
force/torque sequence u [n, 3] and the initial rigid state [6], from a fixed
fluid checkpoint.  Its forward runs the library's rollout (``sph_set_state``,
``sph_rollout``, ``sph_slosh_wrench``); its backward is one adjoint rollout
(``sph_vjp_rollout``: reverse mode, the state kept every 20 steps and each
segment recomputed).  ``wrench_jacobian`` assembles the full Jacobian from
the tangent-linear rollout (``sph_jvp_rollout``, forward mode, 64 directions
per call).  Argument marshalling only: every derivative is computed by the
library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

MAX_DIR = 64
EVERY = 20   # steps between stored states of the adjoint rollout


def input_directions(n_steps: int, first: int, count: int):
    """Unit directions first .. first+count-1 of the flattened input
    (u [n_steps, 3] row-major, then the 6 rigid-state entries)."""
    du = np.zeros((count, n_steps, 3), np.float32)
    dr = np.zeros((count, 6))
    for k in range(count):
        i = first + k
        if i < 3 * n_steps:
            du[k, i // 3, i % 3] = 1.0
        else:
            dr[k, i - 3 * n_steps] = 1.0
    return du, dr


def wrench_jacobian(sim, checkpoint, u_seq, rigid0, theta_ref=None) -> np.ndarray:
    """d wrench / d (u, rigid0): [3, 3 n + 6], column by column from the
    tangent-linear rollout."""
    s, w, tau, step = checkpoint
    n = int(u_seq.shape[0])
    n_in = 3 * n + 6
    jac = np.zeros((3, n_in))
    for b0 in range(0, n_in, MAX_DIR):
        k = min(MAX_DIR, n_in - b0)
        du, dr = input_directions(n, b0, k)
        sim.set_state(s, w, np.asarray(rigid0, np.float64), tau, step)
        r = sim.jvp_rollout(n, u_seq, du, theta_ref, dr)
        jac[:, b0:b0 + k] = r["dwrench"].T
    return jac


class FinalWrench(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u_seq, rigid0, sim, checkpoint, theta_ref=None):
        s, w, tau, step = checkpoint
        n = int(u_seq.shape[0])
        sim.set_state(s, w, rigid0.detach().cpu().double().numpy(), tau, step)
        sim.rollout(n, u_seq.detach(), theta_ref=theta_ref, logs=False)
        out = sim.wrench().double().to(u_seq.device)
        ctx.save_for_backward(u_seq, rigid0)
        ctx.sim, ctx.checkpoint, ctx.theta_ref = sim, checkpoint, theta_ref
        return out

    @staticmethod
    def backward(ctx, grad_out):
        u_seq, rigid0 = ctx.saved_tensors
        s, w, tau, step = ctx.checkpoint
        n = int(u_seq.shape[0])
        sim = ctx.sim
        sim.set_state(s, w, rigid0.detach().cpu().double().numpy(), tau, step)
        g = sim.vjp_rollout(n, grad_out.detach().cpu().double().numpy(), u_seq.detach(), ctx.theta_ref,
                            every=EVERY)
        gu = g["u"].to(device=u_seq.device, dtype=u_seq.dtype)
        gr = torch.as_tensor(g["rigid0"], dtype=rigid0.dtype, device=rigid0.device)
        return gu, gr, None, None, None
