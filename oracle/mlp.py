"""FP64 NumPy reference of the slosh-wrench surrogate network.

TEST INFRASTRUCTURE ONLY.  Shares no code with the HIP kernels.

Network: input window of 32 past samples x 4 channels (theta, omega, input
torque, fill) flattened to 128 features, four hidden Linear(256) + GELU
layers, and a Linear(3) head giving the body-frame slosh force (2) and torque
(1).  GELU is the tanh form of Hendrycks and Gimpel (2016):
    gelu(x) = x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))).
Loss: mean squared error over the batch and the three outputs, the same
criterion as the paper's prediction-error objective (eq. pem) applied to the
wrench.  Optimiser: Adam (Kingma and Ba 2015) with bias correction.

Weights are kept as a list of (W [out, in], b [out]) pairs.
"""
from __future__ import annotations

import math

import numpy as np

K_GELU = math.sqrt(2.0 / math.pi)
C_GELU = 0.044715


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(K_GELU * (x + C_GELU * x ** 3)))


def gelu_grad(x):
    u = K_GELU * (x + C_GELU * x ** 3)
    t = np.tanh(u)
    du = K_GELU * (1.0 + 3.0 * C_GELU * x ** 2)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du


def init_params(rng: np.random.Generator, dims=(128, 256, 256, 256, 256, 3)):
    """Uniform fan-in initialisation, U(-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    params = []
    for i in range(len(dims) - 1):
        bound = 1.0 / math.sqrt(dims[i])
        W = rng.uniform(-bound, bound, size=(dims[i + 1], dims[i]))
        b = rng.uniform(-bound, bound, size=(dims[i + 1],))
        params.append((W, b))
    return params


def forward(params, x):
    """Returns the output [B, 3] and the per-layer pre-activations."""
    a = np.asarray(x, np.float64)
    pre = []
    acts = [a]
    for li, (W, b) in enumerate(params):
        z = a @ W.T + b
        pre.append(z)
        a = gelu(z) if li < len(params) - 1 else z
        acts.append(a)
    return a, pre, acts


def loss(params, x, y):
    out, _, _ = forward(params, x)
    return float(np.mean((out - y) ** 2))


def backward(params, x, y):
    """Gradients of the mean squared error, by the chain rule written out."""
    out, _, _ = forward(params, x)
    B, D = out.shape
    return backward_from(params, x, 2.0 * (out - y) / (B * D))   # dL/d out of the mean


def backward_from(params, x, dy):
    """Gradients of any loss whose derivative with respect to the output is
    dy [B, 3], by the chain rule written out."""
    _, pre, acts = forward(params, x)
    g = np.asarray(dy, np.float64)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        if li < len(params) - 1:
            g = g * gelu_grad(pre[li])     # through the activation
        gW = g.T @ acts[li]
        gb = g.sum(axis=0)
        grads[li] = (gW, gb)
        g = g @ W
    return grads


class Adam:
    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads):
        self.t += 1
        out = []
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for j, (p, gp) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[i][j] + (1 - self.b1) * gp
                v = self.b2 * self.v[i][j] + (1 - self.b2) * gp * gp
                self.m[i] = tuple(m if k == j else self.m[i][k] for k in range(2))
                self.v[i] = tuple(v if k == j else self.v[i][k] for k in range(2))
                new.append(p - self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append((new[0], new[1]))
        return out


# --------------------------------------------------------------------------
# The network in place of SPH: rigid body driven by the surrogate's wrench
# --------------------------------------------------------------------------

def window_input(feat, static, norm, k, window=32):
    """Standardised input of the window that ends at log sample k, for every
    rollout: samples k - window + 1 .. k, four channels each (theta,
    thetadot, input torque, and in the fourth the rollout's constant
    number (t - first sample) mod n_static), each channel minus its training
    mean over its training std.  feat [R, T, 3], static [R, n_static], norm as
    the window kernel takes it (input means, input stds, output means, output
    stds).  Returns [R, window * 4]."""
    feat = np.asarray(feat, np.float64)
    static = np.asarray(static, np.float64)
    norm = np.asarray(norm, np.float64)
    R = feat.shape[0]
    ns = static.shape[1]
    ni = 3 + ns
    mean, std = norm[:ni], norm[ni:2 * ni]
    x = np.empty((R, window, 4))
    for i in range(window):
        t = k - window + 1 + i
        x[:, i, :3] = (feat[:, t, :] - mean[:3]) / std[:3]
        q = i % ns
        x[:, i, 3] = (static[:, q] - mean[3 + q]) / std[3 + q]
    return x.reshape(R, window * 4)


def coupled_rollout(params, norm, static, feat0, rigid0, u_seq, body, log_stride, window=32):
    """The spacecraft simulated with the surrogate standing in for the fluid
    (the use of the surrogate in Section 4 and in the closed-loop validation
    of Section 5.3): at every log sample k from window - 1 on, the network's
    output for the window ending at k, de-standardised, is the mean
    body-frame slosh wrench over log interval k (steps k log_stride .. (k+1)
    log_stride - 1); the free rigid body integrates those steps with that
    wrench and the applied inputs by eq. tankdynamics,
        m r'' = R(theta) F_body[0:2] + u[0:2],   J theta'' = F_body[2] + u[2],
    R(theta) = [[cos, -sin], [sin, cos]], with first-order symplectic Euler
    (Section 3.4: velocities first, positions with the new velocities).
    Sample k + 1 then records the state and the features of the next window
    (theta, thetadot, the input torque of the sample's first step).

    params: network weights; norm: the window norm vector; static [R, ns];
    feat0 [R, window, 3] the first window's features; rigid0 [R, 6] = r_x,
    r_y, theta, rdot_x, rdot_y, thetadot at sample window - 1; u_seq
    [R, n_steps, 3]; body [R, 3] = mass, inertia, dt.  Returns dict(y
    [R, T, 6] with NaN before sample window, wrench [R, T, 3] with NaN before
    interval window - 1, feat [R, T, 3], rigid [R, 6] after the last step)."""
    norm = np.asarray(norm, np.float64)
    u_seq = np.asarray(u_seq, np.float64)
    body = np.asarray(body, np.float64)
    R, n_steps, _ = u_seq.shape
    T = -(-n_steps // log_stride)
    ni = 3 + np.asarray(static).shape[1]
    out_mean, out_std = norm[2 * ni:2 * ni + 3], norm[2 * ni + 3:2 * ni + 6]
    feat = np.zeros((R, T, 3))
    feat[:, :window] = np.asarray(feat0, np.float64)
    y = np.full((R, T, 6), np.nan)
    wrench = np.full((R, T, 3), np.nan)
    st = np.array(rigid0, np.float64)
    mass, inertia, dt = body[:, 0], body[:, 1], body[:, 2]
    for k in range(window - 1, T):
        out, _, _ = forward(params, window_input(feat, static, norm, k, window))
        F = out * out_std + out_mean
        wrench[:, k] = F
        for n in range(k * log_stride, min((k + 1) * log_stride, n_steps)):
            u = u_seq[:, n]
            c, s = np.cos(st[:, 2]), np.sin(st[:, 2])
            acc = np.stack([(c * F[:, 0] - s * F[:, 1] + u[:, 0]) / mass,
                            (s * F[:, 0] + c * F[:, 1] + u[:, 1]) / mass,
                            (F[:, 2] + u[:, 2]) / inertia], axis=1)
            st[:, 3:6] += dt[:, None] * acc
            st[:, 0:3] += dt[:, None] * st[:, 3:6]
        if k + 1 < T:
            y[:, k + 1] = st
            feat[:, k + 1] = np.stack([st[:, 2], st[:, 5], u_seq[:, (k + 1) * log_stride, 2]], axis=1)
    return dict(y=y, wrench=wrench, feat=feat, rigid=st)
