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
