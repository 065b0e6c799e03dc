"""Pins of the FP64 surrogate-network oracle.

* Backward pass equals central finite differences of the loss.
* The tanh GELU is within its known approximation error of the exact
  x Phi(x) (erf form), and its derivative equals finite differences.
* Adam's first bias-corrected step moves every weight by lr * sign(g).
"""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import mlp as M


def test_gelu_close_to_exact_erf_form():
    x = np.linspace(-8, 8, 20001)
    exact = 0.5 * x * (1 + erf(x / math.sqrt(2)))
    assert np.abs(M.gelu(x) - exact).max() < 1e-3


def test_gelu_grad_is_derivative():
    x = np.linspace(-5, 5, 1001)
    e = 1e-6
    fd = (M.gelu(x + e) - M.gelu(x - e)) / (2 * e)
    assert np.abs(M.gelu_grad(x) - fd).max() < 1e-8


@pytest.mark.parametrize("dims", [(6, 5, 4, 3), (128, 256, 256, 256, 256, 3)])
def test_backward_equals_finite_differences(dims):
    rng = np.random.default_rng(1)
    params = M.init_params(rng, dims)
    x = rng.normal(size=(5, dims[0]))
    y = rng.normal(size=(5, dims[-1]))
    grads = M.backward(params, x, y)
    e = 1e-6
    for li in range(len(params)):
        W, b = params[li]
        for _ in range(6):
            i, j = rng.integers(W.shape[0]), rng.integers(W.shape[1])
            Wp = W.copy(); Wp[i, j] += e
            Wm = W.copy(); Wm[i, j] -= e
            lp = M.loss(params[:li] + [(Wp, b)] + params[li + 1:], x, y)
            lm = M.loss(params[:li] + [(Wm, b)] + params[li + 1:], x, y)
            assert grads[li][0][i, j] == pytest.approx((lp - lm) / (2 * e), rel=1e-5, abs=1e-10)
        k = rng.integers(b.shape[0])
        bp = b.copy(); bp[k] += e
        bm = b.copy(); bm[k] -= e
        lp = M.loss(params[:li] + [(W, bp)] + params[li + 1:], x, y)
        lm = M.loss(params[:li] + [(W, bm)] + params[li + 1:], x, y)
        assert grads[li][1][k] == pytest.approx((lp - lm) / (2 * e), rel=1e-5, abs=1e-10)


def test_parameter_count():
    params = M.init_params(np.random.default_rng(0))
    assert sum(W.size + b.size for W, b in params) == 231171


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(2)
    params = M.init_params(rng, (4, 3, 2))
    grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in params]
    opt = M.Adam(params, lr=1e-2, eps=1e-12)
    new = opt.step(params, grads)
    for (W, b), (Wn, bn), (gW, gb) in zip(params, new, grads):
        assert np.allclose(Wn - W, -1e-2 * np.sign(gW), rtol=1e-9, atol=0)
        assert np.allclose(bn - b, -1e-2 * np.sign(gb), rtol=1e-9, atol=0)


def test_adam_fits_a_linear_map():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(2, 4))
    params = [(np.zeros((2, 4)), np.zeros(2))]
    opt = M.Adam(params, lr=5e-2)
    x = rng.normal(size=(64, 4))
    y = x @ A.T
    for _ in range(600):
        params = opt.step(params, M.backward(params, x, y))
    assert np.abs(params[0][0] - A).max() < 1e-3
