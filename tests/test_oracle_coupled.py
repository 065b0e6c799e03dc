"""Pins of the oracle's surrogate-driven rigid body (oracle.mlp.coupled_rollout).

Each pin is fixed by the mathematics, not by the oracle's own formulas:

* a network whose output is a constant (all weights zero, a head bias) gives
  a constant wrench, and first-order symplectic Euler under a constant
  acceleration a has the closed form v_n = v_0 + n dt a,
  x_n = x_0 + n dt v_0 + dt^2 a n (n + 1) / 2: checked for the attitude and,
  with the torques balanced so that the attitude stays put, for the
  translation through the body-to-inertial rotation of eq. tankdynamics;
* with unit standardisation a window is the plain slice of the logs;
* log interval k uses the window ending at sample k and the inputs of its
  own steps only: inputs after it leave everything up to sample k + 1 alone,
  an input on its last step moves sample k + 1.
"""
import numpy as np

from oracle import mlp as M

W = 32


def _const_net(beta):
    rng = np.random.default_rng(0)
    params = [(np.zeros_like(Wl), np.zeros_like(b)) for Wl, b in M.init_params(rng)]
    Wh, bh = params[-1]
    params[-1] = (Wh, np.asarray(beta, np.float64))
    return params


def _norm(n_static, out_mean, out_std):
    ni = 3 + n_static
    return np.concatenate([np.zeros(ni), np.ones(ni), out_mean, out_std])


def _setup(R=3, n_steps=45 * 7 + 4, stride=7, seed=1):
    rng = np.random.default_rng(seed)
    static = rng.uniform(0.2, 0.8, size=(R, 1))
    feat0 = rng.normal(size=(R, W, 3))
    body = np.stack([rng.uniform(500, 1500, R), rng.uniform(200, 800, R), rng.uniform(1e-4, 1e-3, R)], axis=1)
    return rng, static, feat0, body, n_steps, stride


def test_constant_wrench_attitude_closed_form():
    rng, static, feat0, body, n_steps, stride = _setup()
    R = body.shape[0]
    out_mean, out_std, beta = np.array([1.0, -2.0, 3.0]), np.array([2.0, 0.5, 4.0]), np.array([0.5, 1.0, -0.25])
    F = beta * out_std + out_mean                         # (2, -1.5, 2)
    tau = rng.normal(size=R)
    u = np.zeros((R, n_steps, 3))
    u[:, :, 2] = tau[:, None]
    rigid0 = rng.normal(size=(R, 6))
    res = M.coupled_rollout(_const_net(beta), _norm(1, out_mean, out_std), static, feat0, rigid0, u, body, stride)
    T = -(-n_steps // stride)
    assert np.allclose(res["wrench"][:, W - 1:], F, rtol=0, atol=1e-15)
    dt, J = body[:, 2], body[:, 1]
    alpha = (F[2] + tau) / J
    for k in range(W - 1, T - 1):
        n = (k + 1 - (W - 1)) * stride                    # steps since sample W - 1
        om = rigid0[:, 5] + n * dt * alpha
        th = rigid0[:, 2] + n * dt * rigid0[:, 5] + dt * dt * alpha * n * (n + 1) / 2
        np.testing.assert_allclose(res["y"][:, k + 1, 5], om, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(res["y"][:, k + 1, 2], th, rtol=1e-12, atol=1e-14)
        # the features of the next window: theta, thetadot, the torque of the sample's step
        np.testing.assert_array_equal(res["feat"][:, k + 1], np.stack([res["y"][:, k + 1, 2], res["y"][:, k + 1, 5],
                                                                     u[:, (k + 1) * stride, 2]], axis=1))
    # the last (partial) interval: n_steps is not a multiple of the stride
    n = n_steps - (W - 1) * stride
    np.testing.assert_allclose(res["rigid"][:, 5], rigid0[:, 5] + n * dt * alpha, rtol=1e-12, atol=1e-14)


def test_constant_wrench_translation_through_the_rotation():
    rng, static, feat0, body, n_steps, stride = _setup(seed=2)
    R = body.shape[0]
    out_mean, out_std = np.zeros(3), np.ones(3)
    beta = np.array([3.0, -1.0, 0.75])
    F = beta
    u = np.zeros((R, n_steps, 3))
    u[:, :, 0] = rng.normal(size=R)[:, None]
    u[:, :, 1] = rng.normal(size=R)[:, None]
    u[:, :, 2] = -F[2]                                    # balanced torque: the attitude stays put
    rigid0 = rng.normal(size=(R, 6))
    rigid0[:, 2] = np.array([0.7, -2.1, 2.9])             # attitudes in several quadrants
    rigid0[:, 5] = 0.0
    res = M.coupled_rollout(_const_net(beta), _norm(1, out_mean, out_std), static, feat0, rigid0, u, body, stride)
    th0 = rigid0[:, 2]
    c, s = np.cos(th0), np.sin(th0)
    m, dt = body[:, 0], body[:, 2]
    a = np.stack([(c * F[0] - s * F[1] + u[:, 0, 0]) / m, (s * F[0] + c * F[1] + u[:, 0, 1]) / m], axis=1)
    T = -(-n_steps // stride)
    for k in range(W - 1, T - 1):
        n = (k + 1 - (W - 1)) * stride
        np.testing.assert_array_equal(res["y"][:, k + 1, 2], th0)
        v = rigid0[:, 3:5] + n * dt[:, None] * a
        x = rigid0[:, 0:2] + n * dt[:, None] * rigid0[:, 3:5] + (dt * dt * n * (n + 1) / 2)[:, None] * a
        np.testing.assert_allclose(res["y"][:, k + 1, 3:5], v, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(res["y"][:, k + 1, 0:2], x, rtol=1e-12, atol=1e-13)


def test_window_is_the_slice_of_the_logs_under_unit_standardisation():
    rng = np.random.default_rng(3)
    R, T, ns = 4, 50, 3
    feat = rng.normal(size=(R, T, 3))
    static = rng.normal(size=(R, ns))
    norm = np.concatenate([np.zeros(3 + ns), np.ones(3 + ns), np.zeros(3), np.ones(3)])
    for k in (W - 1, 40, T - 1):
        x = M.window_input(feat, static, norm, k).reshape(R, W, 4)
        np.testing.assert_array_equal(x[:, :, :3], feat[:, k - W + 1:k + 1, :])
        for i in range(W):
            np.testing.assert_array_equal(x[:, i, 3], static[:, i % ns])


def test_each_interval_sees_only_its_own_inputs():
    rng, static, feat0, body, n_steps, stride = _setup(seed=4)
    R = body.shape[0]
    params = M.init_params(np.random.default_rng(5))
    norm = np.concatenate([np.zeros(4), np.array([1.0, 1.0, 5.0, 1.0]), np.zeros(3), np.array([50.0, 50.0, 20.0])])
    u = rng.normal(size=(R, n_steps, 3)) * 5.0
    rigid0 = rng.normal(size=(R, 6)) * 0.1
    base = M.coupled_rollout(params, norm, static, feat0, rigid0, u, body, stride)
    k = W + 5
    later = u.copy()
    later[:, (k + 1) * stride:] += 3.0                    # inputs after interval k
    res = M.coupled_rollout(params, norm, static, feat0, rigid0, later, body, stride)
    np.testing.assert_array_equal(res["y"][:, :k + 2], base["y"][:, :k + 2])
    np.testing.assert_array_equal(res["wrench"][:, :k + 1], base["wrench"][:, :k + 1])
    # the window of interval k + 1 ends at sample k + 1, whose torque
    # feature is the input of step (k + 1) stride: it moved
    assert np.all(res["wrench"][:, k + 1] != base["wrench"][:, k + 1])
    last = u.copy()
    last[:, (k + 1) * stride - 1, 2] += 3.0                # the last step of interval k
    res = M.coupled_rollout(params, norm, static, feat0, rigid0, last, body, stride)
    np.testing.assert_array_equal(res["y"][:, :k + 1], base["y"][:, :k + 1])
    np.testing.assert_array_equal(res["wrench"][:, :k + 1], base["wrench"][:, :k + 1])
    assert np.all(res["y"][:, k + 1, 5] != base["y"][:, k + 1, 5])
