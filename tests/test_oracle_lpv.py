"""Pins of the LPV surrogate oracle (oracle/lpv.py).

* With the scheduling-dependent matrices zero the model is the LTI system
  (A0, B0, C0, D = 0): its response equals scipy.signal.dlsim's.
* With A1, B1, C1 nonzero but a scheduling map whose last layer is zero,
  p_k = b3 is constant: the response equals the LTI system A0 + b3 A1, ...
* The loss of the exact parameters on their own outputs is the
  regularization alone; the central-difference gradient of a quadratic
  special case matches its closed form.
* BFR is 100 % for an exact fit and 0 % for the mean.
"""
import numpy as np
import pytest
from scipy import signal

from oracle import lpv as L


def _random_params(rng, scale=0.3):
    v = rng.normal(size=L.N_PARAM) * scale
    P = L.unpack(v)
    P["A0"][:] = 0.5 * np.eye(4) + 0.1 * rng.normal(size=(4, 4))
    return L.pack(P)


def test_parameter_count():
    assert L.N_THETA == 137 and L.N_PARAM == 141


def test_lti_special_case_is_dlsim():
    rng = np.random.default_rng(0)
    P = L.unpack(_random_params(rng))
    for name in ("A1", "B1", "C1"):
        P[name][:] = 0.0
    v = L.pack(P)
    u = rng.normal(size=(60, 3))
    _, y_ref, _ = signal.dlsim((P["A0"], P["B0"], P["C0"], np.zeros((3, 3)), 1.0), u, x0=P["x0"])
    assert np.allclose(L.simulate(v, u), y_ref, rtol=1e-12, atol=1e-12)


def test_constant_schedule_is_a_shifted_lti_system():
    rng = np.random.default_rng(1)
    P = L.unpack(_random_params(rng))
    P["W3"][:] = 0.0
    P["b3"][:] = 0.7
    v = L.pack(P)
    u = rng.normal(size=(40, 3))
    A = P["A0"] + 0.7 * P["A1"]
    B = P["B0"] + 0.7 * P["B1"]
    Cm = P["C0"] + 0.7 * P["C1"]
    _, y_ref, _ = signal.dlsim((A, B, Cm, np.zeros((3, 3)), 1.0), u, x0=P["x0"])
    assert np.allclose(L.simulate(v, u), y_ref, rtol=1e-10, atol=1e-10)


def test_loss_of_the_true_parameters_is_the_regularization():
    rng = np.random.default_rng(2)
    v = _random_params(rng)
    u = rng.normal(size=(30, 3))
    y = L.simulate(v, u)
    s2, sx = 1e-3, 1e-2
    expect = 0.5 * s2 * (v[:L.N_THETA] ** 2).sum() + 0.5 * sx * (v[L.N_THETA:] ** 2).sum()
    assert L.loss(v, u, y, s2, sx) == pytest.approx(expect, rel=1e-12)


def test_fd_gradient_of_the_output_map_closed_form():
    # A = 0, B = 0: y_0 = C0 x0 and y_k = 0 after; J = |y0 - C0 x0|^2 / N
    rng = np.random.default_rng(3)
    P = L.unpack(np.zeros(L.N_PARAM))
    P["C0"][:] = rng.normal(size=(3, 4))
    P["x0"][:] = rng.normal(size=4)
    v = L.pack(P)
    N = 5
    u = np.zeros((N, 3))
    y = np.zeros((N, 3))
    y[0] = rng.normal(size=3)
    g = L.loss_grad_fd(v, u, y, 0.0, 0.0)
    r = P["C0"] @ P["x0"] - y[0]
    gC0 = 2.0 / N * np.outer(r, P["x0"])
    gx0 = 2.0 / N * P["C0"].T @ r
    G = L.unpack(g)
    assert np.allclose(G["C0"], gC0, atol=1e-7)
    assert np.allclose(G["x0"], gx0, atol=1e-7)


def test_bfr_limits():
    rng = np.random.default_rng(4)
    y = rng.normal(size=(50, 3))
    assert np.allclose(L.bfr(y, y), 100.0)
    assert np.allclose(L.bfr(y, np.tile(y.mean(0), (50, 1))), 0.0)


def test_autodiff_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    v = _random_params(rng)
    u = rng.normal(size=(25, 3))
    y = rng.normal(size=(25, 3))
    f, g = L.loss_and_grad(v, u, y, 1e-3, 1e-2)
    assert f == pytest.approx(L.loss(v, u, y, 1e-3, 1e-2), rel=1e-13)
    fd = L.loss_grad_fd(v, u, y, 1e-3, 1e-2)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(fd)))


def test_adam_first_step_is_a_signed_step():
    # with zero moments the bias-corrected first update is lr g / (|g| + eps)
    rng = np.random.default_rng(6)
    v = _random_params(rng)
    u = rng.normal(size=(10, 3))
    y = rng.normal(size=(10, 3))
    _, g = L.loss_and_grad(v, u, y, 0.0, 0.0)
    v1, _ = L.adam(v, u, y, 0.0, 0.0, 1, lr=1e-2)
    assert np.allclose(v - v1, 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_mask_freezes_entries():
    rng = np.random.default_rng(7)
    v = _random_params(rng)
    u = rng.normal(size=(10, 3))
    y = rng.normal(size=(10, 3))
    m = L.lti_mask()
    v1, _ = L.adam(v, u, y, 1e-4, 1e-6, 3, mask=m)
    assert np.array_equal(v1[m == 0], v[m == 0])
    assert np.all(v1[m == 1] != v[m == 1])


def test_lbfgs_solves_a_quadratic():
    rng = np.random.default_rng(8)
    Q = rng.normal(size=(12, 12))
    Q = Q @ Q.T + 12 * np.eye(12)
    b = rng.normal(size=12)

    def fun(x):
        return 0.5 * x @ Q @ x - b @ x, Q @ x - b

    # stops on the gradient or when f no longer decreases in FP64
    x, f, k, status = L.lbfgs(fun, np.zeros(12), 200, gtol=1e-9, ftol=0.0)
    assert status in (1, 2) and k < 60
    assert np.allclose(x, np.linalg.solve(Q, b), rtol=1e-8, atol=1e-8)


def test_lbfgs_rosenbrock():
    def fun(x):
        f = (1 - x[0]) ** 2 + 100 * (x[1] - x[0] ** 2) ** 2
        g = np.array([-2 * (1 - x[0]) - 400 * x[0] * (x[1] - x[0] ** 2), 200 * (x[1] - x[0] ** 2)])
        return f, g

    x, f, k, status = L.lbfgs(fun, np.array([-1.2, 1.0]), 500, gtol=1e-9, ftol=0.0)
    assert status == 1
    assert np.allclose(x, [1.0, 1.0], atol=1e-6)


def test_closed_loop_open_gains_is_the_open_loop_model():
    # kp = kd = 0 and C1 = 0: the measured velocities are the open-loop
    # outputs for the input (force, 0), the positions their running sum * ts
    rng = np.random.default_rng(9)
    P = L.unpack(_random_params(rng))
    P["C1"][:] = 0.0
    v = L.pack(P)
    n, ts = 50, 0.05
    force = rng.normal(size=(n, 2))
    us, ys = np.array([2.0, 3.0, 4.0]), np.array([0.5, 0.25, 2.0])
    out, tau = L.closed_loop(v, force, np.zeros(n), ts, 0.0, 0.0, us, ys, x0=P["x0"])
    u = np.concatenate([force, np.zeros((n, 1))], 1) / us
    y = L.simulate(v, u) * ys
    assert np.allclose(out[:, 3:], y, rtol=1e-12, atol=1e-12)
    pos = np.concatenate([np.zeros((1, 3)), ts * np.cumsum(y, 0)[:-1]])
    assert np.allclose(out[:, :3], pos, rtol=1e-12, atol=1e-12)
    assert np.all(tau == 0.0)


def test_closed_loop_pd_on_a_double_integrator():
    # an LTI model that is exactly the sampled rigid body (velocity += ts F / m,
    # thetadot += ts tau / J) under the PD law: the (theta, thetadot) loop is
    # the linear system [[1, ts], [-ts kp/J, 1 - ts kd/J]] driven by ts kp/J ref
    ts, m, J = 0.05, 1000.0, 133.84
    w, xi = 0.2 * np.pi, 0.7
    kp, kd = J * w * w, 2 * xi * J * w
    P = L.unpack(np.zeros(L.N_PARAM))
    P["A0"][:] = np.diag([1.0, 1.0, 1.0, 0.0])
    P["B0"][:3, :3] = np.diag([ts / m, ts / m, ts / J])
    P["C0"][:, :3] = np.eye(3)
    v = L.pack(P)
    n = 400
    ref = np.where(np.arange(n) >= 20, 0.3, 0.0)
    out, tau = L.closed_loop(v, np.zeros((n, 2)), ref, ts, kp, kd, np.ones(3), np.ones(3))
    A = np.array([[1.0, ts], [-ts * kp / J, 1.0 - ts * kd / J]])
    B = np.array([[0.0], [ts * kp / J]])
    _, yy, _ = signal.dlsim((A, B, np.eye(2), np.zeros((2, 1)), ts), ref[:, None])
    assert np.allclose(out[:, 2], yy[:, 0], rtol=1e-10, atol=1e-12)
    assert np.allclose(out[:, 5], yy[:, 1], rtol=1e-10, atol=1e-12)
    assert abs(out[-1, 2] - 0.3) < 1e-3          # the loop settles on the reference
