"""Pins of the oracle's rigid-body coupling, frames and integrator.

* World-frame mode (eq. kinematicghost read literally): with no external
  load, total linear momentum m_b rdot + sum m v_i and total angular momentum
  J thetadot + m_b r x rdot + sum m x_i x v_i are conserved to rounding by
  symplectic Euler, because every pair force -- fluid-fluid and fluid-wall --
  is central and the tank takes the reactions (eqs. pressure_f2b,
  viscous_f2b, tankdynamics).
* Body frame vs world frame: the two formulations agree to first order in dt.
* A lone particle that feels no SPH force moves on a straight line in the
  world frame whatever the tank does (fictitious accelerations are right).
* Rigid body alone: constant torque gives theta_n = (tau/J) dt^2 n(n+1)/2
  exactly under symplectic Euler; the PD law of Section 5.1 with a fast hold
  follows the textbook second-order step response; the zero-order hold keeps
  the torque constant between control instants; the prescribed rotation is
  A sin(2 pi f t).
* The oracle's central differences (the reference gradient of the
  linearization tests) reproduce the rigid body's closed-form sensitivities.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import sph as O


def _small_circle(seed=0, dx=0.01, fill=0.5, R=0.06):
    rng = np.random.default_rng(seed)
    fluid, ghosts = W.circle_tank(R, dx, fill, 3, rng, 0.01)
    p = W._fluid_params(dx)
    p.motion, p.ctrl = W.MOTION_FREE, W.CTRL_NONE
    p.body_mass, p.body_inertia = 2.0, 0.01
    pad = 6 * dx
    p.domain_min, p.domain_max = (-R - pad, -R - pad), (R + pad, R + pad)
    return p, fluid.astype(np.float64), ghosts.astype(np.float64)


def _body_to_world(s, w, rigid):
    th, thd = rigid[2], rigid[5]
    c, sn = math.cos(th), math.sin(th)
    R = np.array([[c, -sn], [sn, c]])
    x = rigid[:2] + s @ R.T
    Js = np.stack([-s[:, 1], s[:, 0]], 1)
    v = rigid[3:5] + (w + thd * Js) @ R.T
    return x, v


def _momenta(p, x, v, rigid):
    m = p.mass
    P = p.body_mass * rigid[3:5] + m * v.sum(0)
    L = (p.body_inertia * rigid[5] + p.body_mass * (rigid[0] * rigid[4] - rigid[1] * rigid[3])
         + m * (x[:, 0] * v[:, 1] - x[:, 1] * v[:, 0]).sum())
    return P, L


def test_world_mode_conserves_linear_and_angular_momentum():
    p, fluid, ghosts = _small_circle()
    rng = np.random.default_rng(5)
    rigid = np.array([0.01, -0.02, 0.3, 0.05, -0.03, 0.8])
    s = fluid
    w = rng.normal(0, 0.2, s.shape)
    x, v = _body_to_world(s, w, rigid)
    P0, L0 = _momenta(p, x, v, rigid)
    x1, v1, rg1, _, wl = O.rollout_world(p, x, v, ghosts, rigid, 40)
    P1, L1 = _momenta(p, x1, v1, rg1)
    assert np.abs(wl).max() > 0                       # the wall did push
    scaleP = p.body_mass * np.abs(rigid[3:5]).max() + p.mass * np.abs(v).sum()
    assert np.abs(P1 - P0).max() < 1e-12 * scaleP
    scaleL = abs(p.body_inertia * rigid[5]) + p.mass * np.abs(x[:, 0] * v[:, 1] - x[:, 1] * v[:, 0]).sum()
    assert abs(L1 - L0) < 1e-12 * scaleL


def _body_vs_world_error(dt_scale, T=0.02):
    p, fluid, ghosts = _small_circle(fill=0.6)
    p.dt = p.dt * dt_scale
    n = int(round(T / p.dt))
    rigid = np.array([0.0, 0.0, 0.2, 0.0, 0.0, 2.0])
    u = np.zeros((n, 3), np.float32)
    u[:, 0], u[:, 2] = 0.5, 0.01
    st = O.State(fluid.copy(), np.zeros_like(fluid), rigid.copy())
    O.rollout(p, st, ghosts, n, u)
    x0, v0 = _body_to_world(fluid, np.zeros_like(fluid), rigid)
    xw, vw, rgw, _, _ = O.rollout_world(p, x0, v0, ghosts, rigid, n, u)
    xb, vb = _body_to_world(st.s, st.w, st.rigid)
    return np.abs(xb - xw).max(), abs(st.rigid[2] - rgw[2])


def test_body_frame_converges_to_world_frame_first_order():
    e1, t1 = _body_vs_world_error(1.0)
    e2, t2 = _body_vs_world_error(0.5)
    e4, t4 = _body_vs_world_error(0.25)
    assert e1 > 0
    assert 1.6 < e1 / e2 < 2.6 and 1.6 < e2 / e4 < 2.6, (e1, e2, e4)
    assert t2 < t1 and t4 < t2


def _free_particle_world_path(dt_scale):
    p = W._fluid_params(0.01)
    p.motion = W.MOTION_SINE
    p.sine_amp, p.sine_freq = 0.4, 2.0
    p.dt *= dt_scale
    p.domain_min, p.domain_max = (-1, -1), (1, 1)
    n = int(round(0.1 / p.dt))
    rigid = np.array([0, 0, 0, 0, 0, 2 * math.pi * p.sine_freq * p.sine_amp])
    s0 = np.array([[0.2, 0.1]])
    v_world = np.array([0.3, -0.4])
    # body-frame velocity of a particle that moves with v_world at t = 0
    w0 = v_world - rigid[5] * np.array([[-s0[0, 1], s0[0, 0]]])
    st = O.State(s0.copy(), w0.copy(), rigid.copy())
    O.rollout(p, st, np.zeros((0, 2)), n)
    x, _ = _body_to_world(st.s, st.w, st.rigid)
    return np.abs(x[0] - (s0[0] + v_world * n * p.dt)).max()


def test_lone_particle_moves_on_a_straight_line_in_the_world():
    e1 = _free_particle_world_path(1.0)
    e2 = _free_particle_world_path(0.5)
    assert e1 < 2e-3 and 1.6 < e1 / e2 < 2.6, (e1, e2)


def _rigid_only(**kw):
    p = W.Params(h=0.01, h_spiky=0.01, mass=0.1, dt=1e-3, body_mass=10.0, body_inertia=2.0,
                 domain_min=(-1, -1), domain_max=(1, 1))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_constant_load_gives_the_discrete_closed_form():
    p = _rigid_only()
    n = 500
    u = np.tile(np.array([[3.0, -1.0, 0.25]], np.float32), (n, 1))
    st = O.State(np.zeros((0, 2)), np.zeros((0, 2)), np.zeros(6))
    O.rollout(p, st, np.zeros((0, 2)), n, u)
    k = p.dt ** 2 * n * (n + 1) / 2
    assert st.rigid[2] == pytest.approx(0.25 / p.body_inertia * k, rel=1e-12)
    assert st.rigid[0] == pytest.approx(3.0 / p.body_mass * k, rel=1e-12)
    assert st.rigid[1] == pytest.approx(-1.0 / p.body_mass * k, rel=1e-12)
    assert st.rigid[5] == pytest.approx(0.25 / p.body_inertia * n * p.dt, rel=1e-12)


def test_oracle_differences_give_the_rigid_sensitivities():
    # the central differences that serve as the reference gradient of the
    # linearization tests, on the rigid body alone: d theta_n / d u_k =
    # dt^2 (n - k) / J and d theta_n / d thetadot_0 = n dt under symplectic Euler
    p = _rigid_only()
    n, k, eps = 60, 13, 1e-3

    def final(u, rigid0):
        st = O.State(np.zeros((0, 2)), np.zeros((0, 2)), np.asarray(rigid0, np.float64))
        O.rollout(p, st, np.zeros((0, 2)), n, u)
        return st.rigid

    u0 = np.zeros((n, 3), np.float32)
    du = np.zeros((n, 3), np.float32)
    du[k, 2] = 1.0
    d = (final(u0 + eps * du, np.zeros(6)) - final(u0 - eps * du, np.zeros(6))) / (2 * eps)
    assert d[2] == pytest.approx(p.dt ** 2 * (n - k) / p.body_inertia, rel=1e-6)
    assert d[5] == pytest.approx(p.dt / p.body_inertia, rel=1e-6)
    r = np.zeros(6)
    r[5] = 1.0
    d = (final(u0, eps * r) - final(u0, -eps * r)) / (2 * eps)
    assert d[2] == pytest.approx(n * p.dt, rel=1e-9)


def test_pd_attitude_law_tracks_textbook_step_response():
    J, w, xi = 500.0, 0.2 * math.pi, 0.7
    p = _rigid_only(body_inertia=J, ctrl=W.CTRL_PD_ZOH, kp=J * w * w, kd=2 * xi * J * w,
                    ctrl_period=1, dt=2e-3)
    n = 6000
    ref = np.full(n + 1, 0.5)
    st = O.State(np.zeros((0, 2)), np.zeros((0, 2)), np.zeros(6))
    _, logs = O.rollout(p, st, np.zeros((0, 2)), n, theta_ref=ref, log_stride=100)
    t = np.arange(logs["y"].shape[0]) * 100 * p.dt
    wd = w * math.sqrt(1 - xi * xi)
    exact = 0.5 * (1 - np.exp(-xi * w * t) * (np.cos(wd * t) + xi / math.sqrt(1 - xi * xi) * np.sin(wd * t)))
    assert np.abs(logs["y"][:, 2] - exact).max() < 5e-3 * 0.5


def test_zero_order_hold_holds_the_torque():
    J = 500.0
    p = _rigid_only(body_inertia=J, ctrl=W.CTRL_PD_ZOH, kp=100.0, kd=300.0, ctrl_period=7)
    n = 70
    st = O.State(np.zeros((0, 2)), np.zeros((0, 2)), np.zeros(6))
    _, logs = O.rollout(p, st, np.zeros((0, 2)), n, theta_ref=np.full(20, 0.3), log_stride=1)
    tau = logs["u"][:, 2]
    for k in range(10):
        blk = tau[7 * k:7 * k + 7]
        assert np.all(blk == blk[0])
    # each held value is the PD law at the sampled state
    for k in range(10):
        th, thd = logs["y"][7 * k, 2], logs["y"][7 * k, 5]
        assert tau[7 * k] == pytest.approx(100.0 * (0.3 - th) - 300.0 * thd, rel=1e-12, abs=1e-12)


def test_prescribed_rotation_is_the_sine():
    sc = W.plain_rect(n_steps=40)
    st = O.state_from_scenario(sc)
    _, logs = O.rollout(sc.params, st, sc.ghosts, 40, sc.u_seq, log_stride=10)
    t = np.arange(4) * 10 * sc.params.dt
    assert np.allclose(logs["y"][:, 2], 0.1 * np.sin(2 * math.pi * 0.5 * t), rtol=0, atol=1e-15)
    assert np.allclose(logs["y"][:, 5], 0.1 * math.pi * np.cos(math.pi * t), rtol=0, atol=1e-15)
