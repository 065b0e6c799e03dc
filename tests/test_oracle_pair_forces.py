"""Value pins of the oracle's pair forces (eqs. momentum, viscous, pressure_b2f,
viscous_b2f) on configurations small enough to evaluate by hand.

Every expected value below is derived in closed form from the kernel at a
special radius, written out as a number of the normalised cubic-spline
constant c = 5/(14 pi h^2) (eq. cubicspline under the unit-integral reading)
or of the spiky constant 30/(pi hs^5) (eq. spiky3), so a dropped factor, a
wrong sign or a wrong coefficient anywhere in a pair term changes a value:

  W(0) = 4c,  W(h/2) = 23c/8,  W(h) = c,  W(3h/2) = c/8,  W(1.6h) = 0.064c,
  W'(h/2) = -15c/(4h),  W'(h) = -3c/h,  W'(3h/2) = -3c/(4h),
  W_s3'(hs/2) = -7.5/(pi hs^3).

The linear EOS P = k (rho - rho0) gives the pressures from those densities.
A second, purely mathematical pin: with summation density the symmetric
pressure force of eq. momentum is the gradient of the internal energy, so the
power it delivers equals -sum_i m (P_i/rho_i^2) d rho_i/dt exactly; the test
takes d rho/dt by central differences of the oracle's own density.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import sph as O

H = 0.013            # smoothing length of the pins (h = 1.3 dx, dx = 10 mm)
DX = 0.01
M = 1000.0 * DX * DX
C = 5.0 / (14.0 * math.pi * H * H)


def _params(alpha=0.0, beta=0.0, k=2.0e3, rho0=100.0, gamma1=1.0):
    """Linear EOS with rho0 below any density of the pins, so P > 0."""
    p = W._fluid_params(DX)
    assert p.h == pytest.approx(H, rel=1e-15)
    p.h = H
    p.h_spiky = H
    p.mass = M
    p.eos = W.EOS_LINEAR
    p.k_lin = k
    p.rho0 = rho0
    p.visc_alpha = alpha
    p.visc_beta = beta
    p.gamma1 = gamma1
    p.domain_min, p.domain_max = (-0.5, -0.5), (0.5, 0.5)
    return p


def _rhs(p, s, w, g, use_cells=True):
    s = np.asarray(s, np.float64)
    w = np.asarray(w, np.float64)
    st = O.State(s, w, np.zeros(6))
    return O.rhs(p, st, np.asarray(g, np.float64).reshape(-1, 2), use_cells=use_cells)


# --- fluid pair: i at the origin, j on the +x axis at r, and a ghost at
# (-1.6h, 0) that only adds to rho_i (it is 1.6h from i, beyond the spiky
# support h, and at least 2.1h from j), so the two pressures differ.

CASES = {
    # r/h: (W(r)/c, h W'(r)/c)
    0.5: (23.0 / 8.0, -15.0 / 4.0),
    1.5: (1.0 / 8.0, -3.0 / 4.0),
}
W_GHOST = 0.064      # W(1.6h)/c


def _pair_setup(q):
    wr, dwr = CASES[q]
    r = q * H
    s = [[0.0, 0.0], [r, 0.0]]
    g = [[-1.6 * H, 0.0]]
    rho_i = M * C * (4.0 + wr + W_GHOST)
    rho_j = M * C * (4.0 + wr)
    dW = dwr * C / H
    return r, s, g, rho_i, rho_j, dW


@pytest.mark.parametrize("q", [0.5, 1.5])
@pytest.mark.parametrize("use_cells", [True, False])
def test_fluid_pair_pressure_force_value(q, use_cells):
    # eq. momentum: a_i = -m (P_i/rho_i^2 + P_j/rho_j^2) W'(r) (s_i - s_j)/r
    p = _params()
    r, s, g, rho_i, rho_j, dW = _pair_setup(q)
    out = _rhs(p, s, np.zeros((2, 2)), g, use_cells)
    assert out["rho"] == pytest.approx([rho_i, rho_j], rel=1e-13)
    Pi, Pj = p.k_lin * (rho_i - p.rho0), p.k_lin * (rho_j - p.rho0)
    assert out["P"] == pytest.approx([Pi, Pj], rel=1e-12)
    mag = M * (Pi / rho_i**2 + Pj / rho_j**2) * dW       # negative: W' < 0
    # s_i - s_j = (-r, 0): i is pushed towards -x, j towards +x
    expect = np.array([[mag, 0.0], [-mag, 0.0]])
    assert np.abs(out["a_sph"] - expect).max() <= 1e-12 * abs(mag)
    assert out["a_sph"][0, 0] < 0 < out["a_sph"][1, 0]


@pytest.mark.parametrize("q", [0.5, 1.5])
@pytest.mark.parametrize("v", [0.7, -0.7])
def test_fluid_pair_viscous_force_value(q, v):
    # eq. viscous, added to the pressure term with no min(., 0):
    # pi_ij = m 2 alpha h/(rho_i + rho_j) (w_ij . s_ij)/(r^2 + eps h^2),
    # a_i += pi_ij W'(r) (s_i - s_j)/r.  i moves along +x at v (towards j for
    # v > 0, away for v < 0); j rests.
    alpha = 0.4
    r, s, g, rho_i, rho_j, dW = _pair_setup(q)
    w = [[v, 0.0], [0.0, 0.0]]
    p1 = _params(alpha=alpha)
    p0 = _params(alpha=0.0)
    a1 = _rhs(p1, s, w, g)["a_sph"]
    a0 = _rhs(p0, s, w, g)["a_sph"]
    dv = a1 - a0
    wij_sij = v * (-r)
    pi = M * 2.0 * alpha * H / (rho_i + rho_j) * wij_sij / (r * r + p1.eps * H * H)
    expect_i = pi * dW * (-1.0)          # grad_i W = W'(r) (-1, 0)
    assert dv[0, 0] == pytest.approx(expect_i, rel=1e-11)
    assert dv[1, 0] == pytest.approx(-expect_i, rel=1e-11)
    assert np.abs(dv[:, 1]).max() == 0.0
    # the force opposes the relative motion either way (approaching or receding)
    assert dv[0, 0] * v < 0


# --- one fluid particle above one ghost: ghost at (X0, 0), particle at
# (X0, h/2), so r = h/2 = hs/2 with hs = h; rho_i = m (W(0) + gamma1 W(h/2)).

X0 = 0.3


def _wall_setup(gamma1=1.0):
    s = [[X0, 0.5 * H]]
    g = [[X0, 0.0]]
    rho = M * C * (4.0 + gamma1 * 23.0 / 8.0)
    dWs = -7.5 / (math.pi * H**3)        # W_s3'(hs/2)
    return s, g, rho, dWs


@pytest.mark.parametrize("gamma1", [1.0, 0.5])
def test_wall_pressure_force_value_and_reaction(gamma1):
    # eq. pressure_b2f with the ghost inheriting P and rho (reading R3):
    # F = -2 m^2 (P_i/rho_i^2) W_s3'(r) (s_i - g)/r on the fluid,
    # and the tank takes -F at the ghost (eqs. pressure_f2b, tankdynamics).
    p = _params(gamma1=gamma1)
    s, g, rho, dWs = _wall_setup(gamma1)
    out = _rhs(p, s, np.zeros((1, 2)), g)
    assert out["rho"][0] == pytest.approx(rho, rel=1e-13)
    P = p.k_lin * (rho - p.rho0)
    Fy = -2.0 * M * M * P / rho**2 * dWs          # = 15 m^2 P/(pi h^3 rho^2) > 0
    assert Fy == pytest.approx(15.0 * M * M * P / (math.pi * H**3 * rho**2), rel=1e-14)
    a = out["a_sph"][0]
    assert a[0] == 0.0
    assert a[1] == pytest.approx(Fy / M, rel=1e-12)
    wr = out["wrench"]
    assert wr[0] == 0.0
    assert wr[1] == pytest.approx(-Fy, rel=1e-12)
    # torque of the reaction -F at the ghost about the body origin: -(X0 F_y)
    assert wr[2] == pytest.approx(-X0 * Fy, rel=1e-12)


@pytest.mark.parametrize("v", [0.5, -0.5])
def test_wall_viscous_force_value(v):
    # eq. viscous_b2f with rho_g = rho_i: F = m^2 (2 beta/(2 rho_i))
    # min(w_i . s_ik, 0)/(r^2 + eps h^2) W_s3'(r) (s_i - g)/r.
    # v > 0: the particle moves down, into the wall; v < 0: away from it.
    beta = 0.2
    s, g, rho, dWs = _wall_setup()
    w = [[0.0, -v]]
    a1 = _rhs(_params(beta=beta), s, w, g)
    a0 = _rhs(_params(beta=0.0), s, w, g)
    dF = M * (a1["a_sph"][0] - a0["a_sph"][0])
    dwrench = a1["wrench"] - a0["wrench"]
    r = 0.5 * H
    vr = min(-v * r, 0.0)
    Fy = M * M * (2.0 * beta / (2.0 * rho)) * vr / (r * r + 0.01 * H * H) * dWs
    if v > 0:
        # = m^2 (beta/rho) (v h/2)/(h^2 (1/4 + eps)) (7.5/(pi h^3)) > 0: pushes back
        assert Fy == pytest.approx(M * M * beta / rho * 0.5 * v * H / (H * H * 0.26)
                                   * 7.5 / (math.pi * H**3), rel=1e-14)
        assert Fy > 0
        assert dF[1] == pytest.approx(Fy, rel=1e-11)
        assert dwrench[1] == pytest.approx(-Fy, rel=1e-11)
        assert dwrench[2] == pytest.approx(-X0 * Fy, rel=1e-11)
    else:
        assert np.abs(dF).max() == 0.0 and np.abs(dwrench).max() == 0.0
    assert dF[0] == 0.0


def test_wall_pressure_is_twice_the_one_sided_fluid_term():
    # the fluid-fluid pressure term of eq. momentum with the partner inheriting
    # the particle's own P and rho is -2 m (P_i/rho_i^2) grad W, which is what
    # eq. pressure_b2f applies with the spiky kernel: at the same radius the
    # two accelerations differ by exactly W_s3'/W_cb' of the radius.
    p = _params()
    s, g, rho, dWs = _wall_setup()
    a_wall = _rhs(p, s, np.zeros((1, 2)), g)["a_sph"][0, 1]
    P = p.k_lin * (rho - p.rho0)
    dWc = -15.0 / 4.0 * C / H                     # W_cb'(h/2)
    one_sided = -M * (P / rho**2 + P / rho**2) * dWc
    assert a_wall == pytest.approx(one_sided * dWs / dWc, rel=1e-12)


# --- the variational identity of the symmetric pressure force


def _cloud(seed=11, n_side=9):
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(n_side), np.arange(n_side))
    s = np.stack([i.ravel() * DX, j.ravel() * DX], 1)
    s = s * rng.uniform(0.85, 0.95) + rng.uniform(-0.25 * DX, 0.25 * DX, s.shape)
    w = rng.normal(0.0, 0.3, s.shape)
    return s, w


@pytest.mark.parametrize("eos", [W.EOS_LINEAR, W.EOS_TAIT])
def test_pressure_power_equals_internal_energy_rate(eos):
    # summation density rho_i = m sum_j W_ij gives d rho_i/dt = m sum_j w_ij . grad_i W_ij;
    # with the symmetric form of eq. momentum,
    #   sum_i m w_i . a_i = -sum_i m (P_i/rho_i^2) d rho_i/dt   (exactly).
    s, w = _cloud()
    p = _params()
    p.eos = eos
    if eos == W.EOS_TAIT:
        p.rho0 = 900.0
    g = np.zeros((0, 2))
    base = _rhs(p, s, w, g)
    lhs = M * (w * base["a_sph"]).sum()
    # central differences at eps and eps/2 combined by Richardson's rule
    # (truncation O(eps^4))
    def drho(eps):
        rp = _rhs(p, s + eps * w, w, g)["rho"]
        rm = _rhs(p, s - eps * w, w, g)["rho"]
        return (rp - rm) / (2.0 * eps)
    eps = 1e-5
    d = (4.0 * drho(eps / 2) - drho(eps)) / 3.0
    terms = M * base["P"] / base["rho"] ** 2 * d
    rhs = -terms.sum()
    assert abs(lhs) > 1e-6 * np.abs(terms).sum()
    assert abs(lhs - rhs) <= 1e-9 * np.abs(terms).sum()
    assert lhs == pytest.approx(rhs, rel=1e-7)
