"""Pins of the oracle's kernels and equation of state against closed forms.

The cubic spline (eq. cubicspline) and spiky kernel (eq. spiky3) must be
normalised in 2D (eq. normkernel); the cubic spline's value at the origin is
the textbook M4 constant 10/(7 pi h^2); dW/dr must be the derivative of W;
the Tait pressure must vanish at rest density with dP/drho = c0^2 there.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import sph as O

H = 0.01625


def _quad_2d(f, a, b, points=None):
    val, _ = integrate.quad(lambda r: f(r) * 2.0 * math.pi * r, a, b, points=points, limit=400,
                            epsabs=1e-14, epsrel=1e-13)
    return val


@pytest.mark.parametrize("h", [0.004, 0.01625, 0.3])
def test_cubic_spline_normalised(h):
    L = O.lib()
    assert _quad_2d(lambda r: L.ora_w_cubic(r, h, 0), 0.0, 2 * h, points=[h]) == pytest.approx(1.0, abs=1e-10)


def test_cubic_spline_printed_constant_integrates_to_three():
    L = O.lib()
    assert _quad_2d(lambda r: L.ora_w_cubic(r, H, 1), 0.0, 2 * H, points=[H]) == pytest.approx(3.0, abs=1e-9)


@pytest.mark.parametrize("hs", [0.0052, 0.01625])
def test_spiky_normalised(hs):
    L = O.lib()
    assert _quad_2d(lambda r: L.ora_w_spiky(r, hs), 0.0, hs) == pytest.approx(1.0, abs=1e-10)


def test_cubic_value_at_origin_is_textbook_m4_constant():
    # Monaghan's M4 spline in 2D: W(0) = sigma * 1 with sigma = 10 / (7 pi h^2)
    assert O.lib().ora_w_cubic(0.0, H, 0) == pytest.approx(10.0 / (7.0 * math.pi * H * H), rel=1e-14)


def test_kernels_vanish_outside_support():
    L = O.lib()
    for r in (2 * H, 2 * H * (1 + 1e-12), 3 * H):
        assert L.ora_w_cubic(r, H, 0) == 0.0
        assert L.ora_dw_cubic(r, H, 0) == 0.0
    assert L.ora_w_spiky(H, H) == 0.0
    assert L.ora_dw_spiky(1.5 * H, H) == 0.0


@pytest.mark.parametrize("q", [0.05, 0.3, 0.77, 0.999, 1.001, 1.4, 1.9, 1.999])
def test_cubic_gradient_is_derivative(q):
    L = O.lib()
    r, e = q * H, 1e-7 * H
    fd = (L.ora_w_cubic(r + e, H, 0) - L.ora_w_cubic(r - e, H, 0)) / (2 * e)
    an = L.ora_dw_cubic(r, H, 0)
    assert an == pytest.approx(fd, rel=2e-6, abs=1e-9 * abs(L.ora_w_cubic(0, H, 0)) / H)


@pytest.mark.parametrize("x", [0.01, 0.2, 0.5, 0.9, 0.99])
def test_spiky_gradient_is_derivative(x):
    L = O.lib()
    r, e = x * H, 1e-7 * H
    fd = (L.ora_w_spiky(r + e, H) - L.ora_w_spiky(r - e, H)) / (2 * e)
    assert L.ora_dw_spiky(r, H) == pytest.approx(fd, rel=2e-6)


def test_cubic_continuity_at_breakpoints():
    L = O.lib()
    for q in (1.0, 2.0):
        lo, hi = (q - 1e-12) * H, (q + 1e-12) * H
        w0 = L.ora_w_cubic(0.0, H, 0)
        assert abs(L.ora_w_cubic(lo, H, 0) - L.ora_w_cubic(hi, H, 0)) < 1e-9 * w0
        assert abs(L.ora_dw_cubic(lo, H, 0) - L.ora_dw_cubic(hi, H, 0)) < 1e-8 * w0 / H
    # zero slope at the origin: the spline's gradient vanishes at r = 0
    assert abs(L.ora_dw_cubic(0.0, H, 0)) < 1e-12 * L.ora_w_cubic(0.0, H, 0) / H


def test_tait_eos_rest_and_sound_speed():
    import workloads as W
    p = W.plain_rect().params
    assert O.eos(p, p.rho0) == pytest.approx(0.0, abs=1e-9)
    d = 1e-6 * p.rho0
    slope = (O.eos(p, p.rho0 + d) - O.eos(p, p.rho0 - d)) / (2 * d)
    assert slope == pytest.approx(p.c0 ** 2, rel=1e-8)      # c^2 = dP/drho at rest
    # stiffness exponent: P + B = B (rho/rho0)^gamma
    B = p.rho0 * p.c0 ** 2 / p.tait_gamma
    assert (O.eos(p, 2 * p.rho0) + B) / B == pytest.approx(2.0 ** p.tait_gamma, rel=1e-12)


def test_linear_eos_of_the_paper():
    import workloads as W
    p = W.paper_p0(eos=W.EOS_LINEAR).params
    assert O.eos(p, p.rho0) == 0.0
    assert O.eos(p, p.rho0 + 10.0) == pytest.approx(p.k_lin * 10.0, rel=1e-12)
    assert O.eos(p, p.rho0 - 5.0) == pytest.approx(-p.k_lin * 5.0, rel=1e-12)


def test_clamped_linear_eos_has_no_tension():
    import workloads as W
    p = W.paper_p0().params
    assert p.eos == W.EOS_LINEAR_CLAMPED
    assert O.eos(p, p.rho0 + 10.0) == pytest.approx(p.k_lin * 10.0, rel=1e-12)
    assert O.eos(p, p.rho0 - 5.0) == 0.0
    assert O.eos(p, p.rho0) == 0.0


def test_clamped_tait_eos_has_no_tension():
    import workloads as W
    p = W.random_tank(0, n_steps=1, eos=W.EOS_TAIT_CLAMPED).params
    lit = W.random_tank(0, n_steps=1).params
    assert O.eos(p, 1.01 * p.rho0) == pytest.approx(O.eos(lit, 1.01 * lit.rho0), rel=1e-15)
    assert O.eos(lit, 0.99 * lit.rho0) < 0.0
    assert O.eos(p, 0.99 * p.rho0) == 0.0
