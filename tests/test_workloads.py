"""The workload generators reproduce the paper's parameter tables and the
measured configurations' sizes (inputs only; no method arithmetic here)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def test_paper_p0_matches_tables_1_and_2():
    g = json.load(open(GOLD))
    sc = W.paper_p0(n_steps=10)
    p = sc.params
    assert p.body_mass == g["satellite"]["mass_kg"]
    assert p.body_inertia == g["satellite"]["inertia_kg_m2"]
    assert p.h == pytest.approx(g["fluid"]["h_mm"] * 1e-3)
    assert p.k_lin == g["fluid"]["k_stiffness"] and p.rho0 == g["fluid"]["rho0"]
    assert p.visc_alpha == g["fluid"]["alpha"] and p.visc_beta == g["fluid"]["beta"]
    assert p.gamma1 == g["fluid"]["gamma1"]
    assert p.mass == pytest.approx(p.rho0 * (g["fluid"]["particle_length_mm"] * 1e-3) ** 2)
    assert p.dt == g["time"]["dynamics_dt_s"]
    assert p.ctrl_period * p.dt == pytest.approx(g["time"]["control_dt_s"])
    w, xi = g["controller"]["omega_rad_s"], g["controller"]["xi"]
    assert p.kp == pytest.approx(p.body_inertia * w * w) and p.kd == pytest.approx(2 * xi * p.body_inertia * w)
    assert sc.n_ghost == g["fluid"]["n_ghost"]
    assert sc.n_fluid == pytest.approx(g["fluid"]["n_fluid"], rel=0.06)
    rnd = W.paper_p0(n_steps=10, spawn="random")
    assert rnd.n_fluid == g["fluid"]["n_fluid"]
    r = np.sqrt((rnd.pos.astype(np.float64) ** 2).sum(1))
    assert r.max() < 0.2 and rnd.pos[:, 1].max() < W.circle_fill_level(0.2, 0.6)
    d = np.sqrt(((rnd.pos[:, None, :].astype(np.float64) - rnd.pos[None, :, :]) ** 2).sum(-1))
    assert d[np.triu_indices(rnd.n_fluid, 1)].min() >= 0.6 * rnd.dx * (1 - 1e-6)


def test_plain_rect_sizes():
    sc = W.plain_rect(0)
    assert sc.n_fluid == 1600 and sc.n_ghost == 756
    assert sc.params.dt == pytest.approx(0.2 * 1.3 * 0.0125 / 20.0)
    d = sc.pos - W.plain_rect(0, n_steps=1).pos
    assert np.all(d == 0)                           # seeded
    assert not np.array_equal(sc.pos, W.plain_rect(1).pos)
    lat = np.round((sc.pos + [0.5, 0.25]) / 0.0125 - 0.5)
    assert np.abs((sc.pos + [0.5, 0.25]) / 0.0125 - 0.5 - lat).max() <= 0.0100001


def test_closed_loop_circle_sizes():
    sc = W.closed_loop_circle(0, n_steps=100)
    assert 14400 < sc.n_fluid < 14800 and sc.n_ghost == 2385
    area = sc.n_fluid * sc.dx ** 2
    assert area / (math.pi * 0.25) == pytest.approx(0.3, rel=0.02)  # lattice stops dx/2 inside the wall
    assert sc.params.ctrl_period == 962
    assert sc.theta_ref[-1] <= math.radians(30) + 1e-12


def test_trapezoid_slew_profile():
    t = np.linspace(0, 2, 2001)
    th = W.trapezoid_slew(math.radians(30), 0.25, 0.5, t)
    rate = np.gradient(th, t)
    assert th[-1] == pytest.approx(math.radians(30))
    assert rate.max() == pytest.approx(math.radians(30) / 0.75, rel=1e-2)
    assert np.all(np.diff(th) >= -1e-15)


def test_multisine_tones_on_the_grid():
    rng = np.random.default_rng(0)
    t = np.arange(0, 200, 0.01)
    u = W.multisine(rng, 5, 10.0, t)
    spec = np.abs(np.fft.rfft(u))
    f = np.fft.rfftfreq(t.size, 0.01)
    top = np.sort(f[np.argsort(spec)[-5:]])
    assert np.allclose(np.round(top / 0.05) * 0.05, top, atol=1e-9)
    assert np.abs(u).max() <= 10.0 + 1e-12
