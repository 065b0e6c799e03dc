"""Seeded synthetic workloads for the sloshing step.

This module builds the *inputs* of a run -- tank geometry, initial particle
lattice with its jitter, boundary particles, scenario constants and the input
signals -- and nothing of the method itself: no kernel, density, force or
integrator arithmetic lives here.  Both the HIP path and the FP64 oracle take
their inputs from these generators, so the two sides always start from the
same FP32-representable arrays.

Scenario constants follow the paper's benchmark (Section 5.1, Tables 1-2) and
the workloads the implementation is measured on:

* ``plain_rect``  -- rectangular 1.0 x 0.5 m tank, 50 % fill, dx = 12.5 mm,
  3 boundary layers, Tait EOS (gamma 7, c0 = 20 m/s), prescribed sinusoidal
  rotation 0.1 rad at 0.5 Hz, dt from CFL 0.2, 2,000 steps.
* ``closed_loop_circle`` -- circular tank R = 0.5 m, 30 % fill, dx = 4 mm,
  spacecraft m = 1000 kg, J = 500 kg m^2, PD attitude controller (Section 5.1,
  control law with K = [J w^2, 2 xi J w], w = 0.2 pi, xi = 0.7, zero-order
  hold at 0.05 s) tracking a 30-degree trapezoidal-rate slew, 20,000 steps.
* ``random_tank`` -- rectangular or circular tank, fill in [0.2, 0.8], 2k-60k
  particles, torque a 5-tone random-phase multisine on the 0.05 Hz grid of the
  paper's identification signal (Section 5.3).
* ``paper_p0`` -- the paper's own benchmark parameters (Tables 1-2), used for
  timing context only.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

EOS_TAIT, EOS_LINEAR, EOS_LINEAR_CLAMPED, EOS_TAIT_CLAMPED = 0, 1, 2, 3
MOTION_FREE, MOTION_SINE = 0, 1
CTRL_NONE, CTRL_PD_ZOH = 0, 1
KNORM_UNIT, KNORM_PRINTED = 0, 1


@dataclasses.dataclass
class Params:
    """Scenario constants; field meanings mirror the C-ABI ``sph_params``."""
    eos: int = EOS_TAIT
    motion: int = MOTION_FREE
    ctrl: int = CTRL_NONE
    kernel_norm: int = KNORM_UNIT
    h: float = 0.0
    h_spiky: float = 0.0
    rho0: float = 1000.0
    mass: float = 0.0
    c0: float = 20.0
    tait_gamma: float = 7.0
    k_lin: float = 3.0
    visc_alpha: float = 0.4
    visc_beta: float = 0.1923
    eps: float = 0.01
    gamma1: float = 1.0
    dt: float = 0.0
    body_mass: float = 1000.0
    body_inertia: float = 500.0
    kp: float = 0.0
    kd: float = 0.0
    ctrl_period: int = 1
    sine_amp: float = 0.0
    sine_freq: float = 0.0
    domain_min: tuple = (0.0, 0.0)
    domain_max: tuple = (0.0, 0.0)


@dataclasses.dataclass
class Scenario:
    name: str
    params: Params
    pos: np.ndarray            # [N, 2] float32, body frame
    vel: np.ndarray            # [N, 2] float32, body frame
    ghosts: np.ndarray         # [G, 2] float32, body frame (static)
    rigid0: np.ndarray         # [6] float64: r_x, r_y, theta, rdot_x, rdot_y, thetadot
    n_steps: int
    u_seq: np.ndarray          # [n_steps, 3] float32: F_x, F_y (world), torque
    theta_ref: Optional[np.ndarray] = None   # [n_ctrl] float64, reference at control instants
    dx: float = 0.0
    fill: float = 0.0
    shape: str = "rect"
    tank_size: float = 1.0     # characteristic length (rect width, circle diameter)

    @property
    def n_fluid(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_ghost(self) -> int:
        return int(self.ghosts.shape[0])


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def _jitter(rng: np.random.Generator, n: int, amp: float) -> np.ndarray:
    return rng.uniform(-amp, amp, size=(n, 2))


def rect_tank(width: float, height: float, dx: float, fill_rows: int, layers: int,
              rng: Optional[np.random.Generator], jitter: float):
    """Fluid on the half-offset lattice ((i+1/2)dx - W/2, (j+1/2)dx - H/2) for the
    bottom ``fill_rows`` rows; ``layers`` rows of fixed boundary particles on the
    same lattice outside the interior."""
    ncx = int(round(width / dx))
    ncy = int(round(height / dx))
    i = np.arange(ncx)
    j = np.arange(fill_rows)
    ii, jj = np.meshgrid(i, j, indexing="xy")
    fx = (ii.ravel() + 0.5) * dx - width / 2
    fy = (jj.ravel() + 0.5) * dx - height / 2
    fluid = np.stack([fx, fy], axis=1)
    if rng is not None and jitter > 0:
        fluid = fluid + _jitter(rng, fluid.shape[0], jitter * dx)
    bi = np.arange(-layers, ncx + layers)
    bj = np.arange(-layers, ncy + layers)
    bii, bjj = np.meshgrid(bi, bj, indexing="xy")
    bii = bii.ravel(); bjj = bjj.ravel()
    outside = (bii < 0) | (bii >= ncx) | (bjj < 0) | (bjj >= ncy)
    gx = (bii[outside] + 0.5) * dx - width / 2
    gy = (bjj[outside] + 0.5) * dx - height / 2
    ghosts = np.stack([gx, gy], axis=1)
    return fluid, ghosts


def circle_fill_level(radius: float, fill: float) -> float:
    """Height y_f such that the disk area below y = y_f is ``fill`` of the disk."""
    lo, hi = -radius, radius
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        t = math.acos(max(-1.0, min(1.0, -mid / radius)))
        frac = (t - math.sin(t) * math.cos(t)) / math.pi
        if frac < fill:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def circle_tank(radius: float, dx: float, fill: float, rings: int,
                rng: Optional[np.random.Generator], jitter: float):
    """Fluid: half-offset lattice points inside radius - dx/2 and below the fill
    level.  Boundary: ``rings`` rings at radius + (k+1/2) dx, each with
    round(2 pi r_k / dx) evenly spaced particles, alternate rings staggered."""
    yf = circle_fill_level(radius, fill)
    n = int(math.ceil(radius / dx)) + 1
    idx = np.arange(-n, n)
    ii, jj = np.meshgrid(idx, idx, indexing="xy")
    px = (ii.ravel() + 0.5) * dx
    py = (jj.ravel() + 0.5) * dx
    keep = (px * px + py * py < (radius - 0.5 * dx) ** 2) & (py < yf)
    fluid = np.stack([px[keep], py[keep]], axis=1)
    order = np.lexsort((fluid[:, 0], fluid[:, 1]))
    fluid = fluid[order]
    if rng is not None and jitter > 0:
        fluid = fluid + _jitter(rng, fluid.shape[0], jitter * dx)
    gs = []
    for k in range(rings):
        rk = radius + (k + 0.5) * dx
        nk = int(round(2 * math.pi * rk / dx))
        phi = 2 * math.pi * (np.arange(nk) + 0.5 * (k % 2)) / nk
        gs.append(np.stack([rk * np.cos(phi), rk * np.sin(phi)], axis=1))
    ghosts = np.concatenate(gs, axis=0)
    return fluid, ghosts


# ----------------------------------------------------------------------------
# input signals
# ----------------------------------------------------------------------------

def trapezoid_slew(theta_final: float, t_ramp: float, t_coast: float, times: np.ndarray) -> np.ndarray:
    """Angle reference with a trapezoidal rate profile: accelerate for t_ramp,
    coast for t_coast, decelerate for t_ramp, then hold theta_final."""
    peak = theta_final / (t_ramp + t_coast)
    t = np.asarray(times, dtype=np.float64)
    out = np.empty_like(t)
    t1, t2, t3 = t_ramp, t_ramp + t_coast, 2 * t_ramp + t_coast
    a = peak / t_ramp
    m0 = t <= 0
    m1 = (t > 0) & (t <= t1)
    m2 = (t > t1) & (t <= t2)
    m3 = (t > t2) & (t <= t3)
    m4 = t > t3
    out[m0] = 0.0
    out[m1] = 0.5 * a * t[m1] ** 2
    th1 = 0.5 * a * t1 ** 2
    out[m2] = th1 + peak * (t[m2] - t1)
    th2 = th1 + peak * t_coast
    tau = t[m3] - t2
    out[m3] = th2 + peak * tau - 0.5 * a * tau ** 2
    out[m4] = theta_final
    return out


def multisine(rng: np.random.Generator, n_tones: int, amp: float, times: np.ndarray,
              grid_hz: float = 0.05, f_max_hz: float = 2.0) -> np.ndarray:
    """Random-phase multisine: amp/n_tones * sum_q sin(2 pi f_q t + phi_q), f_q
    drawn without replacement from {grid, 2 grid, ..., f_max}."""
    grid = np.arange(1, int(round(f_max_hz / grid_hz)) + 1) * grid_hz
    f = rng.choice(grid, size=n_tones, replace=False)
    phi = rng.uniform(0.0, 2 * math.pi, size=n_tones)
    t = np.asarray(times, dtype=np.float64)[:, None]
    return (amp / n_tones) * np.sin(2 * math.pi * f[None, :] * t + phi[None, :]).sum(axis=1)


# ----------------------------------------------------------------------------
# scenarios
# ----------------------------------------------------------------------------

def _fluid_params(dx: float, h_ratio: float = 1.3, rho0: float = 1000.0, c0: float = 20.0,
                  alpha: float = 0.02) -> Params:
    h = h_ratio * dx
    visc_alpha = alpha * c0                # Monaghan's alpha * c0 convention
    return Params(eos=EOS_TAIT, h=h, h_spiky=h, rho0=rho0, mass=rho0 * dx * dx, c0=c0,
                  tait_gamma=7.0, visc_alpha=visc_alpha,
                  visc_beta=visc_alpha * (4e-4 / 8.32e-4),  # wall/fluid ratio of Table 2
                  eps=0.01, gamma1=1.0, dt=0.2 * h / c0)


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def plain_rect(seed: int = 0, n_steps: int = 2000, dx: float = 0.0125) -> Scenario:
    """Rectangular 1.0 x 0.5 m tank, 50 % fill, prescribed sine rotation."""
    rng = np.random.default_rng(seed)
    W, H = 1.0, 0.5
    fill_rows = int(round(0.5 * H / dx))
    fluid, ghosts = rect_tank(W, H, dx, fill_rows, 3, rng, 0.01)
    p = _fluid_params(dx)
    p.motion = MOTION_SINE
    p.sine_amp, p.sine_freq = 0.1, 0.5
    pad = 4 * dx
    p.domain_min = (-W / 2 - pad, -H / 2 - pad)
    p.domain_max = (W / 2 + pad, H / 2 + pad)
    w0 = 2 * math.pi * p.sine_freq * p.sine_amp
    rigid0 = np.array([0.0, 0.0, 0.0, 0.0, 0.0, w0])
    return Scenario("plain_rect", p, _f32(fluid), np.zeros((fluid.shape[0], 2), np.float32),
                    _f32(ghosts), rigid0, n_steps, np.zeros((n_steps, 3), np.float32),
                    dx=dx, fill=0.5, shape="rect", tank_size=W)


def closed_loop_circle(seed: int = 0, n_steps: int = 20000, dx: float = 0.004,
                       fill: float = 0.3) -> Scenario:
    """Circular R = 0.5 m tank, PD attitude control through a 30-degree slew."""
    rng = np.random.default_rng(seed)
    R = 0.5
    fluid, ghosts = circle_tank(R, dx, fill, 3, rng, 0.01)
    p = _fluid_params(dx)
    p.motion = MOTION_FREE
    p.ctrl = CTRL_PD_ZOH
    p.body_mass, p.body_inertia = 1000.0, 500.0
    w, xi = 0.2 * math.pi, 0.7
    p.kp = p.body_inertia * w * w
    p.kd = 2 * xi * p.body_inertia * w
    p.ctrl_period = max(1, int(round(0.05 / p.dt)))
    pad = 5 * dx
    p.domain_min = (-R - pad, -R - pad)
    p.domain_max = (R + pad, R + pad)
    n_ctrl = (n_steps + p.ctrl_period - 1) // p.ctrl_period + 1
    t_ctrl = np.arange(n_ctrl) * p.ctrl_period * p.dt
    theta_ref = trapezoid_slew(math.radians(30.0), 0.25, 0.5, t_ctrl)
    return Scenario("closed_loop_circle", p, _f32(fluid), np.zeros((fluid.shape[0], 2), np.float32),
                    _f32(ghosts), np.zeros(6), n_steps, np.zeros((n_steps, 3), np.float32),
                    theta_ref=theta_ref, dx=dx, fill=fill, shape="circle", tank_size=2 * R)


def random_tank(seed: int, n_steps: int = 5000, n_min: int = 2000, n_max: int = 60000,
                shape: Optional[str] = None, eos: int = EOS_TAIT, jitter_seed: Optional[int] = None) -> Scenario:
    """Random tank for the surrogate data set: rectangle 1.0 x 0.5 or circle
    R = 0.5 (equal odds), fill U[0.2, 0.8], particle count U{n_min..n_max},
    torque a 5-tone multisine with amplitude U[0, 50] N m.  eos: EOS_TAIT
    (the measured batch configuration) or EOS_TAIT_CLAMPED.  jitter_seed:
    if given, the lattice jitter comes from its own generator, so that tanks
    of one seed and different jitter seeds share shape, size, fill and input
    and differ only in the initial jitter."""
    rng = np.random.default_rng(seed)
    jrng = rng if jitter_seed is None else np.random.default_rng([int(seed), int(jitter_seed)])
    if shape is None:
        shape = "rect" if rng.random() < 0.5 else "circle"
    fill = float(rng.uniform(0.2, 0.8))
    n_target = int(rng.integers(n_min, n_max + 1))
    if shape == "rect":
        W, H = 1.0, 0.5
        dx = math.sqrt(fill * W * H / n_target)
        dx = W / round(W / dx)            # whole number of columns
        ncy = int(round(H / dx))
        fill_rows = max(1, int(round(fill * ncy)))
        fluid, ghosts = rect_tank(W, H, dx, fill_rows, 3, jrng, 0.01)
        ext = (W / 2, H / 2)
        size = W
    else:
        R = 0.5
        dx = math.sqrt(fill * math.pi * R * R / n_target)
        fluid, ghosts = circle_tank(R, dx, fill, 3, jrng, 0.01)
        ext = (R, R)
        size = 2 * R
    p = _fluid_params(dx)
    p.eos = eos
    p.motion = MOTION_FREE
    p.ctrl = CTRL_NONE
    p.body_mass, p.body_inertia = 1000.0, 500.0
    pad = 5 * dx
    p.domain_min = (-ext[0] - pad, -ext[1] - pad)
    p.domain_max = (ext[0] + pad, ext[1] + pad)
    amp = float(rng.uniform(0.0, 50.0))
    t = np.arange(n_steps) * p.dt
    u = np.zeros((n_steps, 3), np.float64)
    u[:, 2] = multisine(rng, 5, amp, t)
    return Scenario("random_tank", p, _f32(fluid), np.zeros((fluid.shape[0], 2), np.float32),
                    _f32(ghosts), np.zeros(6), n_steps, _f32(u), dx=dx, fill=fill,
                    shape=shape, tank_size=size)


def linearization_tank(seed: int = 0, n_steps: int = 400, n_fluid: int = 8000) -> Scenario:
    """Rectangular 1.0 x 0.5 m tank, 50 % fill, about n_fluid particles, free
    spacecraft (m = 1000 kg, J = 500 kg m^2) under a 5-tone multisine torque
    of amplitude 20 N m: the workload of the linearization measurements."""
    rng = np.random.default_rng(seed)
    W_, H = 1.0, 0.5
    dx = math.sqrt(0.5 * W_ * H / n_fluid)
    dx = W_ / round(W_ / dx)
    fill_rows = max(1, int(round(0.5 * H / dx)))
    fluid, ghosts = rect_tank(W_, H, dx, fill_rows, 3, rng, 0.01)
    p = _fluid_params(dx)
    p.motion = MOTION_FREE
    p.ctrl = CTRL_NONE
    p.body_mass, p.body_inertia = 1000.0, 500.0
    pad = 5 * dx
    p.domain_min = (-W_ / 2 - pad, -H / 2 - pad)
    p.domain_max = (W_ / 2 + pad, H / 2 + pad)
    t = np.arange(n_steps) * p.dt
    u = np.zeros((n_steps, 3), np.float64)
    u[:, 2] = multisine(rng, 5, 20.0, t)
    return Scenario("linearization_tank", p, _f32(fluid), np.zeros((fluid.shape[0], 2), np.float32),
                    _f32(ghosts), np.zeros(6), n_steps, _f32(u), dx=dx, fill=0.5, shape="rect", tank_size=W_)


def rect_sweep(k: int, seed: int = 0, n_steps: int = 200) -> Scenario:
    """The rectangular workload refined by 2^k in spacing (N = 1600 * 4^k)."""
    return plain_rect(seed=seed, n_steps=n_steps, dx=0.0125 / (2 ** k))


def _random_fill(rng: np.random.Generator, radius: float, fill: float, n: int, min_dist: float):
    """n points drawn uniformly from the part of the disk r < radius below the
    fill level, each at least min_dist from the earlier ones (dart throwing)."""
    yf = circle_fill_level(radius, fill)
    pts = np.zeros((0, 2))
    tries = 0
    while pts.shape[0] < n:
        tries += 1
        if tries > 200 * n:
            raise RuntimeError("random fill: no room for the requested particles")
        q = rng.uniform(-radius, radius, size=2)
        if q[0] * q[0] + q[1] * q[1] >= radius * radius or q[1] >= yf:
            continue
        if pts.shape[0] and np.min(((pts - q) ** 2).sum(1)) < min_dist * min_dist:
            continue
        pts = np.vstack([pts, q])
    return pts


def paper_p0(seed: int = 0, n_steps: int = 30000, spawn: str = "lattice", eos: int = EOS_LINEAR_CLAMPED) -> Scenario:
    """The paper's benchmark (Tables 1-2): circular tank r = 0.2 m, 60 % fill,
    6 mm particles, one ring of 236 ghosts (5.4 mm), h = 9.42 mm, linear EOS
    k = 3, rho0 = 1017, alpha = 8.32e-4, beta = 4e-4, gamma1 = 0.5,
    dt = 1 ms, PD attitude law at 0.05 s.  spawn="random" places the paper's
    666 particles at random in the filled region (at least 0.6 of the mean
    spacing apart), the initial condition the paper relaxes to rest before
    its runs (Section 5.1); spawn="lattice" uses a jittered lattice.  eos:
    EOS_LINEAR_CLAMPED by default (the linear law without tension: with
    negative pressures the zero-gravity fluid is unstable in this model),
    EOS_LINEAR for the literal law."""
    rng = np.random.default_rng(seed)
    # 666 particles of mass rho0 (6 mm)^2 at 60 % fill sit on a ~10.6 mm
    # lattice; with the kernel constant as printed this is close to rest density.
    R, d_part = 0.2, 0.006
    dx = 0.0106
    if spawn == "random":
        fluid = _random_fill(rng, R - 0.5 * dx, 0.6, 666, 0.6 * dx)
    elif spawn == "lattice":
        fluid, _ = circle_tank(R, dx, 0.6, 1, rng, 0.01)
    else:
        raise ValueError("spawn must be 'lattice' or 'random'")
    ng = 236
    phi = 2 * math.pi * np.arange(ng) / ng
    ghosts = np.stack([R * np.cos(phi), R * np.sin(phi)], axis=1)
    p = Params(eos=eos, kernel_norm=KNORM_PRINTED, h=0.00942, h_spiky=0.00942, rho0=1017.0,
               mass=1017.0 * d_part * d_part, c0=math.sqrt(3.0), tait_gamma=7.0, k_lin=3.0,
               visc_alpha=8.32e-4, visc_beta=4e-4, eps=0.01, gamma1=0.5, dt=1e-3,
               body_mass=1010.71, body_inertia=133.84, motion=MOTION_FREE, ctrl=CTRL_PD_ZOH)
    w, xi = 0.2 * math.pi, 0.7
    p.kp = p.body_inertia * w * w
    p.kd = 2 * xi * p.body_inertia * w
    p.ctrl_period = 50
    pad = 0.03
    p.domain_min = (-R - pad, -R - pad)
    p.domain_max = (R + pad, R + pad)
    n_ctrl = n_steps // p.ctrl_period + 2
    theta_ref = np.zeros(n_ctrl)
    return Scenario("paper_p0", p, _f32(fluid), np.zeros((fluid.shape[0], 2), np.float32),
                    _f32(ghosts), np.zeros(6), n_steps, np.zeros((n_steps, 3), np.float32),
                    theta_ref=theta_ref, dx=dx, fill=0.6, shape="circle", tank_size=2 * R)


# ----------------------------------------------------------------------------
# LPV identification and validation (Section 5.3 set-up)
# ----------------------------------------------------------------------------

LPV_TS = 0.05            # sampling time of the surrogate (Section 5.3)


def lpv_tank(seed: int = 0, dx: float = 0.01, ctrl: bool = False) -> Scenario:
    """The paper's spacecraft (Table 1: circular tank r = 0.2 m at the centre
    of mass, 60 % fill, m = 1010.71 kg, J = 133.84 kg m^2) with this
    library's fluid model (Tait EOS c0 = 20 m/s, 3 boundary rings, dx = 10 mm,
    about 750 particles).  dt is the CFL step shortened so that a whole number
    of steps fills one sample of LPV_TS.  ctrl: PD attitude law with the
    gains of Section 5.1 (w = 0.2 pi, xi = 0.7), applied once per sample."""
    rng = np.random.default_rng(seed)
    R = 0.2
    fluid, ghosts = circle_tank(R, dx, 0.6, 3, rng, 0.01)
    p = _fluid_params(dx)
    steps = int(math.ceil(LPV_TS / p.dt))
    p.dt = LPV_TS / steps
    p.motion = MOTION_FREE
    p.ctrl = CTRL_PD_ZOH if ctrl else CTRL_NONE
    p.body_mass, p.body_inertia = 1010.71, 133.84
    w, xi = 0.2 * math.pi, 0.7
    p.kp = p.body_inertia * w * w
    p.kd = 2 * xi * p.body_inertia * w
    p.ctrl_period = steps
    pad = 5 * dx
    p.domain_min = (-R - pad, -R - pad)
    p.domain_max = (R + pad, R + pad)
    return Scenario("lpv_tank", p, _f32(fluid), np.zeros((fluid.shape[0], 2), np.float32), _f32(ghosts),
                    np.zeros(6), 0, np.zeros((0, 3), np.float32), theta_ref=np.zeros(1), dx=dx, fill=0.6,
                    shape="circle", tank_size=2 * R)


def lpv_input_train(seed: int = 0, n: int = 2200, force_amp: float = 60.0, torque_amp: float = 10.0,
                    ts: float = LPV_TS) -> np.ndarray:
    """Identification input [n, 3] (F_x, F_y world, torque), one value per
    sample (Section 5.3, Fig. iden_profile): per channel, independently, a
    random-phase multisine over the whole [0, 2) Hz band on the 0.05 Hz grid
    (all 39 nonzero tones, equal amplitudes, peak-normalised to a quarter of
    the channel amplitude) plus a train of pulse doublets: a pulse of
    U[0.3, 1.2] x amplitude and random sign held for 10-300 samples
    (0.5-15 s, long enough to reach the velocities of sustained thrust), the
    opposite pulse right after it (no net impulse), then a gap of 20-100
    samples."""
    rng = np.random.default_rng(seed)
    t = np.arange(n) * ts
    grid = np.arange(1, 40) * 0.05
    out = np.zeros((n, 3))
    for ch, amp in enumerate((force_amp, force_amp, torque_amp)):
        phi = rng.uniform(0.0, 2 * math.pi, size=grid.size)
        ms = np.sin(2 * math.pi * grid[None, :] * t[:, None] + phi[None, :]).sum(axis=1)
        ms *= 0.25 * amp / np.max(np.abs(ms))
        pulses = np.zeros(n)
        k = int(rng.integers(10, 60))
        while k < n:
            width = int(rng.integers(10, 301))
            a = amp * float(rng.uniform(0.3, 1.2)) * (1.0 if rng.random() < 0.5 else -1.0)
            pulses[k:k + width] += a
            pulses[k + width:k + 2 * width] -= a
            k += 2 * width + int(rng.integers(20, 101))
        out[:, ch] = ms + pulses
    return out


def manoeuvre_profile(k: int, ts: float = LPV_TS):
    """The two closed-loop manoeuvres of Section 5.1, as this library reads
    their description (their time series are only shown in a figure):
    profile 1 (60 s): constant thrust F_x = 50 N over 1-21 s, an attitude
    reference slew from 0 to 20 degrees over 25-27 s (trapezoidal rate, 0.5 s
    ramps), and a 100 N pulse along y over 40-40.5 s; profile 2 (40 s): a
    60 N pulse along x and y over 1-5 s, a dwell, and the opposite pulse over
    15-19 s, reference zero.  Returns (force [n, 2] world, ref [n] rad), one
    value per sample."""
    if k == 1:
        n = int(round(60.0 / ts))
        t = np.arange(n) * ts
        force = np.zeros((n, 2))
        force[(t >= 1.0) & (t < 21.0), 0] = 50.0
        force[(t >= 40.0) & (t < 40.5), 1] = 100.0
        ref = trapezoid_slew(math.radians(20.0), 0.5, 1.0, t - 25.0)
    elif k == 2:
        n = int(round(40.0 / ts))
        t = np.arange(n) * ts
        force = np.zeros((n, 2))
        on = (t >= 1.0) & (t < 5.0)
        off = (t >= 15.0) & (t < 19.0)
        force[on] = 60.0
        force[off] = -60.0
        ref = np.zeros(n)
    else:
        raise ValueError("profile 1 or 2")
    return force, ref
