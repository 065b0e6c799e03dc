"""ctypes binding of the FP64 SPH oracle (``sph_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Argument marshalling only; every formula lives in
the C file, which cites the paper's equations it follows.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None


class OraParams(C.Structure):
    _fields_ = [
        ("eos", C.c_int32), ("motion", C.c_int32), ("ctrl", C.c_int32), ("kernel_norm", C.c_int32),
        ("h", C.c_double), ("h_spiky", C.c_double), ("rho0", C.c_double), ("mass", C.c_double),
        ("c0", C.c_double), ("tait_gamma", C.c_double), ("k_lin", C.c_double),
        ("visc_alpha", C.c_double), ("visc_beta", C.c_double), ("eps", C.c_double),
        ("gamma1", C.c_double), ("dt", C.c_double),
        ("body_mass", C.c_double), ("body_inertia", C.c_double), ("kp", C.c_double), ("kd", C.c_double),
        ("ctrl_period", C.c_int32), ("use_cells", C.c_int32),
        ("sine_amp", C.c_double), ("sine_freq", C.c_double),
        ("domain_min", C.c_double * 2), ("domain_max", C.c_double * 2),
    ]


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        d, i, i64, p = C.c_double, C.c_int, C.c_int64, C.c_void_p
        for name in ("ora_w_cubic", "ora_dw_cubic"):
            getattr(L, name).restype = d
            getattr(L, name).argtypes = [d, d, i]
        for name in ("ora_w_spiky", "ora_dw_spiky"):
            getattr(L, name).restype = d
            getattr(L, name).argtypes = [d, d]
        L.ora_eos.restype = d
        L.ora_eos.argtypes = [C.POINTER(OraParams), d]
        L.ora_pairs.restype = i
        L.ora_pairs.argtypes = [i, p, p, d, i, p, p, i, p, p]
        L.ora_pairs_f32.restype = i
        L.ora_pairs_f32.argtypes = [i, p, p, C.c_float, i, p, p]
        L.ora_rhs.restype = i
        L.ora_rhs.argtypes = [C.POINTER(OraParams), i, p, p, p, p, i, p, p, p, d, i64, p,
                              p, p, p, p, p, p, p, p, p, p]
        L.ora_rollout.restype = i
        L.ora_rollout.argtypes = [C.POINTER(OraParams), i, p, p, p, p, i, p, p, p, p, p, i, p, p, i,
                                  i, p, p, p, p]
        L.ora_rollout_world.restype = i
        L.ora_rollout_world.argtypes = [C.POINTER(OraParams), i, p, p, p, p, i, p, p, p, p, p, i, p,
                                        p, i, p]
        L.ora_num_threads.restype = i
        L.ora_num_threads.argtypes = []
        L.ora_set_num_threads.restype = None
        L.ora_set_num_threads.argtypes = [i]
        L.ora_set_round_f32.restype = None
        L.ora_set_round_f32.argtypes = [i]
        L.ora_gamma1_terms.restype = None
        L.ora_gamma1_terms.argtypes = [C.POINTER(OraParams), i, p, p, i, p, p, p, p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_params(prm, use_cells: bool = True) -> OraParams:
    """Marshals a ``workloads.Params`` (or any object with the same fields)."""
    o = OraParams()
    for name, _ in OraParams._fields_:
        if name == "use_cells":
            continue
        v = getattr(prm, name)
        if name in ("domain_min", "domain_max"):
            setattr(o, name, (C.c_double * 2)(*[float(x) for x in v]))
        else:
            setattr(o, name, v)
    o.use_cells = 1 if use_cells else 0
    return o


def w_cubic(r, h, printed=False):
    L = lib()
    return np.vectorize(lambda x: L.ora_w_cubic(float(x), float(h), int(printed)))(r)


def dw_cubic(r, h, printed=False):
    L = lib()
    return np.vectorize(lambda x: L.ora_dw_cubic(float(x), float(h), int(printed)))(r)


def w_spiky(r, hs):
    L = lib()
    return np.vectorize(lambda x: L.ora_w_spiky(float(x), float(hs)))(r)


def dw_spiky(r, hs):
    L = lib()
    return np.vectorize(lambda x: L.ora_dw_spiky(float(x), float(hs)))(r)


def eos(prm, rho):
    L = lib()
    o = make_params(prm)
    return np.vectorize(lambda x: L.ora_eos(C.byref(o), float(x)))(rho)


def pairs(pos, radius, use_cells=True, domain_min=None, domain_max=None):
    """Ordered neighbour pairs (i, j), i != j, |p_i - p_j| < radius, sorted."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    x = np.ascontiguousarray(pos[:, 0]); y = np.ascontiguousarray(pos[:, 1])
    lo = np.array(domain_min if domain_min is not None else pos.min(axis=0) - radius, np.float64)
    hi = np.array(domain_max if domain_max is not None else pos.max(axis=0) + radius, np.float64)
    cap = max(1024, 64 * n)
    while True:
        pi = np.empty(cap, np.int32); pj = np.empty(cap, np.int32)
        k = lib().ora_pairs(n, _ptr(x), _ptr(y), float(radius), int(use_cells), _ptr(lo), _ptr(hi),
                            cap, _ptr(pi), _ptr(pj))
        if k >= 0:
            return pi[:k].copy(), pj[:k].copy()
        cap *= 4


def pairs_f32(pos, radius):
    """Brute-force pairs with the single-precision predicate fmaf(dy,dy,dx*dx) < r^2."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    n = pos.shape[0]
    x = np.ascontiguousarray(pos[:, 0]); y = np.ascontiguousarray(pos[:, 1])
    cap = max(1024, 64 * n)
    while True:
        pi = np.empty(cap, np.int32); pj = np.empty(cap, np.int32)
        k = lib().ora_pairs_f32(n, _ptr(x), _ptr(y), C.c_float(radius), cap, _ptr(pi), _ptr(pj))
        if k >= 0:
            return pi[:k].copy(), pj[:k].copy()
        cap *= 4


@dataclass
class State:
    """Body-frame state: s, w [N,2]; rigid [6]; held torque; step counter."""
    s: np.ndarray
    w: np.ndarray
    rigid: np.ndarray
    tau_ctrl: float = 0.0
    step: int = 0

    def copy(self):
        return State(self.s.copy(), self.w.copy(), self.rigid.copy(), self.tau_ctrl, self.step)


def state_from_scenario(sc) -> State:
    return State(sc.pos.astype(np.float64), sc.vel.astype(np.float64),
                 np.array(sc.rigid0, np.float64), 0.0, 0)


def rhs(prm, st: State, ghosts, u=(0.0, 0.0, 0.0), use_cells=True):
    """x_dot at the state: dict of rho, P, a_sph [N,2], wdot [N,2], wrench [3], acc [3],
    wall_terms [N,3], each particle's term of the wrench sum, and wall_abs
    [N,3], per particle the sums over its wall pairs of |F_x|, |F_y| and
    |g_x F_y| + |g_y F_x| (the scale of the rounding of the wrench)."""
    o = make_params(prm, use_cells)
    n = st.s.shape[0]
    g = np.ascontiguousarray(ghosts, np.float64)
    sx = np.ascontiguousarray(st.s[:, 0]); sy = np.ascontiguousarray(st.s[:, 1])
    wx = np.ascontiguousarray(st.w[:, 0]); wy = np.ascontiguousarray(st.w[:, 1])
    gx = np.ascontiguousarray(g[:, 0]); gy = np.ascontiguousarray(g[:, 1])
    rho = np.empty(n); P = np.empty(n); ax = np.empty(n); ay = np.empty(n)
    dwx = np.empty(n); dwy = np.empty(n); wrench = np.empty(3); acc = np.empty(3)
    fwall = np.zeros((max(n, 1), 3))
    fwabs = np.zeros((max(n, 1), 3))
    uu = np.array(u, np.float64)
    rg = np.ascontiguousarray(st.rigid, np.float64)
    lib().ora_rhs(C.byref(o), n, _ptr(sx), _ptr(sy), _ptr(wx), _ptr(wy), g.shape[0], _ptr(gx),
                  _ptr(gy), _ptr(rg), float(st.tau_ctrl), int(st.step), _ptr(uu), _ptr(rho), _ptr(P),
                  _ptr(ax), _ptr(ay), _ptr(dwx), _ptr(dwy), _ptr(wrench), _ptr(acc), _ptr(fwall),
                  _ptr(fwabs))
    return dict(rho=rho, P=P, a_sph=np.stack([ax, ay], 1), wdot=np.stack([dwx, dwy], 1),
                wrench=wrench, acc=acc, wall_terms=fwall[:n], wall_abs=fwabs[:n])


def rollout(prm, st: State, ghosts, n_steps, u_seq=None, theta_ref=None, log_stride=0,
            use_cells=True):
    """Advances ``st`` in place; returns (status, logs dict)."""
    o = make_params(prm, use_cells)
    n = st.s.shape[0]
    g = np.ascontiguousarray(ghosts, np.float64)
    sx = np.ascontiguousarray(st.s[:, 0]); sy = np.ascontiguousarray(st.s[:, 1])
    wx = np.ascontiguousarray(st.w[:, 0]); wy = np.ascontiguousarray(st.w[:, 1])
    gx = np.ascontiguousarray(g[:, 0]); gy = np.ascontiguousarray(g[:, 1])
    rg = np.ascontiguousarray(st.rigid, np.float64).copy()
    tau = np.array([st.tau_ctrl], np.float64)
    step = np.array([st.step], np.int64)
    u = None if u_seq is None else np.ascontiguousarray(u_seq[:n_steps], np.float32)
    tr = None if theta_ref is None else np.ascontiguousarray(theta_ref, np.float64)
    n_log = (n_steps + log_stride - 1) // log_stride if log_stride > 0 else 0
    logs = dict(y=np.zeros((n_log, 6)), wrench=np.zeros((n_log, 3)), u=np.zeros((n_log, 3)),
                wrench_mean=np.zeros((n_log, 3)))
    status = lib().ora_rollout(
        C.byref(o), n, _ptr(sx), _ptr(sy), _ptr(wx), _ptr(wy), g.shape[0], _ptr(gx), _ptr(gy),
        _ptr(rg), _ptr(tau), _ptr(step), int(n_steps), _ptr(u), _ptr(tr),
        0 if tr is None else tr.shape[0], int(log_stride),
        _ptr(logs["y"]) if n_log else None, _ptr(logs["wrench"]) if n_log else None,
        _ptr(logs["u"]) if n_log else None, _ptr(logs["wrench_mean"]) if n_log else None)
    st.s = np.stack([sx, sy], 1); st.w = np.stack([wx, wy], 1)
    st.rigid = rg; st.tau_ctrl = float(tau[0]); st.step = int(step[0])
    return status, logs


def rollout_world(prm, x, v, ghosts_body, rigid, n_steps, u_seq=None, theta_ref=None, step0=0,
                  tau_ctrl=0.0):
    """World-frame rollout (eq. kinematicghost read literally), brute-force
    neighbours.  Returns (x, v, rigid, tau_ctrl, wrench_log[n_steps,3])."""
    o = make_params(prm, False)
    n = x.shape[0]
    g = np.ascontiguousarray(ghosts_body, np.float64)
    xx = np.ascontiguousarray(x[:, 0], np.float64).copy(); xy = np.ascontiguousarray(x[:, 1], np.float64).copy()
    vx = np.ascontiguousarray(v[:, 0], np.float64).copy(); vy = np.ascontiguousarray(v[:, 1], np.float64).copy()
    gx = np.ascontiguousarray(g[:, 0]); gy = np.ascontiguousarray(g[:, 1])
    rg = np.ascontiguousarray(rigid, np.float64).copy()
    tau = np.array([tau_ctrl], np.float64)
    step = np.array([step0], np.int64)
    u = None if u_seq is None else np.ascontiguousarray(u_seq[:n_steps], np.float32)
    tr = None if theta_ref is None else np.ascontiguousarray(theta_ref, np.float64)
    wl = np.zeros((n_steps, 3))
    lib().ora_rollout_world(C.byref(o), n, _ptr(xx), _ptr(xy), _ptr(vx), _ptr(vy), g.shape[0],
                            _ptr(gx), _ptr(gy), _ptr(rg), _ptr(tau), _ptr(step), int(n_steps),
                            _ptr(u), _ptr(tr), 0 if tr is None else tr.shape[0], _ptr(wl))
    return np.stack([xx, xy], 1), np.stack([vx, vy], 1), rg, float(tau[0]), wl


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_num_threads(n: int) -> None:
    lib().ora_set_num_threads(int(n))


def set_round_f32(on: bool) -> None:
    """Rollouts round the fluid state to binary32 after every step (off by
    default): a measure of how much rounding at that precision moves them."""
    lib().ora_set_round_f32(1 if on else 0)


def gamma1_terms(prm, fluid, ghosts):
    """(num [n], den [n]) of eq. gamma1 for every fluid particle:
    num_i = rho0/m - sum_f W_if (self included), den_i = sum_g W_ig."""
    f = np.ascontiguousarray(fluid, np.float64)
    g = np.ascontiguousarray(ghosts, np.float64)
    sx, sy = np.ascontiguousarray(f[:, 0]), np.ascontiguousarray(f[:, 1])
    gx, gy = np.ascontiguousarray(g[:, 0]), np.ascontiguousarray(g[:, 1])
    num = np.zeros(f.shape[0])
    den = np.zeros(f.shape[0])
    o = make_params(prm)
    lib().ora_gamma1_terms(C.byref(o), f.shape[0], _ptr(sx), _ptr(sy), g.shape[0], _ptr(gx), _ptr(gy),
                           _ptr(num), _ptr(den))
    return num, den
