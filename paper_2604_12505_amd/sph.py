"""Python binding of the SPH part of libslosh.so (argument marshalling only).

Every step of the simulation runs in the library's HIP kernels; PyTorch
provides device memory and the stream the library enqueues on.  The names
follow the C ABI: ``Simulator.step`` is ``sph_step``, ``rollout`` is
``sph_rollout`` and so on.  A ``Simulator`` holds one tank
(``sph_init``) or a batch of tanks (``sph_batch_init``); for a batch the
per-tank inputs and outputs carry a leading tank dimension.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from ._lib import SphParams, check, load

FRAME_BODY, FRAME_WORLD = 0, 1
ST_ESCAPED, ST_NONFINITE, ST_SORT = 1, 2, 4


def make_params(prm) -> SphParams:
    """Marshals any object with the fields of ``sph_params`` (e.g. workloads.Params)."""
    o = SphParams()
    for name, _ in SphParams._fields_:
        if name == "reserved":
            continue
        v = getattr(prm, name)
        if name in ("domain_min", "domain_max"):
            setattr(o, name, (C.c_double * 2)(*[float(x) for x in v]))
        else:
            setattr(o, name, v)
    return o


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_f32(a, device) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32) if isinstance(a, np.ndarray) else a,
                           dtype=torch.float32, device=device).contiguous()


def gamma1_terms(params, fluid, ghosts, device="cuda:0"):
    """(num [n], den [n]) FP64 device tensors of eq. gamma1 for every fluid
    particle (``sph_gamma1_terms``)."""
    L = load()
    f = _dev_f32(fluid, device)
    g = _dev_f32(ghosts, device)
    n = f.shape[0]
    num = torch.empty(n, dtype=torch.float64, device=device)
    den = torch.empty(n, dtype=torch.float64, device=device)
    o = make_params(params)
    st = C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    check(L.sph_gamma1_terms(C.byref(o), _ptr(f), n, _ptr(g), g.shape[0], _ptr(num), _ptr(den), st),
          "sph_gamma1_terms")
    return num, den


def gamma1_estimate(params, fluid, ghosts, device="cuda:0", top: float = 0.1) -> float:
    """A representative eq. gamma1 value: the median of num/den over the
    fluid particles whose ghost sum is in the top fraction ``top`` (the
    particles that sit against the wall with a full fluid neighbourhood on
    the other side, the configuration the paper evaluates it for)."""
    L = load()
    f = _dev_f32(fluid, device)
    g = _dev_f32(ghosts, device)
    n = f.shape[0]
    num = torch.empty(n, dtype=torch.float64, device=device)
    den = torch.empty(n, dtype=torch.float64, device=device)
    o = make_params(params)
    out = C.c_double()
    torch.cuda.synchronize(device)
    check(L.sph_gamma1_estimate(C.byref(o), _ptr(f), n, _ptr(g), g.shape[0], float(top), _ptr(num), _ptr(den),
                                C.byref(out)), "sph_gamma1_estimate")
    return float(out.value)


class Simulator:
    """One tank or a batch: ``sph_init`` / ``sph_batch_init`` on construction,
    ``sph_destroy`` on close()."""

    def __init__(self, params, pos, vel, ghosts, rigid0, device="cuda:0",
                 stream: Optional[torch.cuda.Stream] = None):
        self._setup([params], [pos], [vel], [ghosts], [rigid0], device, stream, batch=False)

    @classmethod
    def from_scenario(cls, sc, device="cuda:0", stream=None):
        return cls(sc.params, sc.pos, sc.vel, sc.ghosts, sc.rigid0, device, stream)

    @classmethod
    def batch(cls, scenarios: Sequence, device="cuda:0", stream=None):
        self = cls.__new__(cls)
        self._setup([s.params for s in scenarios], [s.pos for s in scenarios], [s.vel for s in scenarios],
                    [s.ghosts for s in scenarios], [s.rigid0 for s in scenarios], device, stream, batch=True)
        return self

    def _setup(self, params, pos, vel, ghosts, rigid0, device, stream, batch):
        self.L = load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.is_batch = batch
        self.T = len(params)
        self.params = params if batch else params[0]
        prm = (SphParams * self.T)(*[make_params(p) for p in params])
        self._prm = prm
        s0 = torch.cat([_dev_f32(p, self.device).reshape(-1, 2) for p in pos]).contiguous()
        w0 = torch.cat([_dev_f32(v, self.device).reshape(-1, 2) for v in vel]).contiguous()
        g0 = torch.cat([_dev_f32(g, self.device).reshape(-1, 2) for g in ghosts]).contiguous()
        self.counts = [int(np.asarray(p).reshape(-1, 2).shape[0]) for p in pos]
        gcounts = [int(np.asarray(g).reshape(-1, 2).shape[0]) for g in ghosts]
        self.n, self.g = int(s0.shape[0]), int(g0.shape[0])
        nf = (C.c_int32 * self.T)(*self.counts)
        ng = (C.c_int32 * self.T)(*gcounts)
        nbytes = C.c_size_t()
        check(self.L.sph_batch_workspace_bytes(self.T, prm, nf, ng, C.byref(nbytes)), "sph_batch_workspace_bytes")
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + nbytes.value]
        rig = (C.c_double * (6 * self.T))(*np.concatenate([np.asarray(r, np.float64).ravel() for r in rigid0]))
        h = C.c_void_p()
        self._enter()
        if batch:
            rc = self.L.sph_batch_init(self.T, prm, nf, _ptr(s0), _ptr(w0), ng, _ptr(g0), rig, _ptr(self.ws),
                                       C.c_size_t(nbytes.value), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        else:
            rc = self.L.sph_init(C.byref(prm[0]), self.n, _ptr(s0), _ptr(w0), self.g, _ptr(g0), rig,
                                 _ptr(self.ws), C.c_size_t(nbytes.value), C.c_void_p(self.stream.cuda_stream),
                                 C.byref(h))
        check(rc, "sph_init")
        self.h = h
        self._keep = []

    # stream ordering with the caller's current stream
    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def close(self):
        if getattr(self, "h", None):
            self.stream.synchronize()
            check(self.L.sph_destroy(self.h), "sph_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, u: Optional[torch.Tensor] = None):
        self._enter()
        if u is not None:
            u = _dev_f32(u, self.device)
            self._keep.append(u)
        check(self.L.sph_step(self.h, _ptr(u)), "sph_step")
        self._leave()

    def resident_fits(self) -> bool:
        """Every tank fits the LDS-resident rollout (``sph_resident_fits``)."""
        f = C.c_int32()
        check(self.L.sph_resident_fits(self.h, C.byref(f)), "sph_resident_fits")
        return bool(f.value)

    def rollout(self, n_steps: int, u_seq=None, theta_ref=None, log_stride: int = 0, logs: bool = True,
                resident: bool = False):
        """Runs n_steps; returns a dict of device log tensors (y, wrench, u,
        wrench_mean), [n_log, k] for one tank, [T, n_log, k] for a batch.
        Batch inputs: u_seq [T, n_steps, 3], theta_ref [T, n_ref].
        resident: run them with ``sph_rollout_resident`` (small tanks)."""
        self._enter()
        u = None
        if u_seq is not None:
            u = _dev_f32(u_seq, self.device)
            u = u.reshape(self.T, -1, 3)
            if u.shape[1] < n_steps:
                raise ValueError("u_seq shorter than n_steps")
            u = u[:, :n_steps].contiguous()
        ref = None
        if theta_ref is not None:
            ref = torch.as_tensor(theta_ref, dtype=torch.float64, device=self.device).reshape(self.T, -1).contiguous()
        n_log = (n_steps + log_stride - 1) // log_stride if log_stride > 0 else 0
        out = {}
        if n_log and logs:
            shape = (self.T, n_log) if self.is_batch else (n_log,)
            out = {"y": torch.zeros(*shape, 6, device=self.device),
                   "wrench": torch.zeros(*shape, 3, device=self.device),
                   "u": torch.zeros(*shape, 3, device=self.device),
                   "wrench_mean": torch.zeros(*shape, 3, device=self.device)}
            self._enter()
        fn = self.L.sph_rollout_resident if resident else self.L.sph_rollout
        check(fn(self.h, int(n_steps), _ptr(u), _ptr(ref), 0 if ref is None else int(ref.shape[1]),
                 int(log_stride), _ptr(out.get("y")), _ptr(out.get("wrench")), _ptr(out.get("u")),
                 _ptr(out.get("wrench_mean"))), "sph_rollout_resident" if resident else "sph_rollout")
        self._keep = [u, ref]
        self._leave()
        return out

    def rhs(self, u=None):
        """x_dot at the current state (no advance): rho, P, a_sph, wdot, wrench, acc."""
        self._enter()
        uu = None if u is None else _dev_f32(u, self.device)
        tshape = (self.T, 3) if self.is_batch else (3,)
        o = {"rho": torch.empty(self.n, device=self.device), "P": torch.empty(self.n, device=self.device),
             "a_sph": torch.empty(self.n, 2, device=self.device),
             "wdot": torch.empty(self.n, 2, device=self.device),
             "wrench": torch.empty(*tshape, device=self.device), "acc": torch.empty(*tshape, device=self.device)}
        self._enter()
        check(self.L.sph_rhs(self.h, _ptr(uu), _ptr(o["rho"]), _ptr(o["P"]), _ptr(o["a_sph"]),
                             _ptr(o["wdot"]), _ptr(o["wrench"]), _ptr(o["acc"])), "sph_rhs")
        self._keep = [uu]
        self._leave()
        return o

    def wrench(self, frame: int = FRAME_BODY) -> torch.Tensor:
        out = torch.empty(*((self.T, 3) if self.is_batch else (3,)), device=self.device)
        self._enter()
        check(self.L.sph_slosh_wrench(self.h, int(frame), _ptr(out)), "sph_slosh_wrench")
        self._leave()
        return out

    def get_state(self):
        """(s [N,2], w [N,2], rigid, tau_ctrl, step); rigid [6] / [T,6]."""
        s = torch.empty(self.n, 2, device=self.device)
        w = torch.empty(self.n, 2, device=self.device)
        rig = (C.c_double * (6 * self.T))()
        tau = (C.c_double * self.T)()
        step = (C.c_int64 * self.T)()
        self._enter()
        check(self.L.sph_get_state(self.h, _ptr(s), _ptr(w), rig, tau, step), "sph_get_state")
        self._leave()
        r = np.array(list(rig)).reshape(self.T, 6)
        if self.is_batch:
            return s, w, r, np.array(list(tau)), np.array(list(step))
        return s, w, r[0], float(tau[0]), int(step[0])

    def set_state(self, s, w, rigid, tau_ctrl=0.0, step=0):
        s = _dev_f32(s, self.device).reshape(-1, 2)
        w = _dev_f32(w, self.device).reshape(-1, 2)
        r = np.asarray(rigid, np.float64).ravel()
        rig = (C.c_double * r.size)(*r)
        self._enter()
        check(self.L.sph_set_state(self.h, _ptr(s), _ptr(w), rig, float(tau_ctrl), int(step)), "sph_set_state")
        self._leave()

    def status(self) -> int:
        f = C.c_uint32()
        self._enter()
        rc = self.L.sph_status(self.h, C.byref(f))
        if rc not in (0, -4):
            check(rc, "sph_status")
        return int(f.value)

    def neighbours(self, max_nbr: int = 64):
        nbr = torch.full((self.n, max_nbr), -1, dtype=torch.int32, device=self.device)
        cnt = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        self._enter()
        check(self.L.sph_neighbours(self.h, int(max_nbr), _ptr(nbr), _ptr(cnt)), "sph_neighbours")
        self._leave()
        return nbr, cnt

    def autotune(self, reps: int = 10) -> int:
        lanes = C.c_int32()
        self._enter()
        check(self.L.sph_autotune(self.h, int(reps), C.byref(lanes)), "sph_autotune")
        self._leave()
        return int(lanes.value)

    def set_lanes(self, lanes: int) -> None:
        check(self.L.sph_set_lanes(self.h, int(lanes)), "sph_set_lanes")

    def set_near_lists(self, on: bool) -> None:
        check(self.L.sph_set_near_lists(self.h, 1 if on else 0), "sph_set_near_lists")

    def set_rebuild_interval(self, steps: int) -> None:
        """Steps between cell-list rebuilds (1, 2, 4, 8, 16, 32 or 64)."""
        check(self.L.sph_set_rebuild_interval(self.h, int(steps)), "sph_set_rebuild_interval")

    def rebuild_interval(self) -> int:
        n = C.c_int32()
        check(self.L.sph_get_rebuild_interval(self.h, C.byref(n)), "sph_get_rebuild_interval")
        return int(n.value)

    def tuning(self):
        """(lanes per particle, near lists on)."""
        lanes, near = C.c_int32(), C.c_int32()
        check(self.L.sph_get_tuning(self.h, C.byref(lanes), C.byref(near)), "sph_get_tuning")
        return int(lanes.value), bool(near.value)

    def jvp_rollout(self, n_steps: int, u_seq=None, du_seq=None, theta_ref=None, drigid0=None, ds0=None, dw0=None,
                    fluid_tangents: bool = False):
        """sph_jvp_rollout: derivatives of n_steps steps from the current state
        along n_dir directions.  du_seq [n_dir, n_steps, 3], drigid0 [n_dir, 6],
        ds0 / dw0 [n_dir, N, 2] (caller order); at least one of them fixes
        n_dir.  Returns dict(wrench [3], dwrench [n_dir, 3], rigid [6],
        drigid [n_dir, 6], ds, dw [n_dir, N, 2] or None).  The state is not
        advanced."""
        if self.is_batch:
            raise ValueError("the tangent-linear rollout takes single-tank handles")
        sizes = [x.shape[0] for x in (du_seq, drigid0, ds0) if x is not None]
        if not sizes:
            raise ValueError("give at least one of du_seq, drigid0, ds0")
        K = int(sizes[0])
        if any(k != K for k in sizes):
            raise ValueError("direction counts differ")
        u = None if u_seq is None else _dev_f32(u_seq, self.device).reshape(-1, 3)[:n_steps].contiguous()
        du = None if du_seq is None else _dev_f32(du_seq, self.device).reshape(K, -1, 3)[:, :n_steps].contiguous()
        ref = None if theta_ref is None else torch.as_tensor(theta_ref, dtype=torch.float64,
                                                             device=self.device).reshape(-1).contiguous()
        dr = None
        if drigid0 is not None:
            r = np.ascontiguousarray(np.asarray(drigid0, np.float64).reshape(K, 6))
            dr = (C.c_double * r.size)(*r.ravel())
        s0 = None if ds0 is None else _dev_f32(ds0, self.device).reshape(K, self.n, 2).contiguous()
        w0 = None if dw0 is None else _dev_f32(dw0, self.device).reshape(K, self.n, 2).contiguous()
        nbytes = C.c_size_t()
        check(self.L.sph_jvp_workspace_bytes(self.h, K, C.byref(nbytes)), "sph_jvp_workspace_bytes")
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        ws = raw[(-raw.data_ptr()) % 256:]
        wrench, dwrench = (C.c_double * 3)(), (C.c_double * (3 * K))()
        rigid, drigid = (C.c_double * 6)(), (C.c_double * (6 * K))()
        ds = torch.empty(K, self.n, 2, device=self.device) if fluid_tangents else None
        dw = torch.empty(K, self.n, 2, device=self.device) if fluid_tangents else None
        self._enter()
        check(self.L.sph_jvp_rollout(self.h, K, int(n_steps), _ptr(u), _ptr(du), _ptr(ref),
                                     0 if ref is None else int(ref.shape[0]), dr, _ptr(s0), _ptr(w0),
                                     C.c_void_p(ws.data_ptr()), C.c_size_t(nbytes.value), wrench, dwrench, rigid,
                                     drigid, _ptr(ds), _ptr(dw)), "sph_jvp_rollout")
        self._leave()
        return {"wrench": np.array(list(wrench)), "dwrench": np.array(list(dwrench)).reshape(K, 3),
                "rigid": np.array(list(rigid)), "drigid": np.array(list(drigid)).reshape(K, 6),
                "ds": ds, "dw": dw}

    def vjp_rollout(self, n_steps: int, wbar, u_seq=None, theta_ref=None, rbar=None, sbar=None, wbar_fluid=None,
                    every: int = 20):
        """sph_vjp_rollout: adjoints of the inputs of n_steps steps from the
        current state, given the adjoint wbar [3] of the last step's wrench
        (and optionally rbar [6], sbar / wbar_fluid [N, 2] of the final
        state).  Returns dict(wrench [3], rigid0 [6], u [n_steps, 3],
        s0 [N, 2], w0 [N, 2]).  The state is not advanced."""
        if self.is_batch:
            raise ValueError("the adjoint rollout takes single-tank handles")
        u = None if u_seq is None else _dev_f32(u_seq, self.device).reshape(-1, 3)[:n_steps].contiguous()
        ref = None if theta_ref is None else torch.as_tensor(theta_ref, dtype=torch.float64,
                                                             device=self.device).reshape(-1).contiguous()
        wb = (C.c_double * 3)(*[float(x) for x in np.asarray(wbar, np.float64).ravel()])
        rb = None if rbar is None else (C.c_double * 6)(*[float(x) for x in np.asarray(rbar, np.float64).ravel()])
        sb = None if sbar is None else _dev_f32(sbar, self.device).reshape(self.n, 2).contiguous()
        wf = None if wbar_fluid is None else _dev_f32(wbar_fluid, self.device).reshape(self.n, 2).contiguous()
        nbytes = C.c_size_t()
        check(self.L.sph_vjp_workspace_bytes(self.h, int(n_steps), int(every), C.byref(nbytes)),
              "sph_vjp_workspace_bytes")
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        ws = raw[(-raw.data_ptr()) % 256:]
        wrench, g_r = (C.c_double * 3)(), (C.c_double * 6)()
        g_u = torch.zeros(n_steps, 3, device=self.device)
        g_s = torch.zeros(self.n, 2, device=self.device)
        g_w = torch.zeros(self.n, 2, device=self.device)
        self._enter()
        check(self.L.sph_vjp_rollout(self.h, int(n_steps), int(every), _ptr(u), _ptr(ref),
                                     0 if ref is None else int(ref.shape[0]), wb, rb, _ptr(sb), _ptr(wf),
                                     C.c_void_p(ws.data_ptr()), C.c_size_t(nbytes.value), wrench, g_r, _ptr(g_u),
                                     _ptr(g_s), _ptr(g_w)), "sph_vjp_rollout")
        self._leave()
        return {"wrench": np.array(list(wrench)), "rigid0": np.array(list(g_r)), "u": g_u, "s0": g_s, "w0": g_w}

    def time_kernels(self, n_steps: int, u_seq=None, theta_ref=None):
        """Mean per-launch microseconds over n_steps directly launched steps:
        bin, scan, place (per rebuild), density, force, wrench (per step)."""
        u = None if u_seq is None else _dev_f32(u_seq, self.device).reshape(self.T, -1, 3)[:, :n_steps].contiguous()
        ref = None if theta_ref is None else torch.as_tensor(theta_ref, dtype=torch.float64,
                                                              device=self.device).reshape(self.T, -1).contiguous()
        out = (C.c_float * 6)()
        self._enter()
        check(self.L.sph_time_kernels(self.h, int(n_steps), _ptr(u), _ptr(ref),
                                      0 if ref is None else int(ref.shape[1]), out), "sph_time_kernels")
        self._leave()
        return dict(zip(("bin", "scan", "place", "density", "force", "wrench"), [float(x) for x in out]))
