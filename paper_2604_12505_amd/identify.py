"""Identification of the paper's LPV surrogate from SPH data (Section 5.3)
and its closed-loop validation (Section 5.4), on this library's kernels.

    python -m paper_2604_12505_amd.identify --out lpv.json

Steps (orchestration only; every rollout runs in the SPH kernels, every
simulation, gradient and optimizer step in the LPV kernels):

1. SPH data.  The paper's spacecraft and fuel (Tables 1-2: 666 particles
   spawned at random and relaxed to rest, dt = 1 ms; ``--tank tait`` takes
   this library's Tait fluid instead) are driven open loop by the input
   train of ``workloads.lpv_input_train`` (2,200 samples of 0.05 s); the
   velocities (rdot_x, rdot_y, thetadot) are logged at the sample instants.
   The same tank, under the sampled PD attitude law, flies the two
   manoeuvres of ``workloads.manoeuvre_profile``.
2. Scaling.  Each input and output channel is divided by its root mean
   square over the training record (zero stays zero, so the model needs no
   offset terms).
3. LTI initialisation.  The paper initialises M0 with MATLAB's ``ssest``
   (simulation focus, D = 0, no noise model), which is not available here;
   its stand-in is the same simulation-error fit restricted to the LTI part
   (A0, B0, C0, x0), run from ``n_lti`` random stable starts in parallel,
   keeping the best training BFR.
4. LPV fit.  ``n_restarts`` starts (paper: 8): M0 and x0 from the LTI model,
   M1 from a zero-mean normal distribution, the scheduling network by Xavier's
   uniform rule with zero biases; Adam (paper: 2,000 iterations) then L-BFGS
   (paper: up to 6,000); the restart with the best average training BFR is
   kept.  All restarts run at once, 16 per wave.
5. Validation.  The LTI and LPV models, augmented with position integrators,
   fly both manoeuvres in closed loop with the same attitude law; BFR of the
   six outputs against the SPH runs, and simulation times.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time
from typing import Optional

import numpy as np
import torch

import workloads as W

from . import lpv as L
from .sph import Simulator
from .surrogate import _relax


def bfr(y: np.ndarray, yh: np.ndarray) -> np.ndarray:
    """Best fit rate per channel in percent (Section 5.3 footnote)."""
    y = np.asarray(y, np.float64)
    yh = np.asarray(yh, np.float64)
    num = np.sqrt(((y - yh) ** 2).sum(0))
    den = np.sqrt(((y - y.mean(0)) ** 2).sum(0))
    return 100.0 * (1.0 - num / np.maximum(den, 1e-300))


def _gpu_seconds(fn, stream):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    out = fn()
    e1.record(stream)
    e1.synchronize()
    return out, e0.elapsed_time(e1) / 1e3


def tank_scenario(tank: str, seed: int, ctrl: bool):
    """'paper': the paper's spacecraft and fluid (Tables 1-2, 666 particles
    spawned at random, linear EOS without tension, dt = 1 ms); 'tait': the
    same spacecraft with this library's Tait fluid (``workloads.lpv_tank``)."""
    if tank == "paper":
        sc = W.paper_p0(seed, n_steps=1, spawn="random")
        if not ctrl:
            sc = dataclasses.replace(sc, params=dataclasses.replace(sc.params, ctrl=W.CTRL_NONE))
        return sc
    if tank == "tait":
        return W.lpv_tank(seed, ctrl=ctrl)
    raise ValueError("tank must be 'paper' or 'tait'")


def sph_run(u_samples: np.ndarray, ref: Optional[np.ndarray], seed: int = 0, relax=(60, 50),
            device="cuda:0", tank: str = "paper") -> dict:
    """One SPH run: inputs held for one sample each (u_samples [n, 3] world
    forces and torque), the PD law when ref is given, from the fluid relaxed
    to rest (relax = cycles x steps of kinetic damping).  Returns y [n, 6]
    (state at each sample instant), u [n, 3] (applied torque includes the
    law's), the GPU seconds of the rollout (relaxation excluded; the
    LDS-resident rollout when the tank fits it), steps and particles."""
    sc = tank_scenario(tank, seed, ref is not None)
    steps = sc.params.ctrl_period
    n = u_samples.shape[0]
    sim = Simulator.from_scenario(sc, device=device)
    try:
        _relax(sim, relax[0], relax[1])
        u = torch.as_tensor(np.repeat(np.asarray(u_samples, np.float32), steps, axis=0), device=device)
        th = None if ref is None else np.asarray(ref, np.float64)
        torch.cuda.synchronize(device)
        resident = sim.resident_fits()
        lg, secs = _gpu_seconds(lambda: sim.rollout(n * steps, u, theta_ref=th, log_stride=steps, resident=resident),
                                sim.stream)
        st = sim.status()
        if st != 0:
            raise RuntimeError(f"SPH run raised status {st}")
        return {"y": lg["y"].double().cpu().numpy(), "u": lg["u"].double().cpu().numpy(), "sph_seconds": secs,
                "steps": n * steps, "n_fluid": sc.n_fluid, "dt": sc.params.dt, "kp": sc.params.kp,
                "kd": sc.params.kd}
    finally:
        sim.close()


def rms_scales(u: np.ndarray, y: np.ndarray):
    us = np.sqrt((np.asarray(u) ** 2).mean(0))
    ys = np.sqrt((np.asarray(y) ** 2).mean(0))
    return np.maximum(us, 1e-12), np.maximum(ys, 1e-12)


def _pack(A0, B0, C0, A1, B1, C1, W1, b1, W2, b2, W3, b3, x0):
    return np.concatenate([np.ravel(a) for a in (A0, B0, C0, A1, B1, C1, W1, b1, W2, b2, W3, b3, x0)])


def lti_starts(rng, R: int) -> np.ndarray:
    """Random stable LTI starts: A0 near a diagonal of poles in [0.9, 0.999]."""
    out = []
    z = np.zeros
    for _ in range(R):
        A0 = np.diag(rng.uniform(0.9, 0.999, 4)) + 0.01 * rng.normal(size=(4, 4))
        B0 = 0.1 * rng.normal(size=(4, 3))
        C0 = 0.5 * rng.normal(size=(3, 4))
        out.append(_pack(A0, B0, C0, z((4, 4)), z((4, 3)), z((3, 4)), z((4, 7)), z(4), z((4, 4)), z(4), z((1, 4)),
                         z(1), z(4)))
    return np.stack(out)


def lpv_starts(rng, lti: np.ndarray, R: int, m1_std: float = 0.01) -> np.ndarray:
    """M0 and x0 from the LTI model, M1 ~ N(0, m1_std^2), the scheduling
    network by Xavier's uniform rule (bound sqrt(6 / (fan_in + fan_out))),
    zero biases.  The first start has M1 = 0: it is the LTI model itself, so
    the best restart is never worse than the model the fit starts from."""
    out = []
    for r in range(R):
        v = lti.copy()
        v[40:80] = 0.0 if r == 0 else m1_std * rng.normal(size=40)
        o = 80
        for fan_in, fan_out in ((7, 4), (4, 4), (4, 1)):
            a = math.sqrt(6.0 / (fan_in + fan_out))
            v[o:o + fan_in * fan_out] = rng.uniform(-a, a, fan_in * fan_out)
            o += fan_in * fan_out
            v[o:o + fan_out] = 0.0
            o += fan_out
        out.append(v)
    return np.stack(out)


def fit(u_s: np.ndarray, y_s: np.ndarray, starts: np.ndarray, adam_iters: int, lbfgs_iters: int,
        opts: L.Options, device="cuda:0"):
    """Adam then L-BFGS on every start at once.  Returns (params [R, 141]
    numpy, training BFR [R, 3], seconds of Adam, seconds of L-BFGS, L-BFGS
    status [R], L-BFGS iterations [R])."""
    dev = torch.device(device)
    P = torch.as_tensor(starts, dtype=torch.float64, device=dev).contiguous()
    u = torch.as_tensor(u_s, dtype=torch.float64, device=dev).contiguous()
    y = torch.as_tensor(y_s, dtype=torch.float64, device=dev).contiguous()
    ws = L.workspace(P.shape[0], u.shape[0], dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    if adam_iters > 0:
        L.adam(P, u, y, adam_iters, opts, ws=ws)
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    status = iters = np.zeros(P.shape[0], np.int32)
    if lbfgs_iters > 0:
        _, st, it = L.lbfgs(P, u, y, lbfgs_iters, opts, ws=ws)
        status, iters = st.cpu().numpy(), it.cpu().numpy()
    torch.cuda.synchronize(dev)
    t2 = time.perf_counter()
    del stream
    yh = L.simulate(P, u).cpu().numpy()
    fits = np.stack([bfr(y_s, yh[r]) for r in range(P.shape[0])])
    fits[~np.isfinite(fits)] = -np.inf
    return P.cpu().numpy(), fits, t1 - t0, t2 - t1, status, iters


def identify(u_train: np.ndarray, y_train: np.ndarray, n_lti: int = 64, n_restarts: int = 8,
             adam_iters: int = 2000, lbfgs_iters: int = 6000, lti_adam: int = 2000, lti_lbfgs: int = 6000,
             sigma2: float = 1e-4, sigmax: float = 1e-6, lr: float = 1e-3, seed: int = 0, device="cuda:0",
             log=None) -> dict:
    """Scaling, LTI stand-in for ssest, LPV fit; returns the chosen models
    (scaled units) with their training BFR and the timings."""
    us, ys = rms_scales(u_train, y_train)
    u_s, y_s = u_train / us, y_train / ys
    rng = np.random.default_rng(seed)
    lti_opts = L.Options(sigma2=sigma2, sigmax=sigmax, lr=lr, lti_only=True)
    Pl, fl, ta, tb, _, _ = fit(u_s, y_s, lti_starts(rng, n_lti), lti_adam, lti_lbfgs, lti_opts, device)
    best_l = int(np.argmax(fl.mean(1)))
    if log:
        log(f"LTI: {n_lti} starts, best training BFR {fl[best_l].mean():.2f} % ({ta + tb:.1f} s)")
    opts = L.Options(sigma2=sigma2, sigmax=sigmax, lr=lr)
    Pv, fv, tc, td, st, it = fit(u_s, y_s, lpv_starts(rng, Pl[best_l], n_restarts), adam_iters, lbfgs_iters, opts,
                                 device)
    best = int(np.argmax(fv.mean(1)))
    if log:
        log(f"LPV: {n_restarts} restarts, training BFR {np.round(fv.mean(1), 2).tolist()}, "
            f"best {fv[best].mean():.2f} % (Adam {tc:.1f} s, L-BFGS {td:.1f} s)")
    return {"u_scale": us, "y_scale": ys, "lti": Pl[best_l], "lti_bfr": fl[best_l], "lpv": Pv[best],
            "lpv_bfr": fv[best], "lpv_bfr_all": fv.mean(1), "lti_seconds": ta + tb, "adam_seconds": tc,
            "lbfgs_seconds": td, "lbfgs_status": st, "lbfgs_iters": it}


def closed_loop(model: np.ndarray, force: np.ndarray, ref: np.ndarray, res: dict, kp: float, kd: float,
                device="cuda:0", reps: int = 5):
    """The model in closed loop on one manoeuvre: (y [n, 6], mean GPU seconds)."""
    P = torch.as_tensor(model, dtype=torch.float64, device=device).reshape(1, -1)
    f = torch.as_tensor(force, dtype=torch.float64, device=device)
    r = torch.as_tensor(ref, dtype=torch.float64, device=device)
    st = torch.cuda.current_stream(device)
    y = L.closed_loop(P, f, r, W.LPV_TS, kp, kd, res["u_scale"], res["y_scale"])
    _, secs = _gpu_seconds(lambda: [L.closed_loop(P, f, r, W.LPV_TS, kp, kd, res["u_scale"], res["y_scale"])
                                    for _ in range(reps)], st)
    return y[0].cpu().numpy(), secs / reps


def monte_carlo_rate(model: np.ndarray, res: dict, kp: float, kd: float, n_traj: int = 16384, device="cuda:0"):
    """Closed-loop trajectories per second of profile 1 with n_traj random
    slew amplitudes in one launch (the Monte Carlo use of Section 5.4)."""
    force, ref = W.manoeuvre_profile(1)
    rng = np.random.default_rng(0)
    refs = ref[None, :] * rng.uniform(0.2, 1.5, size=(n_traj, 1))
    P = torch.as_tensor(np.tile(model, (n_traj, 1)), dtype=torch.float64, device=device)
    f = torch.as_tensor(force, dtype=torch.float64, device=device)
    r = torch.as_tensor(refs, dtype=torch.float64, device=device)
    st = torch.cuda.current_stream(device)
    L.closed_loop(P, f, r, W.LPV_TS, kp, kd, res["u_scale"], res["y_scale"])
    _, secs = _gpu_seconds(lambda: L.closed_loop(P, f, r, W.LPV_TS, kp, kd, res["u_scale"], res["y_scale"]), st)
    return n_traj / secs, secs


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=2200)
    ap.add_argument("--lti-starts", type=int, default=64)
    ap.add_argument("--restarts", type=int, default=8)
    ap.add_argument("--adam", type=int, default=2000)
    ap.add_argument("--lbfgs", type=int, default=6000)
    ap.add_argument("--lti-adam", type=int, default=2000)
    ap.add_argument("--lti-lbfgs", type=int, default=6000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tank", default="paper", choices=("paper", "tait"))
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)

    t0 = time.time()
    u_train = W.lpv_input_train(a.seed, a.samples)
    log(f"SPH identification run: {a.samples} samples")
    tr = sph_run(u_train, None, seed=a.seed, tank=a.tank)
    log(f"  {tr['steps']} steps of {tr['n_fluid']} particles in {tr['sph_seconds']:.1f} s")
    y_train = tr["y"][:, 3:6]
    res = identify(u_train, y_train, a.lti_starts, a.restarts, a.adam, a.lbfgs, a.lti_adam, a.lti_lbfgs,
                   seed=a.seed, log=log)
    out = {"tank": a.tank, "samples": a.samples, "n_fluid": tr["n_fluid"], "sph_train_seconds": tr["sph_seconds"],
           "sph_train_steps": tr["steps"], "lti_starts": a.lti_starts, "restarts": a.restarts,
           "adam_iters": a.adam, "lbfgs_max_iters": a.lbfgs,
           "train_bfr_lti": res["lti_bfr"].tolist(), "train_bfr_lpv": res["lpv_bfr"].tolist(),
           "train_bfr_lpv_restarts": res["lpv_bfr_all"].tolist(),
           "lti_fit_seconds": res["lti_seconds"], "lpv_adam_seconds": res["adam_seconds"],
           "lpv_lbfgs_seconds": res["lbfgs_seconds"], "lbfgs_status": res["lbfgs_status"].tolist(),
           "lbfgs_iters": res["lbfgs_iters"].tolist(), "profiles": {}}
    for k in (1, 2):
        force, ref = W.manoeuvre_profile(k)
        u = np.concatenate([force, np.zeros((force.shape[0], 1))], 1)
        log(f"SPH manoeuvre {k}: {force.shape[0]} samples")
        run = sph_run(u, ref, seed=a.seed, tank=a.tank)
        prof = {"sph_seconds": run["sph_seconds"], "sph_steps": run["steps"]}
        for name in ("lti", "lpv"):
            y, secs = closed_loop(res[name], force, ref, res, run["kp"], run["kd"])
            prof[name + "_bfr"] = bfr(run["y"], y).tolist()
            prof[name + "_seconds"] = secs
        prof["lpv_speedup"] = run["sph_seconds"] / prof["lpv_seconds"]
        out["profiles"][str(k)] = prof
        log(f"  BFR r_x r_y theta rdot_x rdot_y thetadot: LTI {np.round(prof['lti_bfr'], 2).tolist()} "
            f"LPV {np.round(prof['lpv_bfr'], 2).tolist()}; SPH {run['sph_seconds']:.2f} s, "
            f"LPV {prof['lpv_seconds'] * 1e3:.2f} ms")
    kp, kd = tr["kp"], tr["kd"]
    rate, secs = monte_carlo_rate(res["lpv"], res, kp, kd)
    out["monte_carlo_traj_per_s"] = rate
    out["monte_carlo_seconds_16384"] = secs
    out["wall_seconds"] = time.time() - t0
    log(json.dumps(out))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
