#!/usr/bin/env python
"""Benchmark of the coupled SPH sloshing step on one MI355X.

Workload: the closed-loop circular-tank run -- tank radius 0.5 m, 30 % fill,
particle spacing 4 mm (14,542 fluid + 2,385 boundary particles), h = 1.3 dx,
Tait EOS (gamma 7, c0 = 20 m/s), dt = 0.2 h / c0, spacecraft 1000 kg and
500 kg m^2 under a PD attitude law (zero-order hold 0.05 s) tracking a
30-degree trapezoidal-rate slew.  A step is one pass of the whole step
(cell list, density/EOS, forces, slosh wrench, controller, rigid body,
fictitious accelerations, integrator); the timed region is one rollout of
--steps steps replayed from HIP graphs, inputs resident in HBM.

Prints one JSON line: particle-steps/s, the roofline position of the
dominant kernel (HIP-event kernel times measured in this run), and the FP64
oracle timed on the host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
# FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (packed) x 2 (FMA) x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3

# Algorithmic bytes per launch of each kernel, per fluid particle (p),
# boundary particle (g) and grid cell (c): what the method must move.
#   density: read s, w, a_sph (24 B), write the updated s, w (16 B) and
#            rho, P/rho^2 (8 B); boundary positions 8 B
#   force:   read s, w, rho, P/rho^2 (24 B), write a_sph (8 B); boundary 8 B
#   wrench:  negligible (a few partials per tank)
# and, every SORT_EVERY steps, the cell-list rebuild:
#   bin:     read s (8 B), write the cell key (4 B) (inside the force launch)
#   scan:    read the count, write the start, clear the count (12 B per cell)
#   place:   read key, s, w, a_sph, id (32 B), write s, w, a_sph, id and s at
#            the rebuild (36 B)
BYTES = {"density": (48, 8, 0), "force": (32, 8, 0), "wrench": (0, 0, 0), "bin": (12, 0, 0),
         "scan": (0, 0, 12), "place": (68, 0, 0)}
SORT_EVERY = 4

# Algorithmic FP32 operations per fluid particle and launch: about 20
# in-support fluid neighbours at h = 1.3 dx, times 28 operations per pair
# term of the force (differences, squared distance, square root, kernel
# gradient, viscous quotient, pressure sum, two accumulations) and 14 per
# density term (squared distance, square root, the spline shape, one sum).
NEIGHBOURS = 20
FLOP = {"density": NEIGHBOURS * 14, "force": NEIGHBOURS * 28}

# HBM traffic per launch of the neighbour kernels from rocprofv3 --pmc
# FETCH_SIZE / WRITE_SIZE (per dispatch, scaled by the copy-kernel
# calibration, averaged over the plain and the rebuild-step variants in the
# proportion they run), on the closed-loop tank for the configurations the
# autotuner picks from (profiles/hbm_traffic_closed_loop_circle.md); valid
# for the source whose hash is recorded, null once the kernel source changes.
TRAFFIC = {"src_sha1": "edc4a7216d9360e4305a2ec70cea0791bf63e82e",
           "bytes_per_launch": {"sph_force/16/0": 1735751, "sph_density/16/0": 2017587, "sph_force/16/1": 3199024, "sph_density/16/1": 3367910, "sph_force/32/0": 1792229, "sph_density/32/0": 2024753, "sph_force/32/1": 3245754, "sph_density/32/1": 3372735}}


def progress(msg: str) -> None:
    """A progress line on stderr (stdout carries the one JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def src_hash() -> str:
    h = hashlib.sha1()
    with open(os.path.join(ROOT, "paper_2604_12505_amd", "csrc", "sph.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def cpu_baseline(sc, n_steps: int):
    """The FP64 oracle, as it stands, on the first n_steps of the workload."""
    from oracle import sph as O
    st = O.state_from_scenario(sc)
    t0 = time.perf_counter()
    O.rollout(sc.params, st, sc.ghosts.astype(np.float64), n_steps, sc.u_seq[:n_steps], sc.theta_ref)
    dt = time.perf_counter() - t0
    return {"value": sc.n_fluid * n_steps / dt, "unit": "particle-steps/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"first {n_steps} steps of the same workload ({sc.n_fluid} fluid particles), "
                      f"{dt:.1f} s, FP64 C with OpenMP over particles"}


def kernel_roofline(kus, n_fluid, n_ghost, n_cells, lanes=None, near=None, traffic_workload=None):
    """Roofline position of the kernel that takes the most time per step.

    The neighbour kernels are arithmetic-bound, not HBM-bound, by the
    operation count (bound "alu", against the FP32 vector peak); the HBM
    view of the same launch is reported beside it."""
    per_step = {k: v / (SORT_EVERY if k in ("bin", "scan", "place") else 1) for k, v in kus.items()}
    dominant = max(per_step, key=per_step.get)
    bp, bg, bc = BYTES[dominant]
    alg_bytes = bp * n_fluid + bg * n_ghost + bc * n_cells
    secs = kus[dominant] * 1e-6
    gbs = alg_bytes / secs / 1e9
    # measured traffic exists for the closed-loop tank only
    key = f"sph_{dominant}/{lanes}/{1 if near else 0}"
    traffic = (TRAFFIC["bytes_per_launch"].get(key)
               if traffic_workload == "closed_loop_circle" and TRAFFIC["src_sha1"] == src_hash() else None)
    hbm = {"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
           "algorithmic_bytes_per_launch": alg_bytes}
    if dominant in FLOP:
        flops = FLOP[dominant] * n_fluid
        tf = flops / secs / 1e12
        return {"bound": "alu", "achieved": round(tf, 4), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic, "kernel": "sph_" + dominant,
                "algorithmic_flop_per_launch": flops, "launch_us": kus[dominant], "hbm": hbm}
    return {"bound": "hbm", "achieved": hbm["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": hbm["frac"], "traffic": traffic, "kernel": "sph_" + dominant,
            "algorithmic_bytes_per_launch": alg_bytes, "launch_us": kus[dominant]}


def n_cells_of(sc):
    cell = (2.0 + 1.0) * sc.params.h * (1 + 1e-6)
    return int(np.ceil((sc.params.domain_max[0] - sc.params.domain_min[0]) / cell)) * \
        int(np.ceil((sc.params.domain_max[1] - sc.params.domain_min[1]) / cell))


def batch_leg(n_tanks: int, steps: int, warmup: int, kernel_steps: int, lanes: int = 0, near: int = -1):
    """Many random tanks (rectangular or circular, fill U[0.2, 0.8], 2k-60k
    particles, multisine torque) advanced together in the same launches."""
    import torch
    import workloads as W
    from paper_2604_12505_amd.sph import Simulator
    total = warmup + steps + kernel_steps
    scs = [W.random_tank(seed, n_steps=total) for seed in range(n_tanks)]
    dev = torch.device("cuda:0")
    sim = Simulator.batch(scs, device=dev)
    if lanes > 0:
        sim.set_lanes(lanes)
        sim.set_near_lists(near == 1)
    else:
        sim.autotune(reps=5)
    lanes, near = sim.tuning()
    u = torch.stack([torch.as_tensor(sc.u_seq) for sc in scs]).to(dev)
    sim.rollout(warmup, u[:, :warmup])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.rollout(steps, u[:, warmup:warmup + steps])
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kus = sim.time_kernels(kernel_steps, u[:, warmup + steps:])
    status = sim.status()
    sim.close()
    n = sum(sc.n_fluid for sc in scs)
    g = sum(sc.n_ghost for sc in scs)
    nc = sum(n_cells_of(sc) for sc in scs)
    return {"tanks": n_tanks, "n_fluid": n, "n_ghost": g, "steps": steps, "lanes": lanes, "near_lists": near,
            "value": n * steps / (ms / 1e3), "unit": "particle-steps/s", "ms_per_step": ms / steps,
            "status": status, "kernel_us": {k: round(v, 3) for k, v in kus.items()},
            "roofline": kernel_roofline(kus, n, g, nc)}


def paper_leg(relax_cycles: int = 60, relax_steps: int = 50, max_steps: int = 0):
    """The paper's benchmark (Tables 1-2: 666 particles spawned at random in a
    circular tank, relaxed to rest, linear EOS without tension, dt = 1 ms, PD
    attitude law at 0.05 s) flying the two reconstructed manoeuvres (60 s and
    40 s, 60,000 and 40,000 steps), each timed from the relaxed state: the
    like-for-like counterpart of the SPH rows of the paper's Table 3."""
    import torch
    import workloads as W
    from paper_2604_12505_amd.sph import Simulator, gamma1_estimate
    from paper_2604_12505_amd.surrogate import _relax
    sc = W.paper_p0(seed=0, n_steps=1, spawn="random")
    dev = torch.device("cuda:0")
    sim = Simulator.from_scenario(sc, device=dev)
    _relax(sim, relax_cycles, relax_steps)
    s0, w0, _, _, _ = sim.get_state()
    g1 = gamma1_estimate(sc.params, s0, sc.ghosts, device=dev)      # eq. gamma1 at the relaxed state
    per = sc.params.ctrl_period
    out = {"workload": f"paper Tables 1-2: {sc.n_fluid} fluid + {sc.n_ghost} boundary particles, random spawn "
                       f"relaxed for {relax_cycles} x {relax_steps} steps, 1 ms steps",
           "gamma1_estimate_relaxed": g1, "gamma1_used": sc.params.gamma1,
           "paper_hardware": "i7-13850HX + RTX 2000 Ada laptop, JAX", "profiles": {}}
    for k, paper_s in ((1, 9.9093), (2, 5.1876)):
        force, ref = W.manoeuvre_profile(k, ts=per * sc.params.dt)
        n = force.shape[0] * per
        if max_steps > 0:
            n = min(n, max_steps)
        u = np.zeros((n, 3), np.float32)
        u[:, :2] = np.repeat(force, per, axis=0)[:n]
        uu = torch.as_tensor(u, device=dev)
        th = torch.as_tensor(ref, dtype=torch.float64, device=dev)
        res = {"steps": n, "paper_wall_s": paper_s}
        for name, resident in (("multi_kernel", False), ("lds_resident", True)):
            sim.set_state(s0, w0, np.zeros(6), 0.0, 0)
            sim.rollout(64, uu[:64].contiguous(), theta_ref=th, resident=resident)   # warm-up, graphs captured
            sim.set_state(s0, w0, np.zeros(6), 0.0, 0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lg = sim.rollout(n, uu, theta_ref=th, log_stride=per, resident=resident)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            y = lg["y"].cpu().numpy()
            res[name] = {"wall_s": wall, "status": sim.status(), "final_theta_deg": float(np.degrees(y[-1, 2])),
                         "final_rdot": [float(y[-1, 3]), float(y[-1, 4])]}
        res["status"] = res["multi_kernel"]["status"] | res["lds_resident"]["status"]
        out["profiles"][str(k)] = res
    sim.close()
    # many copies of the scenario at once (Monte Carlo use): 256 tanks from
    # different random spawns, profile 1's first 4,000 steps, both paths
    n_b, steps_b = 256, (min(4000, max_steps) if max_steps > 0 else 4000)
    scs = [W.paper_p0(seed=s, n_steps=1, spawn="random") for s in range(n_b)]
    bsim = Simulator.batch(scs, device=dev)
    _relax(bsim, 10, relax_steps)
    sb0, wb0, _, _, _ = bsim.get_state()
    force, ref = W.manoeuvre_profile(1, ts=per * sc.params.dt)
    u = np.zeros((steps_b, 3), np.float32)
    u[:, :2] = np.repeat(force, per, axis=0)[:steps_b]
    ub = torch.as_tensor(np.broadcast_to(u, (n_b, steps_b, 3)).copy(), device=dev)
    refb = np.broadcast_to(ref, (n_b, ref.size)).copy()
    n_part = sum(x.n_fluid for x in scs)
    batch = {"tanks": n_b, "steps": steps_b, "particles": n_part}
    for name, resident in (("multi_kernel", False), ("lds_resident", True)):
        bsim.set_state(sb0, wb0, np.zeros((n_b, 6)), 0.0, 0)
        bsim.rollout(64, ub[:, :64].contiguous(), theta_ref=refb, resident=resident)
        bsim.set_state(sb0, wb0, np.zeros((n_b, 6)), 0.0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bsim.rollout(steps_b, ub, theta_ref=refb, resident=resident)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        batch[name] = {"wall_s": wall, "particle_steps_per_s": n_part * steps_b / wall, "status": bsim.status()}
    bsim.close()
    out["batch_256_tanks"] = batch
    return out


def sweep_leg(ks=(0, 1, 2, 3, 4, 5, 6), steps: int = 200, warmup: int = 40, kernel_steps: int = 16):
    """The rectangular tank refined by 2^k in spacing (N = 1,600 x 4^k fluid
    particles, up to 6.55M at k = 6), prescribed sine rotation, autotuned:
    particle-steps/s and the roofline of the dominant kernel per size.  At
    k = 5 the working set still fits the 256 MB last-level cache, at k = 6 it
    does not."""
    import torch
    import workloads as W
    from paper_2604_12505_amd.sph import Simulator
    dev = torch.device("cuda:0")
    rows = []
    for k in ks:
        sc = W.rect_sweep(k, seed=0, n_steps=warmup + steps + kernel_steps)
        sim = Simulator.from_scenario(sc, device=dev)
        lanes = sim.autotune(reps=3 if k >= 5 else 10)
        near = sim.tuning()[1]
        sim.rollout(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.rollout(steps)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        kus = sim.time_kernels(kernel_steps)
        rows.append({"k": k, "n_fluid": sc.n_fluid, "n_ghost": sc.n_ghost, "lanes": lanes, "near_lists": near,
                     "ms_per_step": ms, "particle_steps_per_s": sc.n_fluid / (ms / 1e3), "status": sim.status(),
                     "kernel_us": {q: round(v, 2) for q, v in kus.items()},
                     "roofline": kernel_roofline(kus, sc.n_fluid, sc.n_ghost, n_cells_of(sc), lanes, near)})
        sim.close()
        progress(f"sweep k={k}: {sc.n_fluid} particles, {ms:.3f} ms per step")
    return {"workload": "rect_sweep: rectangle 1.0 x 0.5 m, 50 % fill, dx = 12.5 mm / 2^k, sine rotation",
            "steps": steps, "rows": rows}


def surrogate_leg(n_train: int = 192, n_test: int = 32, steps: int = 2000, epochs: int = 30):
    """The wrench surrogate end to end at reduced size: relaxed, forced
    random tanks (2k-8k particles, the Tait law without tension) from the SPH
    kernels, windows, MFMA training, held-out NRMSE beside the training-mean
    predictor, and the network's time for the held-out windows against the
    SPH time that produced them (the full-size run is train_surrogate.py)."""
    import torch
    from paper_2604_12505_amd import surrogate as S
    kw = dict(n_steps=steps, log_stride=25, relax_cycles=10, relax_steps=100, n_min=2000, n_max=8000)
    tr = S.generate(list(range(1000, 1000 + n_train)), **kw)
    te = S.generate(list(range(900000, 900000 + n_test)), **kw)
    norm = S.norm_from(tr)
    xtr, ytr = S.windows(tr, norm)
    xte, yte = S.windows(te, norm)
    net = S.train(xtr, ytr, epochs=epochs, batch=1024, lr=2e-3, lr_final=1e-4)
    inf = S.inference_net(net, max_batch=65536)
    err = S.nrmse(S.predict(inf, xte), yte, norm)
    base = S.nrmse(torch.zeros_like(yte), yte, norm)
    t_nn = S.time_inference(inf, xte)
    net.close()
    inf.close()
    return {"workload": f"{n_train} training / {n_test} held-out random tanks (2k-8k particles), {steps} steps, "
                        f"log stride 25, window 32, {epochs} epochs",
            "nrmse": [float(v) for v in err], "nrmse_mean_predictor": [float(v) for v in base],
            "heldout_windows": int(xte.shape[0]), "nn_seconds": t_nn, "sph_seconds": te.sph_seconds,
            "speedup": te.sph_seconds / t_nn}


def lpv_leg():
    """The LPV surrogate kernels at the paper's identification size (2,200
    samples): one loss + gradient evaluation for 8 models (the paper's
    restart count) and for 4,096 at once, 100 Adam iterations of 8 models,
    and 16,384 closed-loop runs of manoeuvre 1 in one launch."""
    import torch
    import workloads as W
    from paper_2604_12505_amd import lpv as L
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(0)
    n = 2200
    u = torch.as_tensor(W.lpv_input_train(0, n) / 40.0, device=dev)
    y = torch.as_tensor(rng.normal(size=(n, 3)) * 0.1, device=dev)
    out = {"workload": f"LPV-SS (n_x 4, n_u 3, n_y 3, 2x4 tanh scheduling), {n} samples"}

    def models(R):
        V = rng.normal(size=(R, L.N_PARAM)) * 0.1
        V[:, :16] = np.tile((0.95 * np.eye(4)).ravel(), (R, 1))
        return torch.as_tensor(V, device=dev)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    for R in (8, 4096):
        P = models(R)
        ws = L.workspace(R, n, dev)
        out[f"loss_grad_ms_{R}_models"] = 1e3 * timed(lambda: L.loss_grad(P, u, y, ws=ws), 5)
    P = models(8)
    ws = L.workspace(8, n, dev)
    out["adam_ms_per_iteration_8_models"] = 1e3 * timed(lambda: L.adam(P, u, y, 100, ws=ws), 1) / 100
    force, ref = W.manoeuvre_profile(1)
    Pc = models(16384)
    refs = torch.as_tensor(np.broadcast_to(ref, (16384, ref.size)).copy(), device=dev)
    fc = torch.as_tensor(force, device=dev)
    secs = timed(lambda: L.closed_loop(Pc, fc, refs, W.LPV_TS, 50.0, 30.0, [40.0] * 3, [0.1] * 3), 3)
    out["closed_loop_16384_runs_ms"] = 1e3 * secs
    out["closed_loop_runs_per_s"] = 16384 / secs
    return out


def linearization_leg(n_dir: int = 64, steps: int = 400):
    """Linearizations on a rectangular tank of ~8,000 particles over `steps`
    steps: the tangent-linear rollout along n_dir directions (input torque
    sequence and initial rigid state; the gradient of the final slosh torque
    with respect to all 400 torques and 6 initial rigid-state entries would
    take 406 of them), and the same gradient from one adjoint rollout."""
    import torch
    import workloads as W
    from paper_2604_12505_amd.sph import Simulator
    sc = W.linearization_tank(seed=0, n_steps=steps + 40)
    dev = torch.device("cuda:0")
    sim = Simulator.from_scenario(sc, device=dev)
    u = torch.as_tensor(sc.u_seq)
    sim.rollout(40, u[:40].contiguous())
    rng = np.random.default_rng(0)
    du = (rng.normal(size=(n_dir, steps, 3)) * 10.0).astype(np.float32)
    dr = rng.normal(size=(n_dir, 6)) * 0.01
    sim.jvp_rollout(8, u[40:48].contiguous(), du[:, :8].copy(), None, dr)   # warm-up
    t0 = time.perf_counter()
    sim.jvp_rollout(steps, u[40:40 + steps].contiguous(), du, None, dr)
    secs = time.perf_counter() - t0
    # the whole gradient of the final slosh torque in one adjoint rollout,
    # the state kept every 20 steps
    sim.vjp_rollout(8, [0.0, 0.0, 1.0], u[40:48].contiguous(), every=20)   # warm-up
    t0 = time.perf_counter()
    sim.vjp_rollout(steps, [0.0, 0.0, 1.0], u[40:40 + steps].contiguous(), every=20)
    adj = time.perf_counter() - t0
    n = sc.n_fluid
    sim.close()
    return {"workload": f"linearization_tank: rectangle 1.0 x 0.5 m, 50 % fill, {n} fluid + {sc.n_ghost} "
                        f"boundary particles, free body, {steps} steps",
            "directions": n_dir, "seconds": secs,
            "direction_particle_steps_per_s": n_dir * steps * n / secs,
            "gradient_by_tangents_s": secs * (steps + 6) / n_dir,
            "adjoint_gradient_s": adj, "adjoint_checkpoint_every": 20}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--cpu-steps", type=int, default=6000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-steps", type=int, default=200)
    ap.add_argument("--dx", type=float, default=0.004)
    ap.add_argument("--batch-tanks", type=int, default=256,
                    help="tanks of the batched leg (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--no-paper-leg", action="store_true")
    ap.add_argument("--no-linearization-leg", action="store_true")
    ap.add_argument("--no-lpv-leg", action="store_true")
    ap.add_argument("--no-sweep-leg", action="store_true")
    ap.add_argument("--no-surrogate-leg", action="store_true")
    ap.add_argument("--sweep-only", action="store_true", help="run only the size sweep")
    ap.add_argument("--paper-only", action="store_true", help="run only the paper-scenario leg")
    ap.add_argument("--paper-steps", type=int, default=0, help="cap on the paper leg's steps per run (0: full)")
    ap.add_argument("--lanes", type=int, default=0,
                    help="lanes per particle of the closed-loop leg (0: sph_autotune chooses)")
    ap.add_argument("--near-lists", type=int, default=-1,
                    help="near lists on (1) or off (0) with --lanes (-1: off); with --batch-only they apply to the batch")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched leg and print its JSON object (profiling)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (HBM-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        return 2

    import torch
    import workloads as W
    from paper_2604_12505_amd.sph import Simulator

    if args.calibrate_copy_mb > 0:
        n = args.calibrate_copy_mb * (1 << 20) // 4
        src = torch.ones(n, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.sweep_only:
        res = sweep_leg()
        print(json.dumps(res))
        return 0 if all(r["status"] == 0 for r in res["rows"]) else 1
    if args.paper_only:
        res = paper_leg(max_steps=args.paper_steps)
        print(json.dumps(res))
        ok = all(p["status"] == 0 for p in res["profiles"].values())
        return 0 if ok else 1
    if args.batch_only:
        res = batch_leg(args.batch_tanks, args.batch_steps, 16, 16, args.lanes, args.near_lists)
        print(json.dumps(res))
        return 0 if res["status"] == 0 else 1

    total = args.warmup + args.steps + args.kernel_steps
    sc = W.closed_loop_circle(seed=0, n_steps=total, dx=args.dx)
    dev = torch.device("cuda:0")
    sim = Simulator.from_scenario(sc, device=dev)
    u = torch.as_tensor(sc.u_seq, device=dev)
    ref = torch.as_tensor(sc.theta_ref, dtype=torch.float64, device=dev)
    if args.lanes > 0:
        # a fixed choice (profiler runs, where serialised launches would
        # mislead the autotuner)
        sim.set_lanes(args.lanes)
        sim.set_near_lists(args.near_lists == 1)
        lanes, near = sim.tuning()
    else:
        lanes = sim.autotune(reps=20)
        near = sim.tuning()[1]

    sim.rollout(args.warmup, u[:args.warmup], ref)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.rollout(args.steps, u[args.warmup:args.warmup + args.steps], ref)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    status = sim.status()
    value = sc.n_fluid * args.steps / (ms / 1e3)

    # per-kernel durations, HIP events around each kernel of directly launched steps
    kus = sim.time_kernels(args.kernel_steps, u[args.warmup + args.steps:], ref)
    status |= sim.status()
    roofline = kernel_roofline(kus, sc.n_fluid, sc.n_ghost, n_cells_of(sc), lanes, near,
                               traffic_workload="closed_loop_circle" if args.dx == 0.004 else None)
    sim.close()

    out = {
        "metric": "SPH particle-steps/s at 1 GPU (% HBM roofline); NN vs SPH speedup at <=2% err",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"closed_loop_circle: R 0.5 m, fill 0.3, dx {sc.dx * 1e3:g} mm, "
                               f"{sc.n_fluid} fluid + {sc.n_ghost} boundary particles, PD slew",
                   "n_fluid": sc.n_fluid, "n_ghost": sc.n_ghost, "dt": sc.params.dt,
                   "lanes_per_particle": lanes, "near_lists": near, "parallelism": "single GPU"},
        "status": status,
        "kernel_us": {k: round(v, 3) for k, v in kus.items()},
        "roofline": roofline,
    }
    progress("closed-loop tank measured")
    if not args.no_paper_leg:
        # the paper's own scenario (timing context for its Table 3)
        out["paper_scenario"] = paper_leg(max_steps=args.paper_steps)
        progress("paper scenario leg done")
        for prof in out["paper_scenario"]["profiles"].values():
            status |= prof["status"]
    if args.batch_tanks > 0:
        out["batch"] = batch_leg(args.batch_tanks, args.batch_steps, 16, 16)
        status |= out["batch"]["status"]
        progress("batch leg done")
    if not args.no_linearization_leg:
        out["linearization"] = linearization_leg()
        progress("linearization leg done")
    if not args.no_lpv_leg:
        out["lpv"] = lpv_leg()
        progress("LPV leg done")
    if not args.no_surrogate_leg:
        out["surrogate"] = surrogate_leg()
        progress("surrogate leg done")
    if not args.no_sweep_leg:
        out["size_sweep"] = sweep_leg()
        for r in out["size_sweep"]["rows"]:
            status |= r["status"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_steps)
        progress("CPU baseline done")
    print(json.dumps(out))
    return 0 if status == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
