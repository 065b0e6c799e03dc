#!/usr/bin/env python
"""Benchmark of the coupled SPH sloshing step on one MI355X.

Headline workload: 256 independent tanks advanced together in the same
launches (rectangular 1.0 x 0.5 m or circular R = 0.5 m by the seed, fill
U[0.2, 0.8], 2k-60k fluid particles each, 7,722,150 fluid + 730,107
boundary particles in all; Tait EOS, gamma 7, c0 = 20 m/s, h = 1.3 dx,
dt = 0.2 h / c0 per tank; spacecraft 1000 kg, 500 kg m^2, free body under a
5-tone random multisine torque).  A step is one pass of the whole step for
every tank (cell list, density/EOS, forces, slosh wrench, rigid body,
fictitious accelerations, integrator); the timed region is one rollout of
--steps steps replayed from HIP graphs, inputs resident in HBM.

Prints one JSON line: fluid particle-steps/s of the batch, the roofline
position of its dominant kernel (HIP-event kernel times measured in this
run), the FP64 oracle timed on the host on a bounded sample of the same
tanks, and the other workloads as extra keys (the batch's full 5,000-step
run, the closed-loop circular tank and its 44k variant, the paper's
scenario, the size sweep, linearizations, the LPV and MLP surrogates).
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


# The same for the 256-tank batch (4 lanes per particle, near lists: the
# autotuner's choice there), from the counter runs of
# profiles/hbm_traffic_batch_256_random_tanks.md.
TRAFFIC_BATCH = {"src_sha1": "b7ecaf84fe2e8bd058b904413ea6024a5e35a7ba",
                 "bytes_per_launch": {"sph_force/4/1": 1567141121, "sph_density/4/1": 1664766378}}

# The binding ceiling of the step (VALU issue, each unordered fluid pair
# evaluated once): about 590 issue slots per fluid particle-step against
# 3.93e13 lane-operations/s, 6.7e10 particle-steps/s; the straightforward
# gather that evaluates every pair from both sides costs about 1,580 slots,
# 2.5e10 particle-steps/s.
BINDING_CEILING = 6.7e10
GATHER_CEILING = 2.5e10


def progress(msg: str) -> None:
    """A progress line on stderr (stdout carries the one JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def src_hash() -> str:
    h = hashlib.sha1()
    with open(os.path.join(ROOT, "paper_2604_12505_amd", "csrc", "sph.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def host_info() -> dict:
    """The host the CPU baseline ran on: logical CPUs, the CPUs this process
    may use, and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "logical_cpus": os.cpu_count(), "cpu_model": model,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(seeds=(0, 1, 2), n_steps: int = 200, n_steps_1t: int = 20):
    """The FP64 oracle, as it stands, on a bounded sample of the headline
    workload: the first tanks of the 256-tank batch (the same generator and
    seeds), n_steps steps each with OpenMP over particles on every thread it
    gets, and n_steps_1t steps on one thread."""
    import workloads as W
    from oracle import sph as O
    scs = [W.random_tank(seed, n_steps=n_steps) for seed in seeds]
    n_part = sum(sc.n_fluid for sc in scs)

    def run(steps):
        t0 = time.perf_counter()
        for sc in scs:
            st = O.state_from_scenario(sc)
            O.rollout(sc.params, st, sc.ghosts.astype(np.float64), steps, sc.u_seq[:steps])
        return time.perf_counter() - t0

    threads = O.num_threads()
    secs = run(n_steps)
    O.set_num_threads(1)
    secs_1t = run(n_steps_1t)
    O.set_num_threads(threads)
    return {"value": n_part * n_steps / secs, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"tanks {', '.join(str(q) for q in seeds)} of the 256-tank batch ({n_part} fluid particles), "
                      f"{n_steps} steps each, {secs:.1f} s, FP64 C with OpenMP over particles",
            "single_thread": {"value": n_part * n_steps_1t / secs_1t, "unit": "particle-steps/s",
                              "sample": f"the same tanks, {n_steps_1t} steps each, {secs_1t:.1f} s"},
            "host": host_info()}


def kernel_roofline(kus, n_fluid, n_ghost, n_cells, lanes=None, near=None, traffic_workload=None, rate=None):
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
    table = {"closed_loop_circle": TRAFFIC, "batch_256_random_tanks": TRAFFIC_BATCH}.get(traffic_workload)
    traffic = table["bytes_per_launch"].get(key) if table and table["src_sha1"] == src_hash() else None
    hbm = {"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
           "algorithmic_bytes_per_launch": alg_bytes}
    binding = None
    if rate is not None:
        binding = {"ceiling": BINDING_CEILING, "unit": "particle-steps/s", "frac": rate / BINDING_CEILING,
                   "gather_ceiling": GATHER_CEILING, "gather_frac": rate / GATHER_CEILING}
    if dominant in FLOP:
        flops = FLOP[dominant] * n_fluid
        tf = flops / secs / 1e12
        out = {"bound": "alu", "achieved": round(tf, 4), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": tf / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic, "kernel": "sph_" + dominant,
               "algorithmic_flop_per_launch": flops, "launch_us": kus[dominant], "hbm": hbm}
        if binding:
            out["binding_roofline"] = binding
        return out
    return {"bound": "hbm", "achieved": hbm["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": hbm["frac"], "traffic": traffic, "kernel": "sph_" + dominant,
            "algorithmic_bytes_per_launch": alg_bytes, "launch_us": kus[dominant]}


def n_cells_of(sc):
    cell = (2.0 + 1.0) * sc.params.h * (1 + 1e-6)
    return int(np.ceil((sc.params.domain_max[0] - sc.params.domain_min[0]) / cell)) * \
        int(np.ceil((sc.params.domain_max[1] - sc.params.domain_min[1]) / cell))


def batch_leg(n_tanks: int, steps: int, warmup: int, kernel_steps: int, lanes: int = 0, near: int = -1,
              full_steps: int = 0):
    """Many random tanks (rectangular or circular, fill U[0.2, 0.8], 2k-60k
    particles, multisine torque) advanced together in the same launches:
    `steps` steps timed after `warmup`, the kernels timed over
    `kernel_steps` more, and, if full_steps > 0, a separate timed run of
    full_steps steps from the initial state (the workload's full length)."""
    import torch
    import workloads as W
    from paper_2604_12505_amd.sph import Simulator
    total = max(warmup + steps + kernel_steps, full_steps)
    scs = [W.random_tank(seed, n_steps=total) for seed in range(n_tanks)]
    dev = torch.device("cuda:0")
    sim = Simulator.batch(scs, device=dev)
    s0, w0, r0, _, _ = sim.get_state()
    s0, w0 = s0.clone(), w0.clone()
    if lanes > 0:
        sim.set_lanes(lanes)
        sim.set_near_lists(near == 1)
    else:
        sim.autotune(reps=5)
    lanes, near = sim.tuning()
    progress(f"batch: {n_tanks} tanks set up, lanes {lanes}, near lists {near}")
    u = torch.stack([torch.as_tensor(sc.u_seq) for sc in scs]).to(dev)
    sim.rollout(warmup, u[:, :warmup].contiguous())
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.rollout(steps, u[:, warmup:warmup + steps].contiguous())
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    status = sim.status()
    kus = sim.time_kernels(kernel_steps, u[:, warmup + steps:warmup + steps + kernel_steps].contiguous())
    status |= sim.status()
    n = sum(sc.n_fluid for sc in scs)
    g = sum(sc.n_ghost for sc in scs)
    nc = sum(n_cells_of(sc) for sc in scs)
    rate = n * steps / (ms / 1e3)
    out = {"tanks": n_tanks, "n_fluid": n, "n_ghost": g, "steps": steps, "lanes": lanes, "near_lists": near,
           "value": rate, "unit": "particle-steps/s", "ms_per_step": ms / steps,
           "status": status, "kernel_us": {k: round(v, 3) for k, v in kus.items()},
           "roofline": kernel_roofline(kus, n, g, nc, lanes, near, "batch_256_random_tanks" if n_tanks == 256 else None,
                                       rate=rate)}
    progress(f"batch: {steps} steps timed, {ms / steps:.3f} ms per step, status {status}")
    if full_steps > 0:
        sim.set_state(s0, w0, r0, 0.0, 0)
        torch.cuda.synchronize()
        e0.record(sim.stream)
        sim.rollout(full_steps, u[:, :full_steps].contiguous())
        e1.record(sim.stream)
        torch.cuda.synchronize()
        fms = e0.elapsed_time(e1)
        fst = sim.status()
        out["full_run"] = {"steps": full_steps, "from": "initial state", "ms_per_step": fms / full_steps,
                           "value": n * full_steps / (fms / 1e3), "status": fst}
        out["status"] |= fst
        progress(f"batch: full run of {full_steps} steps, {fms / full_steps:.3f} ms per step, status {fst}")
    sim.close()
    return out


def closed_loop_leg(dx: float, steps: int, warmup: int, kernel_steps: int, lanes: int = 0, near: int = -1):
    """The closed-loop circular tank (R 0.5 m, 30 % fill, spacing dx, PD slew):
    one rollout of `steps` graph-replayed steps timed after `warmup`."""
    import torch
    import workloads as W
    from paper_2604_12505_amd.sph import Simulator
    total = warmup + steps + kernel_steps
    sc = W.closed_loop_circle(seed=0, n_steps=total, dx=dx)
    dev = torch.device("cuda:0")
    sim = Simulator.from_scenario(sc, device=dev)
    u = torch.as_tensor(sc.u_seq, device=dev)
    ref = torch.as_tensor(sc.theta_ref, dtype=torch.float64, device=dev)
    if lanes > 0:
        # a fixed choice (profiler runs, where serialised launches would
        # mislead the autotuner)
        sim.set_lanes(lanes)
        sim.set_near_lists(near == 1)
        lanes, near = sim.tuning()
    else:
        lanes = sim.autotune(reps=20)
        near = sim.tuning()[1]
    sim.rollout(warmup, u[:warmup], ref)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.rollout(steps, u[warmup:warmup + steps], ref)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    status = sim.status()
    # per-kernel durations, HIP events around each kernel of directly launched steps
    kus = sim.time_kernels(kernel_steps, u[warmup + steps:], ref)
    status |= sim.status()
    rate = sc.n_fluid * steps / (ms / 1e3)
    roofline = kernel_roofline(kus, sc.n_fluid, sc.n_ghost, n_cells_of(sc), lanes, near,
                               traffic_workload="closed_loop_circle" if dx == 0.004 else None)
    sim.close()
    progress(f"closed loop dx {dx * 1e3:g} mm: {sc.n_fluid} particles, {ms / steps * 1e3:.2f} us per step")
    return {"workload": f"closed_loop_circle: R 0.5 m, fill 0.3, dx {sc.dx * 1e3:g} mm, "
                        f"{sc.n_fluid} fluid + {sc.n_ghost} boundary particles, PD slew",
            "n_fluid": sc.n_fluid, "n_ghost": sc.n_ghost, "dt": sc.params.dt, "steps": steps, "warmup": warmup,
            "lanes_per_particle": lanes, "near_lists": near, "value": rate, "unit": "particle-steps/s",
            "ms_per_step": ms / steps, "status": status, "kernel_us": {k: round(v, 3) for k, v in kus.items()},
            "roofline": roofline}


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
    # dt = 1 ms moves a particle at 1 m/s by a tenth of h per step: the
    # multi-kernel path rebuilds its cell list every 2 steps here (every 4 let
    # a particle outrun the skin late in the 60 s manoeuvre; the LDS-resident
    # path rebuilds at every step)
    sim.set_rebuild_interval(2)
    _relax(sim, relax_cycles, relax_steps)
    s0, w0, _, _, _ = sim.get_state()
    g1 = gamma1_estimate(sc.params, s0, sc.ghosts, device=dev)      # eq. gamma1 at the relaxed state
    per = sc.params.ctrl_period
    out = {"workload": f"paper Tables 1-2: {sc.n_fluid} fluid + {sc.n_ghost} boundary particles, random spawn "
                       f"relaxed for {relax_cycles} x {relax_steps} steps, 1 ms steps",
           "gamma1_estimate_relaxed": g1, "gamma1_used": sc.params.gamma1,
           "paper_hardware": "i7-13850HX + RTX 2000 Ada laptop, JAX", "profiles": {}}
    # profile 1 is timed over the 30 s the paper's Table 3 row covers (its
    # Section 6: below 10 s for a 30 s simulation), and over the whole
    # reconstructed 60 s manoeuvre; profile 2 (duration not stated in the
    # paper) over its reconstructed 40 s
    for key, k, paper_s, secs in (("1", 1, 9.9093, 30.0), ("1_full", 1, None, None), ("2", 2, 5.1876, None)):
        force, ref = W.manoeuvre_profile(k, ts=per * sc.params.dt)
        n = force.shape[0] * per
        if secs is not None:
            n = min(n, int(round(secs / sc.params.dt)))
        if max_steps > 0 and max_steps < n:
            n = max_steps
            paper_s = None   # a shortened run is no like-for-like comparison
        u = np.zeros((n, 3), np.float32)
        u[:, :2] = np.repeat(force, per, axis=0)[:n]
        uu = torch.as_tensor(u, device=dev)
        th = torch.as_tensor(ref, dtype=torch.float64, device=dev)
        res = {"steps": n, "simulated_s": n * sc.params.dt, "paper_wall_s": paper_s}
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
            if paper_s:
                res[name]["speedup_vs_paper"] = paper_s / wall
        res["status"] = res["multi_kernel"]["status"] | res["lds_resident"]["status"]
        out["profiles"][key] = res
    sim.close()
    # many copies of the scenario at once (Monte Carlo use): 256 tanks from
    # different random spawns, profile 1's first 4,000 steps, both paths
    n_b, steps_b = 256, (min(4000, max_steps) if max_steps > 0 else 4000)
    scs = [W.paper_p0(seed=s, n_steps=1, spawn="random") for s in range(n_b)]
    bsim = Simulator.batch(scs, device=dev)
    bsim.set_rebuild_interval(2)
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


def surrogate_leg(n_train: int = 192, n_test: int = 64, steps: int = 2000, epochs: int = 30):
    """The wrench surrogate end to end at reduced size: relaxed, forced
    random tanks (2k-8k particles, the Tait law without tension) from the SPH
    kernels, windows (theta, thetadot, torque and the tank's fill, shape and
    spacing), MFMA training, and on held-out tanks simulated twice (differing
    only in the initial jitter): the network's NRMSE against one set, the SPH
    noise floor (NRMSE between the two sets), the constant predictor, and the
    network's time for the held-out windows against the SPH time that
    produced them.  The speedup at the 2 % error target is reported only if
    every channel meets it (null otherwise); the speedup at the noise floor
    when every channel is below it (the full-size run is train_surrogate.py)."""
    import torch
    from paper_2604_12505_amd import surrogate as S
    kw = dict(n_steps=steps, log_stride=25, relax_cycles=10, relax_steps=100, n_min=2000, n_max=8000)
    tr = S.generate(list(range(1000, 1000 + n_train)), **kw)
    held = list(range(900000, 900000 + n_test))
    te = S.generate(held, jitter_seed=1, **kw)
    te2 = S.generate(held, jitter_seed=2, **kw)
    norm = S.norm_from(tr)
    xtr, ytr = S.windows(tr, norm)
    xte, yte = S.windows(te, norm)
    net = S.train(xtr, ytr, epochs=epochs, batch=1024, lr=2e-3, lr_final=1e-4)
    inf = S.inference_net(net, max_batch=65536)
    err = S.nrmse(S.predict(inf, xte), yte, norm)
    base = S.nrmse(torch.zeros_like(yte), yte, norm)
    floor = S.noise_floor(te, te2)
    t_nn = S.time_inference(inf, xte)
    # the rigid body driven by the network instead of SPH from the first full
    # window on, against SPH's trajectories (set te); the mean wrench as the
    # baseline, the second SPH set as SPH's own spread
    S.coupled(inf, te, norm)                         # warm-up
    cpl = S.coupled(inf, te, norm)
    const = S.constant_net(norm, max_batch=max(64, n_test))
    e_nn = S.trajectory_nrmse(cpl["y"], te)
    e_c = S.trajectory_nrmse(S.coupled(const, te, norm)["y"], te)
    e_b = S.trajectory_nrmse(te2.y, te)
    const.close()
    net.close()
    inf.close()
    speedup = te.sph_seconds / t_nn
    ch = S.TRAJ_CHANNELS
    return {"workload": f"{n_train} training / {n_test} held-out random tanks (2k-8k particles), {steps} steps, "
                        f"log stride 25, window 32 (theta, thetadot, torque; fill, shape, dx), {epochs} epochs",
            "nrmse": [float(v) for v in err], "sph_noise_floor": [float(v) for v in floor],
            "nrmse_mean_predictor": [float(v) for v in base],
            "heldout_windows": int(xte.shape[0]), "nn_seconds": t_nn, "sph_seconds": te.sph_seconds,
            "speedup": speedup,
            "speedup_at_2pct": speedup if bool(np.all(err <= 0.02)) else None,
            "speedup_at_noise_floor": speedup if bool(np.all(err <= floor)) else None,
            "coupled": {"what": "rigid body driven by the network instead of SPH from sample 31 on, same inputs; "
                                "trajectory NRMSE = RMS(run - SPH) / RMS(SPH - SPH at the hand-over)",
                        "trajectory_nrmse": dict(zip(ch, (float(v) for v in e_nn))),
                        "mean_wrench_nrmse": dict(zip(ch, (float(v) for v in e_c))),
                        "sph_vs_sph_nrmse": dict(zip(ch, (float(v) for v in e_b))),
                        "out_of_range_rollouts": int((cpl["flags"] & 1).sum().item()),
                        "seconds": cpl["seconds"], "sph_seconds": te.sph_seconds,
                        "speedup": te.sph_seconds / cpl["seconds"]}}


# MI355X dense BF16 matrix peak (no sparsity)
BF16_MFMA_PEAK_TFLOPS = 2500.0
# multiply-adds per row of the surrogate network: 128x256 + 3 x 256x256 + 256x3
MLP_MACS_PER_ROW = 128 * 256 + 3 * 256 * 256 + 256 * 3


def mlp_leg(batch: int = 65536, train_batch: int = 4096, reps: int = 20):
    """The surrogate network's kernels alone: one fused inference launch on
    `batch` windows (mlp_forward) and one training step on train_batch
    (mlp_train_step: forward with activations kept, backward, Adam), each
    timed with HIP events over `reps` calls on the network's stream, against
    the BF16 matrix-core peak (2 FLOP per multiply-add; a training step is
    counted as 3 forward passes).  Inference is timed as back-to-back
    launches (Mlp.launch); the same through Mlp.forward, which brackets each
    launch with a hand-over between torch's stream and the network's, is
    reported as us_per_forward_call."""
    import torch
    from paper_2604_12505_amd import surrogate as S
    from paper_2604_12505_amd.mlp import Mlp
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    out = {"workload": f"MLP 128-256x4-3 (GELU, BF16 MFMA, FP32 accumulation): inference batch {batch}, "
                       f"training batch {train_batch}"}
    for name, B in (("inference", batch), ("train_step", train_batch)):
        net = Mlp(S.init_params(0), max_batch=B, device=dev)
        x = torch.randn(B, 128, device=dev, generator=gen)
        t = torch.randn(B, 3, device=dev, generator=gen)
        y = torch.empty(B, 3, device=dev)
        call = (lambda: net.launch(x, y)) if name == "inference" else (lambda: net.train_step(x, t, lr=1e-4))

        def timed(fn):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(net.stream)
            for _ in range(reps):
                fn()
            e1.record(net.stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / 1e3 / reps

        net.forward(x, out=y)   # x, y ordered on the network's stream before the back-to-back launches
        secs = timed(call)
        flop = 2.0 * MLP_MACS_PER_ROW * B * (1 if name == "inference" else 3)
        tf = flop / secs / 1e12
        out[name] = {"batch": B, "us_per_call": secs * 1e6, "flop_per_call": flop, "tflops": tf,
                     "mfma_peak_tflops": BF16_MFMA_PEAK_TFLOPS, "frac": tf / BF16_MFMA_PEAK_TFLOPS}
        if name == "inference":
            out[name]["us_per_forward_call"] = timed(lambda: net.forward(x, out=y)) * 1e6
        net.close()
    return out


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
    ap.add_argument("--steps", type=int, default=5000, help="timed steps of the 256-tank batch")
    ap.add_argument("--warmup", type=int, default=100, help="untimed steps before them")
    ap.add_argument("--kernel-steps", type=int, default=16, help="steps of the per-kernel timing")
    ap.add_argument("--full-steps", type=int, default=5000,
                    help="a separate run of the batch over its full length from the initial state (0 skips it)")
    ap.add_argument("--batch-tanks", type=int, default=256)
    ap.add_argument("--closed-loop-steps", type=int, default=20000)
    ap.add_argument("--closed-loop-warmup", type=int, default=1000)
    ap.add_argument("--dx", type=float, default=0.004, help="spacing of the closed-loop tank")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=200, help="oracle steps per sampled tank")
    ap.add_argument("--no-closed-loop-leg", action="store_true")
    ap.add_argument("--no-paper-leg", action="store_true")
    ap.add_argument("--no-linearization-leg", action="store_true")
    ap.add_argument("--no-lpv-leg", action="store_true")
    ap.add_argument("--no-sweep-leg", action="store_true")
    ap.add_argument("--no-surrogate-leg", action="store_true")
    ap.add_argument("--sweep-only", action="store_true", help="run only the size sweep")
    ap.add_argument("--paper-only", action="store_true", help="run only the paper-scenario leg")
    ap.add_argument("--paper-steps", type=int, default=0, help="cap on the paper leg's steps per run (0: full)")
    ap.add_argument("--lanes", type=int, default=0,
                    help="lanes per particle of the batch (or, with --closed-loop-only, of the closed-loop tank); "
                         "0: sph_autotune chooses")
    ap.add_argument("--near-lists", type=int, default=-1,
                    help="near lists on (1) or off (0) with --lanes")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batch (timed steps and kernel timing) and print its JSON object (profiling)")
    ap.add_argument("--closed-loop-only", action="store_true",
                    help="run only the closed-loop tank and print its JSON object (profiling)")
    ap.add_argument("--mlp-only", action="store_true",
                    help="run only the surrogate network's kernel timing and print its JSON object (profiling)")
    ap.add_argument("--no-mlp-leg", action="store_true")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (HBM-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        return 2

    import torch

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
    if args.mlp_only:
        print(json.dumps(mlp_leg()))
        return 0
    if args.closed_loop_only:
        res = closed_loop_leg(args.dx, args.closed_loop_steps, args.closed_loop_warmup, args.kernel_steps,
                              args.lanes, args.near_lists)
        print(json.dumps(res))
        return 0 if res["status"] == 0 else 1
    if args.batch_only:
        res = batch_leg(args.batch_tanks, args.steps, args.warmup, args.kernel_steps, args.lanes, args.near_lists)
        print(json.dumps(res))
        return 0 if res["status"] == 0 else 1

    b = batch_leg(args.batch_tanks, args.steps, args.warmup, args.kernel_steps, args.lanes, args.near_lists,
                  full_steps=args.full_steps)
    status = b["status"]
    out = {
        "metric": "SPH particle-steps/s at 1 GPU (% HBM roofline); NN vs SPH speedup at <=2% err",
        "value": b["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": b["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch_256_random_tanks: {b['tanks']} tanks in the same launches, rectangular "
                               f"1.0 x 0.5 m or circular R 0.5 m by seed, fill U[0.2, 0.8], 2k-60k fluid particles "
                               f"each ({b['n_fluid']} fluid + {b['n_ghost']} boundary), Tait EOS, dt = 0.2 h / c0, "
                               f"free body under 5-tone multisine torques",
                   "tanks": b["tanks"], "n_fluid": b["n_fluid"], "n_ghost": b["n_ghost"],
                   "lanes_per_particle": b["lanes"], "near_lists": b["near_lists"], "parallelism": "single GPU"},
        "status": status,
        "kernel_us": b["kernel_us"],
        "roofline": b["roofline"],
    }
    if "full_run" in b:
        out["batch_full_run"] = b["full_run"]
    if not args.no_closed_loop_leg:
        out["closed_loop"] = closed_loop_leg(args.dx, args.closed_loop_steps, args.closed_loop_warmup, 200)
        out["closed_loop_44k"] = closed_loop_leg(0.002314, args.closed_loop_steps, args.closed_loop_warmup, 200)
        status |= out["closed_loop"]["status"] | out["closed_loop_44k"]["status"]
    if not args.no_paper_leg:
        # the paper's own scenario (timing context for its Table 3)
        out["paper_scenario"] = paper_leg(max_steps=args.paper_steps)
        progress("paper scenario leg done")
        for prof in out["paper_scenario"]["profiles"].values():
            status |= prof["status"]
    if not args.no_linearization_leg:
        out["linearization"] = linearization_leg()
        progress("linearization leg done")
    if not args.no_lpv_leg:
        out["lpv"] = lpv_leg()
        progress("LPV leg done")
    if not args.no_mlp_leg:
        out["mlp"] = mlp_leg()
        progress("MLP kernel leg done")
    if not args.no_surrogate_leg:
        out["surrogate"] = surrogate_leg()
        progress("surrogate leg done")
    if not args.no_sweep_leg:
        out["size_sweep"] = sweep_leg()
        for r in out["size_sweep"]["rows"]:
            status |= r["status"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n_steps=args.cpu_steps)
        progress("CPU baseline done")
    out["status"] = status
    print(json.dumps(out))
    return 0 if status == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
