"""Trains the slosh-wrench surrogate on SPH rollouts and measures it.

    python -m paper_2604_12505_amd.train_surrogate --train 4096 --test 512 --out result.json

Generates training and held-out rollouts with the random-tank generator
(relaxed, then forced by a multisine torque), trains the MLP with the
library's MFMA kernels and reports, on the held-out set, the per-channel
wrench NRMSE, the SPH noise floor (the held-out tanks are simulated a second
time with another initial jitter and nothing else changed; the floor is the
NRMSE between the two sets) and the speedup: GPU time of the SPH rollouts
that produced the held-out samples (the tanks advanced together, relaxation
excluded) over the network's time for the same samples in batches of 65,536
windows.  Then the held-out rollouts again with the rigid body driven by the
network instead of SPH from the first full window on (the same inputs): the
trajectory NRMSE against SPH per rigid-body channel, next to the same with
the fluid's mean wrench and between the two SPH sets, and that run's time
against SPH's.  The window's inputs are theta, thetadot and the input torque and,
in the fourth channel, the tank's constants (--static 3: fill, shape,
spacing; --static 1: the fill ratio alone, the configured window).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import surrogate as S


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--test", type=int, default=512)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--stride", type=int, default=25)
    ap.add_argument("--relax-cycles", type=int, default=40)
    ap.add_argument("--relax-steps", type=int, default=100)
    ap.add_argument("--n-min", type=int, default=2000)
    ap.add_argument("--n-max", type=int, default=60000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tanks-per-launch", type=int, default=256)
    ap.add_argument("--literal-tait", action="store_true",
                    help="data with the Tait law as written (negative pressures allowed)")
    ap.add_argument("--static", type=int, default=3, help="per-tank constants in the window (1: fill only)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)

    t0 = time.time()
    train_seeds = list(range(1000, 1000 + a.train))
    test_seeds = list(range(900000, 900000 + a.test))
    import workloads as W
    kw = dict(n_steps=a.steps, log_stride=a.stride, relax_cycles=a.relax_cycles,
              relax_steps=a.relax_steps, n_min=a.n_min, n_max=a.n_max,
              eos=W.EOS_TAIT if a.literal_tait else W.EOS_TAIT_CLAMPED)
    log(f"generating {a.train} training rollouts")
    tr = S.generate(train_seeds, batch=a.tanks_per_launch, log=log, **kw)
    log(f"generating {a.test} held-out rollouts")
    te = S.generate(test_seeds, batch=a.tanks_per_launch, log=log, jitter_seed=1, **kw)
    log(f"generating the {a.test} held-out rollouts again with another jitter")
    te2 = S.generate(test_seeds, batch=a.tanks_per_launch, log=log, jitter_seed=2, **kw)
    floor = S.noise_floor(te, te2)
    norm = S.norm_from(tr, a.static)
    xtr, ytr = S.windows(tr, norm)
    xte, yte = S.windows(te, norm)
    log(f"windows: train {xtr.shape[0]}, held-out {xte.shape[0]}")
    net = S.train(xtr, ytr, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
    net = S.inference_net(net, 65536)
    pred = S.predict(net, xte, 65536)
    err = S.nrmse(pred, yte, norm)
    base = S.nrmse(torch.zeros_like(yte), yte, norm)      # the training-mean predictor
    n_win = xte.shape[0]
    t_nn = 0.0
    for b in range(0, n_win, 65536):
        t_nn += S.time_inference(net, xte[b:b + 65536].contiguous())
    S.coupled(net, te, norm)                                # warm-up
    cpl = S.coupled(net, te, norm)
    const = S.constant_net(norm, max_batch=max(64, a.test))
    e_nn = S.trajectory_nrmse(cpl["y"], te)
    e_c = S.trajectory_nrmse(S.coupled(const, te, norm)["y"], te)
    e_b = S.trajectory_nrmse(te2.y, te)
    const.close()
    ch = S.TRAJ_CHANNELS
    res = {
        "train_rollouts": a.train, "test_rollouts": a.test, "steps": a.steps, "log_stride": a.stride,
        "eos": "tait" if a.literal_tait else "tait_clamped",
        "relax": [a.relax_cycles, a.relax_steps], "epochs": a.epochs, "batch": a.batch,
        "train_windows": int(xtr.shape[0]), "test_windows": int(n_win),
        "static_inputs": a.static,
        "nrmse": [float(v) for v in err], "nrmse_max": float(np.max(err)),
        "sph_noise_floor": [float(v) for v in floor],
        "below_noise_floor": bool(np.all(err <= floor)),
        "nrmse_mean_predictor": [float(v) for v in base],
        "sph_seconds_heldout": te.sph_seconds,
        "sph_particle_steps_heldout": int(te.n_fluid.sum()) * a.steps,
        "nn_seconds_heldout": t_nn,
        "speedup": te.sph_seconds / t_nn if t_nn > 0 else None,
        "nn_windows_per_s": n_win / t_nn if t_nn > 0 else None,
        "coupled": {"trajectory_nrmse": dict(zip(ch, (float(v) for v in e_nn))),
                    "mean_wrench_nrmse": dict(zip(ch, (float(v) for v in e_c))),
                    "sph_vs_sph_nrmse": dict(zip(ch, (float(v) for v in e_b))),
                    "out_of_range_rollouts": int((cpl["flags"] & 1).sum().item()),
                    "seconds": cpl["seconds"], "speedup": te.sph_seconds / cpl["seconds"]},
        "wall_seconds": time.time() - t0,
    }
    log(json.dumps(res))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
