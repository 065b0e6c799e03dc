"""Writes adjoint_400_fd.npz: the FP64 oracle's central differences of the
final slosh wrench along 32 random directions of the adjoint workload (the
~8,000-particle rectangular tank, 400 steps after a 40-step lead-in), from
the lead-in state and from MEMBERS copies of it perturbed at binary32
rounding level (every position and velocity times 1 + 2^-24 u, u uniform in
[-1, 1]).  Past ~100 steps this system's derivative depends on where the
trajectory goes; the spread of the members' derivatives around the
unperturbed one is what a rounding-level change of the trajectory does to
it, set against how far their trajectories end from the unperturbed one
(final positions of the runs with the unperturbed input are stored too):
the reference the GPU test's bound is derived from.  (Rounding the
oracle's state at every step, ora_set_round_f32, does not give a usable
reference here: the central differences of a rounded run are dominated by
the rounding itself, hundreds of times the derivative.)

Calls only oracle/ and workloads/ (no GPU code).  Run from the repository
root:  python tests/golden/make_adjoint_fd.py   (a few minutes)."""
from __future__ import annotations

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import sph as O  # noqa: E402

STEPS, LEAD, K, EPS, SEED, MEMBERS = 400, 40, 32, 1e-3, 8, 4
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_400_fd.npz")


def directions():
    """The 32 directions: input sequences du [K, STEPS, 3] (binary32) and
    initial rigid-state perturbations dr [K, 6]."""
    rng = np.random.default_rng(SEED)
    du = (rng.normal(size=(K, STEPS, 3)) * 10.0).astype(np.float32)
    dr = rng.normal(size=(K, 6)) * 0.01
    return du, dr


def lead_in(sc):
    st = O.state_from_scenario(sc)
    status, _ = O.rollout(sc.params, st, sc.ghosts.astype(np.float64), LEAD, sc.u_seq[:LEAD], sc.theta_ref)
    assert status == 0
    st.s = st.s.astype(np.float32).astype(np.float64)
    st.w = st.w.astype(np.float32).astype(np.float64)
    return st


def final_wrench(sc, ck, u, rigid):
    st = O.State(ck.s.copy(), ck.w.copy(), np.asarray(rigid, np.float64).copy(), ck.tau_ctrl, ck.step)
    _, lg = O.rollout(sc.params, st, sc.ghosts.astype(np.float64), u.shape[0], u, sc.theta_ref, log_stride=1)
    return lg["wrench"][-1], st.rigid


def main():
    sc = W.linearization_tank(seed=0, n_steps=STEPS + LEAD)
    ck = lead_in(sc)
    u = sc.u_seq[LEAD:LEAD + STEPS].astype(np.float64)
    du, dr = directions()
    prng = np.random.default_rng(12345)
    starts = [ck]
    for _ in range(MEMBERS):
        m = O.State(ck.s * (1.0 + 2.0 ** -24 * prng.uniform(-1, 1, ck.s.shape)),
                    ck.w * (1.0 + 2.0 ** -24 * prng.uniform(-1, 1, ck.w.shape)), ck.rigid.copy(), ck.tau_ctrl,
                    ck.step)
        starts.append(m)
    fw = np.zeros((MEMBERS + 1, K, 3))
    fr = np.zeros((MEMBERS + 1, K, 6))
    t0 = time.time()
    for q, st in enumerate(starts):
        for k in range(K):
            wp, rp = final_wrench(sc, st, u + EPS * du[k], st.rigid + EPS * dr[k])
            wm, rm = final_wrench(sc, st, u - EPS * du[k], st.rigid - EPS * dr[k])
            fw[q, k] = (wp - wm) / (2 * EPS)
            fr[q, k] = (rp - rm) / (2 * EPS)
            print(f"start {q} direction {k}: dwrench {fw[q, k]} ({time.time() - t0:.0f} s)", flush=True)
    # final fluid positions of the unperturbed-input runs: how far the
    # members' trajectories end from the lead-in state's (the derivative's
    # spread is set against this distance)
    finals = []
    for st in starts:
        run = O.State(st.s.copy(), st.w.copy(), st.rigid.copy(), st.tau_ctrl, st.step)
        O.rollout(sc.params, run, sc.ghosts.astype(np.float64), STEPS, u, sc.theta_ref)
        finals.append(run.s)
    finals = np.stack(finals)
    np.savez(OUT, steps=STEPS, lead=LEAD, eps=EPS, seed=SEED, n_fluid=sc.n_fluid,
             du_sum=float(np.abs(du).astype(np.float64).sum()), dwrench=fw[0], drigid=fr[0],
             dwrench_members=fw[1:], drigid_members=fr[1:], s_final=finals[0], s_final_members=finals[1:])
    print("wrote", OUT)


if __name__ == "__main__":
    main()
