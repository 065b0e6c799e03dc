"""The LDS-resident rollout (sph_rollout_resident) against the FP64 oracle
and against the multi-kernel path, through the C ABI.

Same bars as tests/test_gpu_sph.py (binary32 kernels vs a binary64
oracle): 50-step positions within 1e-3 of the tank size, theta within
1e-3 rad, logged rigid outputs within 1e-3, the logged wrench within 1e-4
of the sum of the wall-term magnitudes.  Runs of the same tank are bitwise
identical, alone or in a batch; a resident rollout hands a consistent state
to the multi-kernel path and back.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402
from oracle import sph as O  # noqa: E402

pytestmark = pytest.mark.gpu

SCENARIOS = {
    "paper_p0": lambda: W.paper_p0(0, n_steps=50),
    "paper_p0_random_literal_eos": lambda: W.paper_p0(1, n_steps=50, spawn="random", eos=W.EOS_LINEAR),
    "lpv_tank": lambda: _with_u(W.lpv_tank(0), 50, 40.0),
    "small_circle_pd": lambda: W.closed_loop_circle(0, n_steps=50, dx=0.02),
    "small_rect_sine": lambda: W.plain_rect(0, n_steps=50, dx=0.025),
}


def _with_u(sc, n, amp):
    rng = np.random.default_rng(7)
    sc.n_steps = n
    sc.u_seq = (rng.normal(size=(n, 3)) * [amp, amp, amp / 10]).astype(np.float32)
    return sc


def _sim(sc):
    from paper_2604_12505_amd.sph import Simulator
    return Simulator.from_scenario(sc)


@pytest.mark.parametrize("name", list(SCENARIOS))
def test_resident_trajectory_matches_oracle(name):
    sc = SCENARIOS[name]()
    sim = _sim(sc)
    assert sim.resident_fits()
    n = 50
    u = sc.u_seq[:n]
    logs = sim.rollout(n, torch.as_tensor(u), theta_ref=sc.theta_ref, log_stride=10, resident=True)
    s, w, rig, tau, step = sim.get_state()
    assert step == n and sim.status() == 0
    st = O.state_from_scenario(sc)
    _, ol = O.rollout(sc.params, st, sc.ghosts.astype(np.float64), n, u, sc.theta_ref, log_stride=10)
    err = np.sqrt(((s.cpu().numpy().astype(np.float64) - st.s) ** 2).sum(1)).max()
    print(name, "pos err / L", err / sc.tank_size, "theta err", abs(rig[2] - st.rigid[2]))
    assert err <= 1e-3 * sc.tank_size
    assert abs(rig[2] - st.rigid[2]) <= 1e-3
    assert np.abs(logs["y"].cpu().numpy() - ol["y"]).max() <= 1e-3
    assert np.allclose(logs["u"].cpu().numpy(), ol["u"], rtol=1e-5, atol=1e-3)
    scale = np.abs(O.rhs(sc.params, O.state_from_scenario(sc), sc.ghosts.astype(np.float64))["wall_terms"]).sum(0)
    wl = logs["wrench"].cpu().numpy()
    assert (np.abs(wl[0] - ol["wrench"][0]) / np.maximum(scale, 1e-12)).max() <= 1e-4
    sim.close()


def test_resident_is_deterministic_and_batch_equals_single():
    scs = [W.paper_p0(s, n_steps=120, spawn="random") for s in range(3)] + [_with_u(W.lpv_tank(1), 120, 40.0)]
    from paper_2604_12505_amd.sph import Simulator
    singles = []
    for sc in scs:
        outs = []
        for _ in range(2):
            sim = _sim(sc)
            sim.rollout(120, torch.as_tensor(sc.u_seq[:120]), theta_ref=sc.theta_ref, resident=True)
            outs.append(sim.get_state())
            assert sim.status() == 0
            sim.close()
        assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
        singles.append(outs[0])
    b = Simulator.batch(scs)
    u = torch.stack([torch.as_tensor(sc.u_seq[:120]) for sc in scs])
    n_ref = max(len(sc.theta_ref) for sc in scs)
    ref = np.stack([np.pad(sc.theta_ref, (0, n_ref - len(sc.theta_ref)), mode="edge") for sc in scs])
    b.rollout(120, u, theta_ref=ref, resident=True)
    s, w, rig, _, _ = b.get_state()
    assert b.status() == 0
    o = 0
    for t, sc in enumerate(scs):
        n = sc.n_fluid
        assert torch.equal(s[o:o + n], singles[t][0]) and torch.equal(w[o:o + n], singles[t][1])
        assert np.array_equal(rig[t], singles[t][2])
        o += n
    b.close()


def test_resident_and_multikernel_paths_hand_over():
    # 30 resident steps, 40 multi-kernel steps (graph-replayed), 30 resident
    # steps: against the oracle over the 100 steps, and against 100
    # multi-kernel steps
    sc = _with_u(W.lpv_tank(2), 100, 40.0)
    u = torch.as_tensor(sc.u_seq)
    a = _sim(sc)
    a.rollout(30, u[:30].contiguous(), resident=True)
    a.rollout(40, u[30:70].contiguous())
    a.rollout(30, u[70:].contiguous(), resident=True)
    sa, wa, ra, _, step = a.get_state()
    assert step == 100 and a.status() == 0
    b = _sim(sc)
    b.rollout(100, u)
    sb, _, rb, _, _ = b.get_state()
    st = O.state_from_scenario(sc)
    O.rollout(sc.params, st, sc.ghosts.astype(np.float64), 100, sc.u_seq)
    L = sc.tank_size
    assert np.sqrt(((sa.cpu().numpy().astype(np.float64) - st.s) ** 2).sum(1)).max() <= 1e-3 * L
    assert torch.sqrt(((sa - sb).double() ** 2).sum(1)).max().item() <= 1e-3 * L
    assert np.abs(ra - st.rigid).max() <= 1e-3 and np.abs(ra - rb).max() <= 1e-3
    a.close()
    b.close()


def test_resident_refuses_a_large_tank():
    sc = W.closed_loop_circle(0, n_steps=10)
    sim = _sim(sc)
    assert not sim.resident_fits()
    with pytest.raises(RuntimeError):
        sim.rollout(10, resident=True)
    sim.rollout(10)   # the multi-kernel path still runs
    assert sim.status() == 0
    sim.close()


def _emptied(sc):
    z = np.zeros((0, 2), np.float32)
    return dataclasses.replace(sc, name=sc.name + "_empty", pos=z, vel=z)


@pytest.mark.parametrize("resident", [False, True], ids=["multi_kernel", "resident"])
@pytest.mark.parametrize("where", [0, 1, 2], ids=["first", "middle", "last"])
def test_batch_with_an_empty_tank(where, resident):
    # a tank with walls and no fluid anywhere in a batch: the other tanks run
    # bitwise as they do alone, and the empty one flies its rigid body under
    # its input and attitude law exactly as the oracle's empty tank does
    from paper_2604_12505_amd.sph import Simulator
    n = 140   # two graph-replayed chunks on the multi-kernel path
    scs = [W.paper_p0(0, n_steps=n, spawn="random"), _with_u(W.lpv_tank(1), n, 40.0)]
    scs.insert(where, _emptied(_with_u(W.paper_p0(2, n_steps=n, spawn="random"), n, 40.0)))
    n_ref = max(len(sc.theta_ref) for sc in scs)
    ref = np.stack([np.pad(sc.theta_ref, (0, n_ref - len(sc.theta_ref)), mode="edge") for sc in scs])
    b = Simulator.batch(scs)
    assert b.resident_fits()
    u = torch.stack([torch.as_tensor(sc.u_seq[:n]) for sc in scs])
    logs = b.rollout(n, u, theta_ref=ref, log_stride=10, resident=resident)
    s, w, rig, _, step = b.get_state()
    assert b.status() == 0 and list(step) == [n] * 3
    o = 0
    for t, sc in enumerate(scs):
        one = _sim(sc)
        one.rollout(n, torch.as_tensor(sc.u_seq[:n]), theta_ref=sc.theta_ref, resident=resident)
        s1, w1, r1, _, _ = one.get_state()
        assert one.status() == 0
        k = sc.n_fluid
        assert torch.equal(s[o:o + k], s1) and torch.equal(w[o:o + k], w1)
        assert np.array_equal(rig[t], r1)
        o += k
        one.close()
    e = scs[where]
    st = O.state_from_scenario(e)
    O.rollout(e.params, st, e.ghosts.astype(np.float64), n, e.u_seq[:n], e.theta_ref)
    assert np.allclose(rig[where], st.rigid, rtol=1e-9, atol=1e-12)
    assert not logs["wrench"][where].any()
    b.close()
