"""Failure flags of the HIP path, forced from the host, against the oracle's
flags on the same states (every kernel still exits normally: a non-finite
value or a fast particle only changes what the kernels compute and latch).

* a NaN velocity latches SPH_ST_NONFINITE (oracle: ORA_NONFINITE);
* a time step above the Courant limit at rest is refused by sph_init;
* a particle fast enough to push the step's Courant number dt (c + |w|) / h
  above 0.4 latches SPH_ST_CFL after one step (oracle: ORA_CFL), with c the
  sound speed of the equation of state (Tait c0, linear sqrt(k)); a slower
  one does not.
"""
import copy
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W
from oracle import sph as O

pytestmark = pytest.mark.gpu

ST_NONFINITE, ST_CFL = 2, 8          # device status bits (slosh.h)
ORA_NONFINITE, ORA_CFL = 2, 4        # oracle status bits


def _sim_at(sc, w):
    from paper_2604_12505_amd.sph import Simulator
    sim = Simulator.from_scenario(sc)
    sim.set_state(torch.as_tensor(sc.pos), torch.as_tensor(w.astype(np.float32)), sc.rigid0, 0.0, 0)
    return sim


def _oracle_status(sc, w, n=1):
    st = O.state_from_scenario(sc)
    st.w = w.astype(np.float32).astype(np.float64)
    status, _ = O.rollout(sc.params, st, sc.ghosts.astype(np.float64), n, sc.u_seq)
    return status


def test_nan_velocity_latches_nonfinite():
    sc = W.plain_rect(0, n_steps=4)
    w = sc.vel.copy()
    w[5, 0] = np.nan
    print("flags case: NaN velocity, plain rectangle", flush=True)
    sim = _sim_at(sc, w)
    assert sim.status() & ST_NONFINITE          # seen when the state is loaded
    sim.rollout(2, torch.as_tensor(sc.u_seq[:2]))
    assert sim.status() & ST_NONFINITE
    # the steps still run to the end (the value spreads to the neighbours
    # through the viscous term, the flag stays latched)
    _, _, _, _, step = sim.get_state()
    assert step == 2
    sim.close()
    assert _oracle_status(sc, w) & ORA_NONFINITE


def test_time_step_above_the_courant_limit_is_refused():
    from paper_2604_12505_amd.sph import Simulator
    sc = W.plain_rect(0, n_steps=2)
    p = copy.deepcopy(sc.params)
    p.dt = 3.0 * sc.params.dt                   # Courant number 0.6 at rest
    with pytest.raises(RuntimeError):
        Simulator(p, sc.pos, sc.vel, sc.ghosts, sc.rigid0)
    st = O.state_from_scenario(sc)
    status, _ = O.rollout(p, st, sc.ghosts.astype(np.float64), 1, sc.u_seq)
    assert status & ORA_CFL


@pytest.mark.parametrize("case", ["tait", "linear"])
def test_fast_particle_latches_the_courant_flag(case):
    if case == "tait":
        sc = W.plain_rect(0, n_steps=2)
        limit = sc.params.c0                    # dt = 0.2 h / c0: |w| <= c0
        i, axis = 100, 0
    else:
        sc = W.paper_p0(0, n_steps=2)
        limit = 0.4 * sc.params.h / sc.params.dt - math.sqrt(sc.params.k_lin)   # 2.04 m/s
        i, axis = 10, 1
    for speed, flagged in ((1.25 * limit, True), (0.75 * limit, False)):
        w = sc.vel.copy()
        w[i, axis] = speed
        print(f"flags case: {case}, speed {speed:.3f} m/s (limit {limit:.3f})", flush=True)
        sim = _sim_at(sc, w)
        assert sim.status() == 0
        sim.rollout(1, torch.as_tensor(sc.u_seq[:1]))
        got = sim.status()
        sim.close()
        assert bool(got & ST_CFL) == flagged, (speed, got)
        assert bool(_oracle_status(sc, w) & ORA_CFL) == flagged, speed
