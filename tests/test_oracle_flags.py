"""The oracle's failure flags: a non-finite state and a step above the
Courant limit are reported in its status word.

The Courant number of a step is dt (c + |w|) / h, with c the equation of
state's sound speed at rest (c0 for the Tait law, sqrt(k) for the linear law
of eq. EOS); a step is flagged when a particle's number after the update
exceeds 0.4, twice the 0.2 the workloads' time step is set from."""
import copy
import math

import numpy as np

import workloads as W
from oracle import sph as O

ST_NONFINITE, ST_CFL = 2, 4


def _state(sc):
    return O.state_from_scenario(sc)


def test_clean_run_sets_no_flag():
    sc = W.plain_rect(0, n_steps=20)
    status, _ = O.rollout(sc.params, _state(sc), sc.ghosts.astype(np.float64), 20, sc.u_seq)
    assert status == 0


def test_nan_velocity_is_flagged():
    sc = W.plain_rect(0, n_steps=2)
    st = _state(sc)
    st.w[5, 0] = math.nan
    status, _ = O.rollout(sc.params, st, sc.ghosts.astype(np.float64), 1, sc.u_seq)
    assert status & ST_NONFINITE


def test_time_step_above_the_courant_limit_is_flagged():
    # dt three times the CFL step: Courant number 0.6 even at rest
    sc = W.plain_rect(0, n_steps=2)
    p = copy.deepcopy(sc.params)
    p.dt = 3.0 * sc.params.dt
    status, _ = O.rollout(p, _state(sc), sc.ghosts.astype(np.float64), 1, sc.u_seq)
    assert status & ST_CFL
    # the configured step (0.2 h / c0) at the same state is clean
    status, _ = O.rollout(sc.params, _state(sc), sc.ghosts.astype(np.float64), 1, sc.u_seq)
    assert status == 0


def test_a_fast_particle_pushes_the_step_over_the_limit():
    # Tait, dt = 0.2 h / c0: the limit is |w| = c0 = 20 m/s
    sc = W.plain_rect(0, n_steps=2)
    for speed, flagged in ((25.0, True), (15.0, False)):
        st = _state(sc)
        st.w[100] = (speed, 0.0)
        status, _ = O.rollout(sc.params, st, sc.ghosts.astype(np.float64), 1, sc.u_seq)
        assert bool(status & ST_CFL) == flagged, speed


def test_linear_law_uses_its_own_sound_speed():
    # the paper's scenario: c = sqrt(3) m/s, dt = 1 ms, h = 9.42 mm; the limit
    # is |w| = 0.4 h / dt - c = 2.04 m/s
    sc = W.paper_p0(0, n_steps=2)
    c = math.sqrt(sc.params.k_lin)
    limit = 0.4 * sc.params.h / sc.params.dt - c
    assert 2.0 < limit < 2.1
    for speed, flagged in ((limit + 0.3, True), (limit - 0.5, False)):
        st = _state(sc)
        st.w[10] = (0.0, speed)
        status, _ = O.rollout(sc.params, st, sc.ghosts.astype(np.float64), 1, sc.u_seq)
        assert bool(status & ST_CFL) == flagged, speed
