"""End-to-end identification on a short SPH record (Section 5.3 pipeline at
reduced size): SPH data -> LTI stand-in for ssest -> LPV fit -> closed loop.

Asserts what holds at any size: the SPH record is the open-loop response
(the logged torque is the input), the LTI fit explains the velocities, the
LPV fit is at least as good as the LTI model it starts from (within a small
margin: its restarts start from it), the selected model runs in closed
loop, and the surrogate is orders of magnitude faster than the SPH run it
replaces.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def test_identification_pipeline_short_record():
    from paper_2604_12505_amd import identify as I
    n = 240
    u = W.lpv_input_train(0, n)
    run = I.sph_run(u, None, relax=(20, 50))
    assert run["y"].shape == (n, 6)
    assert np.allclose(run["u"], u, rtol=1e-6, atol=1e-4)
    res = I.identify(u, run["y"][:, 3:6], n_lti=16, n_restarts=16, adam_iters=200, lbfgs_iters=200,
                     lti_adam=300, lti_lbfgs=300)
    print("train BFR LTI", res["lti_bfr"], "LPV", res["lpv_bfr"])
    assert res["lti_bfr"].mean() > 90.0
    assert res["lpv_bfr"].mean() >= res["lti_bfr"].mean() - 2.0
    force, ref = W.manoeuvre_profile(2)
    force, ref = force[:200], ref[:200]
    kp, kd = run["kp"], run["kd"]
    # the closed-loop kernel is checked against the oracle on seeded models in
    # test_gpu_lpv.py; the identified model is this pipeline's output, so here
    # it is only run
    y, secs = I.closed_loop(res["lpv"], force, ref, res, kp, kd)
    assert y.shape[0] == 200 and np.all(np.isfinite(y))
    sph_per_sample = run["sph_seconds"] / n
    assert sph_per_sample * 200 / secs > 100.0
