"""The one-step Jacobian of the open-loop coupled step from the tangent-linear
kernels (paper_2604_12505_amd.eigen) against central differences of the FP64
oracle's step, on a small free tank after some evolution.

Bars: the whole matrix within 1e-3 of its largest entry and each block
(rigid, position, velocity rows x columns) within 5e-3 of its own largest
entry (binary32 tangents against binary64 differences).  Structure: the
body frame makes the fluid blind to r and, with no applied force, to theta,
so J has the eigenvalue 1 at least three times (the position integrators).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402
from oracle import sph as O  # noqa: E402

pytestmark = pytest.mark.gpu


def test_step_jacobian_matches_oracle_differences():
    from paper_2604_12505_amd.eigen import step_jacobian, continuous_eigenvalues
    from paper_2604_12505_amd.sph import Simulator
    sc = W.linearization_tank(0, n_steps=60, n_fluid=100)
    # the oracle advances the tank 60 steps; the GPU starts from the state it
    # reaches, rounded to binary32, and the differences are taken around it
    st = O.state_from_scenario(sc)
    status, _ = O.rollout(sc.params, st, sc.ghosts.astype(np.float64), 60, sc.u_seq[:60])
    assert status == 0
    s = st.s.astype(np.float32)
    w = st.w.astype(np.float32)
    rig, step = st.rigid.copy(), st.step
    sim = Simulator.from_scenario(sc)
    sim.set_state(torch.as_tensor(s), torch.as_tensor(w), rig, st.tau_ctrl, step)
    u = (0.0, 0.0, float(sc.u_seq[-1, 2]))
    J = step_jacobian(sim, u, block=64)
    N = sc.n_fluid
    n = 6 + 4 * N
    assert J.shape == (n, n)
    s0 = s.astype(np.float64)
    w0 = w.astype(np.float64)
    g = sc.ghosts.astype(np.float64)
    useq = np.array([u], np.float32)

    def one_step(x):
        st = O.State(x[6:6 + 2 * N].reshape(N, 2).copy(), x[6 + 2 * N:].reshape(N, 2).copy(), x[:6].copy(), 0.0,
                     step)
        O.rollout(sc.params, st, g, 1, useq)
        return np.concatenate([st.rigid, st.s.ravel(), st.w.ravel()])

    x0 = np.concatenate([rig, s0.ravel(), w0.ravel()])
    Jf = np.zeros((n, n))
    eps = 1e-6
    for c in range(n):
        e = np.zeros(n)
        e[c] = eps
        Jf[:, c] = (one_step(x0 + e) - one_step(x0 - e)) / (2 * eps)
    err = np.abs(J - Jf)
    assert err.max() <= 1e-3 * np.abs(Jf).max(), err.max() / np.abs(Jf).max()
    cuts = [0, 6, 6 + 2 * N, n]
    for a in range(3):
        for b in range(3):
            blk = np.s_[cuts[a]:cuts[a + 1], cuts[b]:cuts[b + 1]]
            ref = np.abs(Jf[blk]).max()
            if ref > 0:
                assert err[blk].max() <= 5e-3 * ref, (a, b, err[blk].max() / ref)
    mu = np.linalg.eigvals(J)
    assert np.sum(np.abs(mu - 1.0) < 1e-6) >= 3
    lam = continuous_eigenvalues(J, sc.params.dt)
    assert np.all(np.isfinite(lam.real))
    sim.close()
