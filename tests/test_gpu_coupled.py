"""GPU parity of mlp_coupled_rollout (the rigid body driven by the surrogate
network instead of SPH) against the FP64 oracle, oracle.mlp.coupled_rollout.

Inputs are seeded and synthetic (window features, tank constants, inputs,
body constants and start states drawn at random); none comes from the GPU.

* A constant network (all weights zero, a head bias) makes the wrench exact
  on both sides up to its FP32 de-standardisation, so the integration and
  the logging are compared tightly: the FP64 states agree to 1e-9 of their
  scale and the FP32 logs to their own rounding.
* A random network is compared as the forward-parity test compares it: the
  oracle runs on the BF16-rounded weights.  The windows differ by the BF16
  rounding of the inputs on the GPU side (2^-9 relative) and the network's
  4 roundings between layers, so each interval's wrench agrees to 2e-2 of
  the output scale.  The body constants make the feedback weak: a wrench
  error moves thetadot by at most stride dt dF / J per interval, and that
  moves the next windows' inputs by far less than their BF16 rounding, so
  the state errors are bounded by integrating the per-interval wrench bound.
* The out-of-range flag, and the argument checks.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp as M

pytestmark = pytest.mark.gpu

W = 32


def _bf16(a):
    return torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _case(R, n_steps, stride, seed, ns=3):
    rng = np.random.default_rng(seed)
    static = rng.uniform(0.2, 0.8, size=(R, ns)).astype(np.float32)
    feat0 = (rng.normal(size=(R, W, 3)) * [0.3, 0.2, 5.0]).astype(np.float32)
    u = (rng.normal(size=(R, n_steps, 3)) * [20.0, 20.0, 10.0]).astype(np.float32)
    body = np.stack([rng.uniform(800, 1200, R), rng.uniform(400, 600, R), rng.uniform(2e-4, 1e-3, R)], 1)
    rigid0 = rng.normal(size=(R, 6)) * [0.1, 0.1, 0.3, 0.05, 0.05, 0.2]
    ni = 3 + ns
    norm = np.concatenate([[0.0, 0.0, 0.0], np.full(ns, 0.5), [1.0, 1.0, 5.0], np.full(ns, 0.2),
                           [5.0, -3.0, 1.0], [50.0, 50.0, 20.0]]).astype(np.float32)
    assert norm.size == 2 * ni + 6
    return static, feat0, u, body, rigid0, norm


def _gpu(vec, R, *args, **kw):
    from paper_2604_12505_amd.mlp import Mlp
    net = Mlp(vec, max_batch=max(R, 64))
    res = net.coupled_rollout(*args, **kw)
    out = {k: v.cpu().numpy() for k, v in res.items()}
    net.close()
    return out


# log strides 10, 25 and 70 (a ragged last interval in each)
@pytest.mark.parametrize("R,n_steps,stride", [(16, 41 * 10 + 3, 10), (70, 40 * 25, 25), (20, 35 * 70 + 11, 70)])
def test_constant_network_integration_matches_oracle(R, n_steps, stride):
    from paper_2604_12505_amd import mlp as G
    static, feat0, u, body, rigid0, norm = _case(R, n_steps, stride, seed=R)
    beta = np.array([0.5, -1.25, 0.75])
    params = [(np.zeros_like(Wl), np.zeros_like(b)) for Wl, b in M.init_params(np.random.default_rng(0))]
    params[-1] = (params[-1][0], beta)
    vec = G.pack(params)
    g = _gpu(vec, R, norm, static, feat0, rigid0, u, body, stride, z_max=1e6)
    o = M.coupled_rollout(params, norm.astype(np.float64), static, feat0, rigid0, u, body, stride)
    T = -(-n_steps // stride)
    assert np.all(g["flags"] == 0)
    F = beta * norm[-3:] + norm[-6:-3]
    np.testing.assert_allclose(g["wrench"][:, W - 1:], np.broadcast_to(F, (R, T - W + 1, 3)), rtol=1e-6)
    assert np.all(np.isnan(g["wrench"][:, :W - 1])) and np.all(np.isnan(g["y"][:, :W]))
    scale = np.abs(o["y"][:, W:]).max(axis=(0, 1)) + 1e-30
    assert np.all(np.abs(g["y"][:, W:] - o["y"][:, W:]) <= 2e-6 * scale + 1e-30)
    np.testing.assert_allclose(g["rigid"], o["rigid"], rtol=1e-9, atol=1e-9 * np.abs(o["rigid"]).max())
    np.testing.assert_array_equal(g["feat"][:, :W], feat0)
    assert np.all(np.abs(g["feat"][:, W:] - o["feat"][:, W:]) <= 2e-6 * (np.abs(o["feat"][:, W:]).max() + 1e-30))


def test_random_network_matches_oracle_within_the_bf16_bound():
    from paper_2604_12505_amd import mlp as G
    R, stride = 40, 20
    n_steps = 44 * stride
    static, feat0, u, body, rigid0, norm = _case(R, n_steps, stride, seed=7)
    params = M.init_params(np.random.default_rng(11))
    vec = G.pack(params)
    g = _gpu(vec, R, norm, static, feat0, rigid0, u, body, stride, z_max=1e6)
    rounded = [(_bf16(Wl), b.astype(np.float32).astype(np.float64)) for Wl, b in G.unpack(vec)]
    o = M.coupled_rollout(rounded, norm.astype(np.float64), static, feat0, rigid0, u, body, stride)
    T = -(-n_steps // stride)
    dF = np.abs(g["wrench"][:, W - 1:] - o["wrench"][:, W - 1:])
    tolF = 2e-2 * np.abs(o["wrench"][:, W - 1:]).max(axis=(0, 1))
    print("worst wrench error / output scale", (dF.max(axis=(0, 1)) / np.abs(o["wrench"][:, W - 1:]).max(axis=(0, 1))))
    assert np.all(dF <= tolF)
    # state bounds from integrating the per-interval wrench bound
    m, J, dt = body[:, 0], body[:, 1], body[:, 2]
    ba_lin, ba_rot = np.sqrt(2.0) * max(tolF[0], tolF[1]) / m, tolF[2] / J
    bv = np.zeros((R, 2))
    bx = np.zeros((R, 2))
    for k in range(W - 1, T - 1):
        for _ in range(stride):
            bv += dt[:, None] * np.stack([ba_lin, ba_rot], 1)
            bx += dt[:, None] * bv
        y_err = np.abs(g["y"][:, k + 1] - o["y"][:, k + 1])
        y_scale = np.abs(o["y"][:, k + 1])
        lim = np.stack([bx[:, 0], bx[:, 0], bx[:, 1], bv[:, 0], bv[:, 0], bv[:, 1]], 1) * 1.01 + 2e-6 * y_scale + 1e-9
        assert np.all(y_err <= lim), (k, (y_err / lim).max())


def test_out_of_range_windows_are_flagged():
    from paper_2604_12505_amd import mlp as G
    R, stride = 8, 10
    n_steps = 40 * stride
    static, feat0, u, body, rigid0, norm = _case(R, n_steps, stride, seed=3)
    feat0[2, 5, 2] = 1e4                         # an input torque far outside the training range
    feat0[5, W - 1, 0] = np.nan                  # not a number
    vec = G.pack(M.init_params(np.random.default_rng(1)))
    g = _gpu(vec, R, norm, static, feat0, rigid0, u, body, stride, z_max=50.0)
    flagged = np.nonzero(g["flags"] & 1)[0].tolist()
    assert flagged == [2, 5]
    assert np.all(g["flags"][[0, 1, 3, 4, 6, 7]] == 0)


def test_argument_checks():
    from paper_2604_12505_amd import mlp as G
    R, stride = 4, 10
    static, feat0, u, body, rigid0, norm = _case(R, 40 * stride, stride, seed=5)
    vec = G.pack(M.init_params(np.random.default_rng(2)))
    net = G.Mlp(vec, max_batch=64)
    with pytest.raises(RuntimeError):
        net.coupled_rollout(norm, static, feat0, rigid0, u, body, stride, z_max=0.0)
    bad = norm.copy()
    bad[3 + 3] = 0.0                             # a zero input std
    with pytest.raises(RuntimeError):
        net.coupled_rollout(bad, static, feat0, rigid0, u, body, stride)
    with pytest.raises(RuntimeError):               # more rollouts than the handle's batch
        n = 65
        net.coupled_rollout(norm, np.repeat(static[:1], n, 0), np.repeat(feat0[:1], n, 0),
                            np.repeat(rigid0[:1], n, 0), np.repeat(u[:1], n, 0), np.repeat(body[:1], n, 0), stride)
    net.close()
