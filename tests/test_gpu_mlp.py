"""GPU parity of the BF16-MFMA surrogate network against the FP64 oracle.

The oracle runs on the BF16-rounded weights and inputs the GPU sees, so the
remaining differences are the BF16 rounding of activations (and gradients)
between layers: 4 roundings of relative size 2^-9 each bound the forward
error by ~1e-2 of the output scale; gradients pass through 8 such roundings,
hence 3e-2.  Adam is checked exactly (FP32) on the GPU's own gradients.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _bf16(a):
    return torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _net(seed=0):
    from paper_2604_12505_amd import mlp as G
    rng = np.random.default_rng(seed)
    params = M.init_params(rng)
    vec = G.pack(params)
    return G, rng, params, vec


def _rounded_params(vec):
    from paper_2604_12505_amd import mlp as G
    return [(_bf16(W), b.astype(np.float32).astype(np.float64)) for W, b in G.unpack(vec)]


@pytest.mark.parametrize("B", [1, 37, 64, 1000])
def test_forward_matches_oracle(B):
    G, rng, params, vec = _net(1)
    net = G.Mlp(vec, max_batch=1024)
    x = rng.normal(size=(B, 128)).astype(np.float32)
    y = net.forward(torch.as_tensor(x)).cpu().numpy().astype(np.float64)
    ref, _, _ = M.forward(_rounded_params(vec), _bf16(x))
    err = np.abs(y - ref).max() / np.abs(ref).max()
    print("forward rel err", B, err)
    assert err < 1e-2
    net.close()


def test_launch_equals_forward():
    # back-to-back launches on the network's stream (no stream hand-over)
    # give forward()'s output bit for bit, a ragged last tile included
    G, rng, params, vec = _net(3)
    net = G.Mlp(vec, max_batch=1000)
    x = torch.as_tensor(rng.normal(size=(1000, 128)).astype(np.float32), device="cuda:0")
    y1 = net.forward(x)
    y2 = torch.full_like(y1, float("nan"))
    torch.cuda.synchronize()
    for _ in range(3):
        net.launch(x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    with pytest.raises(ValueError):
        net.launch(x.double(), y2)
    net.close()


def test_misaligned_input_is_refused():
    # the input rows are read four floats at a time: an input pointer that
    # is not 16-byte aligned is refused with SPH_E_INVAL, nothing launched
    import ctypes as C
    G, rng, params, vec = _net(4)
    net = G.Mlp(vec, max_batch=256)
    x = torch.zeros(129 * 128, device="cuda:0")
    y = torch.zeros(128, 3, device="cuda:0")
    t = torch.zeros(128, 3, device="cuda:0")
    bad = C.c_void_p(x.data_ptr() + 4)
    assert net.L.mlp_forward(net.h, bad, 128, C.c_void_p(y.data_ptr())) < 0
    assert net.L.mlp_train_step(net.h, bad, C.c_void_p(t.data_ptr()), 128, 1e-3, 0.9, 0.999, 1e-8, None, None) < 0
    assert net.L.mlp_forward(net.h, C.c_void_p(x.data_ptr()), 128, C.c_void_p(y.data_ptr())) == 0
    torch.cuda.synchronize()
    net.close()


def test_forward_at_the_inference_batch_size():
    # the surrogate workload's inference batch, 65,536 windows in one launch:
    # sampled rows (and the last ones, the ragged end of the grid) against
    # the oracle
    G, rng, params, vec = _net(2)
    B = 65536
    net = G.Mlp(vec, max_batch=B)
    x = rng.normal(size=(B, 128)).astype(np.float32)
    y = net.forward(torch.as_tensor(x)).cpu().numpy().astype(np.float64)
    rows = np.concatenate([rng.choice(B - 64, 2048, replace=False), np.arange(B - 64, B)])
    ref, _, _ = M.forward(_rounded_params(vec), _bf16(x[rows]))
    err = np.abs(y[rows] - ref).max() / np.abs(ref).max()
    print("forward rel err at B = 65,536", err)
    assert err < 1e-2
    net.close()


def test_gradients_match_oracle():
    G, rng, params, vec = _net(2)
    B = 256
    net = G.Mlp(vec, max_batch=B)
    x = rng.normal(size=(B, 128)).astype(np.float32)
    t = rng.normal(size=(B, 3)).astype(np.float32)
    loss, grad = net.train_step(torch.as_tensor(x), torch.as_tensor(t), lr=0.0, want_grad=True)
    gp = _rounded_params(vec)
    ref = M.backward(gp, _bf16(x), t.astype(np.float64))
    g_gpu = G.unpack(grad.cpu().numpy())
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(g_gpu, ref)):
        eW = np.abs(gW - rW).max() / np.abs(rW).max()
        eb = np.abs(gb - rb).max() / np.abs(rb).max()
        cos = (gW * rW).sum() / np.sqrt((gW * gW).sum() * (rW * rW).sum())
        print("layer", li, "dW rel", eW, "db rel", eb, "cos", cos)
        assert eW < 3e-2 and eb < 3e-2 and cos > 0.999
    ref_loss = M.loss(gp, _bf16(x), t.astype(np.float64))
    assert float(loss.item()) == pytest.approx(ref_loss, rel=1e-2)
    net.close()


def test_adam_step_matches_oracle_on_gpu_gradients():
    G, rng, params, vec = _net(3)
    B = 64
    net = G.Mlp(vec, max_batch=B)
    x = torch.as_tensor(rng.normal(size=(B, 128)).astype(np.float32))
    t = torch.as_tensor(rng.normal(size=(B, 3)).astype(np.float32))
    opt = M.Adam(G.unpack(vec), lr=1e-3)
    cur = G.unpack(vec)
    for _ in range(3):
        _, grad = net.train_step(x, t, lr=1e-3, want_grad=True)
        cur = opt.step(cur, G.unpack(grad.cpu().numpy()))
    got = net.params().cpu().numpy().astype(np.float64)
    ref = G.pack(cur).astype(np.float64)
    assert np.abs(got - ref).max() < 1e-6
    net.close()


def test_training_fits_a_smooth_map():
    G, rng, params, vec = _net(4)
    B = 512
    net = G.Mlp(vec, max_batch=B)
    x = rng.normal(size=(B, 128)).astype(np.float32)
    A = rng.normal(size=(128, 3)) / np.sqrt(128)
    t = np.tanh(x @ A).astype(np.float32)
    xt, tt = torch.as_tensor(x), torch.as_tensor(t)
    first = None
    for it in range(300):
        loss, _ = net.train_step(xt, tt, lr=1e-3)
        if first is None:
            first = float(loss.item())
    last = float(loss.item())
    print("loss", first, "->", last)
    assert last < 0.05 * first
    net.close()


def test_backward_of_a_given_output_gradient_matches_oracle():
    # mlp_backward: any dL/dy, not only the mean-squared-error one; the
    # weights do not move
    G, rng, params, vec = _net(5)
    B = 96
    net = G.Mlp(vec, max_batch=B)
    x = rng.normal(size=(B, 128)).astype(np.float32)
    dy = (rng.normal(size=(B, 3)) / B).astype(np.float32)
    grad = net.backward(torch.as_tensor(x), torch.as_tensor(dy))
    ref = M.backward_from(_rounded_params(vec), _bf16(x), dy.astype(np.float64))
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(G.unpack(grad.cpu().numpy()), ref)):
        eW = np.abs(gW - rW).max() / np.abs(rW).max()
        eb = np.abs(gb - rb).max() / np.abs(rb).max()
        print("layer", li, "dW rel", eW, "db rel", eb)
        assert eW < 3e-2 and eb < 3e-2
    assert np.array_equal(net.params().cpu().numpy(), np.asarray(vec, np.float32))
    # linear in dy: the gradient of 2 dy is twice the gradient of dy, exactly
    # (scaling by 2 is exact in binary32 and in BF16)
    grad2 = net.backward(torch.as_tensor(x), torch.as_tensor(2.0 * dy))
    assert torch.equal(grad2, 2.0 * grad)
    net.close()


def test_split_backward_and_adam_step_match_oracle_adam():
    # mlp_backward + mlp_adam_step, step by step, against the oracle's Adam on
    # the same gradients; the bias correction follows the step number given
    G, rng, params, vec = _net(6)
    B = 64
    net = G.Mlp(vec, max_batch=B)
    x = torch.as_tensor(rng.normal(size=(B, 128)).astype(np.float32))
    opt = M.Adam(G.unpack(vec), lr=2e-3)
    cur = G.unpack(vec)
    for t in (1, 2, 3):
        dy = torch.as_tensor((rng.normal(size=(B, 3)) / B).astype(np.float32))
        grad = net.backward(x, dy)
        net.adam_step(grad, t, lr=2e-3)
        cur = opt.step(cur, G.unpack(grad.cpu().numpy()))
    got = net.params().cpu().numpy().astype(np.float64)
    assert np.abs(got - G.pack(cur).astype(np.float64)).max() < 1e-6
    with pytest.raises(RuntimeError):
        net.adam_step(grad, 0)
    net.close()
