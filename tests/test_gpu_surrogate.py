"""The trained surrogate against the SPH it replaces (small version of the
full training run): the network, trained on relaxed and forced random-tank
rollouts by the library's own kernels, must predict held-out wrenches far
better than the best constant predictor and faster than SPH produces them."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_surrogate_gain_over_sph():
    from paper_2604_12505_amd import surrogate as S
    kw = dict(n_steps=1000, log_stride=10, relax_cycles=10, relax_steps=100, n_min=2000, n_max=4000)
    tr = S.generate(list(range(10, 34)), **kw)
    te = S.generate(list(range(500, 506)), **kw)
    norm = S.norm_from(tr)
    xtr, ytr = S.windows(tr, norm)
    xte, yte = S.windows(te, norm)
    assert xtr.shape == (24 * (100 - 31), 128)
    # the window kernel against a direct slicing of the logs
    f = tr.feat[3, 5:37].cpu().numpy()
    x0 = xtr[3 * 69 + 5].reshape(32, 4).cpu().numpy()
    ref = (np.concatenate([f, np.full((32, 1), tr.fill[3].item())], 1) - norm[:4]) / norm[4:8]
    assert np.allclose(x0, ref, rtol=1e-5, atol=1e-5)
    net = S.train(xtr, ytr, epochs=60, batch=256, lr=2e-3, lr_final=1e-4)
    inf = S.inference_net(net, max_batch=4096)
    err = S.nrmse(S.predict(inf, xte), yte, norm)
    base = S.nrmse(torch.zeros_like(yte), yte, norm)
    t_nn = S.time_inference(inf, xte)
    speedup = te.sph_seconds / t_nn
    print("held-out NRMSE", err, "constant predictor", base, "speedup", speedup)
    assert np.all(err < 0.5 * base)
    assert speedup > 10.0
    net.close()
    inf.close()
