"""lpv_loss_grad_noalloc (no workspace; a fixed per-GPU array holds the
reverse sweep's record) against lpv_loss_grad (caller's workspace), both
through the C ABI: two calls in a row, the second on a smaller input, so
the second reuses the array the first filled.  The two run the same kernel
on the same inputs, so loss and gradient must agree bit for bit; the
gradient is also checked against the FP64 oracle on a few models.
A request larger than the array is refused before any launch."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import lpv as O  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _models(rng, R, scale=0.3):
    out = []
    for _ in range(R):
        P = O.unpack(rng.normal(size=O.N_PARAM) * scale)
        P["A0"][:] = 0.8 * np.eye(4) + 0.05 * rng.normal(size=(4, 4))
        P["A1"][:] = 0.05 * rng.normal(size=(4, 4))
        out.append(O.pack(P))
    return np.stack(out)


@pytest.mark.parametrize("lti_only", [False, True])
def test_noalloc_equals_workspace_entry_point_twice(lti_only):
    from paper_2604_12505_amd import lpv as L
    rng = np.random.default_rng(11)
    opts = L.Options(sigma2=1e-3, sigmax=1e-2, lti_only=lti_only)
    # first call: 3 waves of models (one partly filled), 2,200 samples;
    # second: fewer models and samples, so the array holds stale data beyond
    for R, n in ((37, 2200), (5, 300)):
        print(f"noalloc case R={R} n={n} lti_only={lti_only}", flush=True)
        V = torch.as_tensor(_models(rng, R), device=DEV)
        u = torch.as_tensor(rng.normal(size=(n, 3)), device=DEV)
        y = torch.as_tensor(rng.normal(size=(n, 3)), device=DEV)
        f_ws, g_ws = L.loss_grad(V, u, y, opts)
        f_na, g_na = L.loss_grad_noalloc(V, u, y, opts)
        torch.cuda.synchronize()
        assert torch.equal(f_ws, f_na), (R, n)
        assert torch.equal(g_ws, g_na), (R, n)
        g = g_na.cpu().numpy()
        mask = O.lti_mask() if lti_only else np.ones(O.N_PARAM)
        for r in (0, R - 1):
            f_ref, g_ref = O.loss_and_grad(V[r].cpu().numpy(), u.cpu().numpy(), y.cpu().numpy(), 1e-3, 1e-2)
            assert float(f_na[r]) == pytest.approx(f_ref, rel=1e-12)
            assert np.max(np.abs(g[r] - g_ref * mask)) <= 1e-9 * np.max(np.abs(g_ref)), r


def test_noalloc_refuses_a_request_beyond_its_array():
    from paper_2604_12505_amd import _lib
    from paper_2604_12505_amd import lpv as L
    lib = _lib.load()
    R, n = 16, 16385   # one wave of models: 16,384 samples fit, one more does not
    V = torch.zeros(R, L.N_PARAM, dtype=torch.float64, device=DEV)
    u = torch.zeros(n, 3, dtype=torch.float64, device=DEV)
    loss = torch.full((R,), -1.0, dtype=torch.float64, device=DEV)
    o = L.Options().c()
    rc = lib.lpv_loss_grad_noalloc(C.c_void_p(V.data_ptr()), R, C.c_void_p(u.data_ptr()),
                                   C.c_void_p(u.data_ptr()), n, C.byref(o), C.c_void_p(loss.data_ptr()),
                                   None, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -3   # SPH_E_CAPACITY
    torch.cuda.synchronize()
    assert bool((loss == -1.0).all())   # nothing was launched
    f, _ = L.loss_grad_noalloc(V[:, :], u[:16384], u[:16384], grad=False)
    assert torch.isfinite(f).all()
