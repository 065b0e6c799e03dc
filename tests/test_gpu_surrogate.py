"""The trained surrogate against the SPH it replaces (the reduced-size
configuration of the benchmark's surrogate leg: random tanks of 2k-8k
particles, the Tait law without tension, 2,000 forced steps logged every
25).

The network is trained by the library's own kernels on relaxed, then
forced, random-tank rollouts and judged on held-out tanks.  Its inputs are
the configured window (theta, thetadot, input torque) and the tank's
constants (fill ratio, shape, particle spacing) in the fourth channel.

The bar is SPH's own reproducibility.  The held-out tanks are simulated
twice with the same shapes, sizes, fills and inputs, differing only in the
initial lattice jitter (1 % of the spacing): set A and set B.  The
per-channel NRMSE between A's and B's wrench is the noise floor, how far
this weakly compressible SPH reproduces its own wrench (measured 0.83 /
0.32 / 0.35 for F_x / F_y / torque on 64 held-out tanks; 0.29 / 0.12 / 0.14
at full size, 2k-60k particles over 5,000 steps).  No predictor of the
wrench from these inputs can do much better than about floor / sqrt(2)
against one realization.  What is asserted:

* the window kernel builds exactly the standardised windows of the logs;
* against set A, every channel's NRMSE is below that channel's floor (the
  network disagrees with SPH less than SPH disagrees with itself), and
  below the constant predictor's;
* the network answers the held-out windows far faster than SPH produced
  them;
* driving the rigid body with the network instead of SPH (from the
  hand-over at the first full window on, the same inputs), its attitude
  and rate stay closer to SPH's than with the fluid's mean wrench, and the
  run is far faster than SPH;
* with every window declared out of range, the SPH fallback reproduces the
  SPH logs bit for bit.

The 2 % target on the wrench error lies below the floor on every channel,
so no surrogate of this SPH can be held to it.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_surrogate_reaches_the_sph_noise_floor_and_is_faster_than_sph():
    from paper_2604_12505_amd import surrogate as S
    kw = dict(n_steps=2000, log_stride=25, relax_cycles=10, relax_steps=100, n_min=2000, n_max=8000)
    tr = S.generate(list(range(1000, 1192)), **kw)
    held = list(range(900000, 900064))
    te_a = S.generate(held, jitter_seed=1, **kw)
    te_b = S.generate(held, jitter_seed=2, **kw)
    norm = S.norm_from(tr)
    xtr, ytr = S.windows(tr, norm)
    xa, ya = S.windows(te_a, norm)
    T = 2000 // 25
    per = T - 31
    assert xtr.shape == (192 * per, 128)
    # the window kernel against a direct slicing of the logs (fourth
    # channel: the tank's constants in turn, fill, shape, dx)
    ns = S.N_STATIC
    f = tr.feat[3, 5:37].cpu().numpy()
    x0 = xtr[3 * per + 5].reshape(32, 4).cpu().numpy()
    q = np.arange(32) % ns
    st = tr.static[3].cpu().numpy()[q]
    ref = np.concatenate([(f - norm[:3]) / norm[3 + ns:6 + ns], ((st - norm[3 + q]) / norm[6 + ns + q])[:, None]], 1)
    assert np.allclose(x0, ref, rtol=1e-5, atol=1e-5)
    om, osd = S.out_norm(norm)
    y_ref = (tr.wrench[3, 36].cpu().numpy() - om) / osd
    assert np.allclose(ytr[3 * per + 5].cpu().numpy(), y_ref, rtol=1e-5, atol=1e-5)
    net = S.train(xtr, ytr, epochs=30, batch=1024, lr=2e-3, lr_final=1e-4)
    inf = S.inference_net(net, max_batch=8192)
    err = S.nrmse(S.predict(inf, xa), ya, norm)
    base = S.nrmse(torch.zeros_like(ya), ya, norm)
    floor = S.noise_floor(te_a, te_b)
    t_nn = S.time_inference(inf, xa)
    speedup = te_a.sph_seconds / t_nn
    print("held-out NRMSE", err, "noise floor", floor, "constant predictor", base, "speedup", speedup)
    assert np.all(np.isfinite(err))
    assert np.all(err <= floor), (err, floor)
    assert np.all(err < base)
    assert speedup > 10.0

    # the rigid body driven by the network instead of SPH, against SPH
    # (set A); set B gives SPH's own spread, the mean wrench the baseline
    cpl = S.coupled(inf, te_a, norm)
    e_nn = S.trajectory_nrmse(cpl["y"], te_a)
    const = S.constant_net(norm, max_batch=64)
    e_c = S.trajectory_nrmse(S.coupled(const, te_a, norm)["y"], te_a)
    e_b = S.trajectory_nrmse(te_b.y, te_a)
    speedup_c = te_a.sph_seconds / cpl["seconds"]
    print("coupled trajectory NRMSE (r_x, r_y, theta, rdot_x, rdot_y, thetadot): network", e_nn,
          "mean wrench", e_c, "SPH B vs A", e_b, "flagged", int((cpl["flags"] & 1).sum().item()),
          "coupled speedup", speedup_c)
    assert np.all(np.isfinite(e_nn))
    assert e_nn[2] < e_c[2] and e_nn[5] < e_c[5]
    assert speedup_c > 10.0

    # the fallback: every window out of range, every rollout back on SPH
    import workloads as W
    scs = [W.random_tank(sd, n_steps=2000, n_min=2000, n_max=8000, eos=W.EOS_TAIT_CLAMPED, jitter_seed=1)
           for sd in held]
    fb = S.coupled_or_sph(inf, te_a, norm, scs, z_max=1e-6, relax=(10, 100))
    assert fb["fell_back"] == list(range(len(held)))
    assert torch.equal(fb["y"], te_a.y) and torch.equal(fb["wrench"], te_a.wrench)
    const.close()
    net.close()
    inf.close()
