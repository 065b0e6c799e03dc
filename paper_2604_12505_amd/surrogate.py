"""Slosh-wrench surrogate: data from SPH rollouts, training and evaluation.

Orchestration only: every rollout runs in the SPH kernels (``sph_rollout``),
windows are built by ``mlp_make_windows``, and the network is trained and
evaluated by the MFMA kernels (``mlp_train_step``, ``mlp_forward``).

Data recipe (the random-tank generator of ``workloads.random_tank``, with
the Tait law clamped at zero pressure by default, see ``generate``):
rectangular or circular tank, fill U[0.2, 0.8], 2k-60k particles, torque a
5-tone random-phase multisine on the 0.05 Hz grid with amplitude U[0, 50] N m,
spacecraft m = 1000 kg, J = 500 kg m^2.  Each tank is first brought to rest
(the paper initialises the fluid at rest after a preliminary simulation,
Section 5.1): ``relax_cycles`` times, ``relax_steps`` unforced steps followed
by zeroing every velocity (kinetic damping).  Then ``n_steps`` forced steps
are logged every ``log_stride`` steps; the target is the mean body-frame slosh
wrench over each log interval, the inputs the logged (theta, thetadot, input
torque) and the per-tank constants: the fill ratio and, as an extension of the
window's inputs, the tank's shape (0 rectangle, 1 circle) and its particle
spacing dx in mm (without them the network cannot tell how large the tank's
resting wall forces are, which set the mean of the wrench).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
from typing import Optional, Sequence

import numpy as np
import torch

import workloads as W

from ._lib import check, load
from .mlp import Mlp
from .sph import Simulator

WINDOW = 32


N_STATIC = 3               # per-tank constants: fill ratio, shape, dx [mm]


@dataclasses.dataclass
class RolloutSet:
    feat: torch.Tensor      # [R, T, 3] theta, thetadot, input torque (device)
    static: torch.Tensor    # [R, N_STATIC] fill ratio, shape (0 rect, 1 circle), dx in mm (device)
    wrench: torch.Tensor    # [R, T, 3] mean body-frame wrench per log interval (device)
    n_fluid: np.ndarray     # [R]
    sph_seconds: float      # GPU time of the logged (forced) rollouts
    sph_steps: int          # SPH steps per rollout (logged part)
    y: Optional[torch.Tensor] = None     # [R, T, 6] r, theta, rdot, thetadot per log sample (device)
    u: Optional[torch.Tensor] = None     # [R, sph_steps, 3] applied force and torque per step (device)
    body: Optional[torch.Tensor] = None  # [R, 3] body mass, inertia, dt (device, float64)
    log_stride: int = 0

    @property
    def fill(self) -> torch.Tensor:
        return self.static[:, 0]


def _relax(sim: Simulator, cycles: int, steps: int) -> None:
    zero_rigid = np.zeros((sim.T, 6))
    for _ in range(cycles):
        sim.rollout(steps)
        s, _, _, _, _ = sim.get_state()
        sim.set_state(s, torch.zeros_like(s), zero_rigid, 0.0, 0)


def generate(seeds: Sequence[int], n_steps: int = 5000, log_stride: int = 25, relax_cycles: int = 40,
             relax_steps: int = 100, n_min: int = 2000, n_max: int = 60000, device="cuda:0",
             batch: int = 256, lanes: Optional[int] = None, eos: int = W.EOS_TAIT_CLAMPED,
             log=None, jitter_seed: Optional[int] = None) -> RolloutSet:
    """Runs one relaxed, forced rollout per seed, up to ``batch`` tanks per
    handle (one set of launches).  sph_seconds sums the GPU time of the forced
    rollouts (relaxation excluded).  eos: the Tait law without tension by
    default; with the literal one (W.EOS_TAIT) the zero-gravity fluid
    oscillates by itself (tensile instability) and its wrench does not
    follow the inputs."""
    dev = torch.device(device)
    R = len(seeds)
    T = (n_steps + log_stride - 1) // log_stride
    feat = torch.empty(R, T, 3, device=dev)
    wrench = torch.empty(R, T, 3, device=dev)
    static = torch.empty(R, N_STATIC, device=dev)
    y_all = torch.empty(R, T, 6, device=dev)
    u_all = torch.empty(R, n_steps, 3, device=dev)
    body = torch.empty(R, 3, device=dev, dtype=torch.float64)
    n_fluid = np.zeros(R, np.int64)
    sph_seconds = 0.0
    for g0 in range(0, R, batch):
        idx = list(range(g0, min(R, g0 + batch)))
        scs = [W.random_tank(int(seeds[i]), n_steps=n_steps, n_min=n_min, n_max=n_max, eos=eos,
                             jitter_seed=jitter_seed) for i in idx]
        for i, sc in zip(idx, scs):
            n_fluid[i] = sc.n_fluid
            static[i] = torch.tensor([float(sc.fill), 1.0 if sc.shape == "circle" else 0.0, sc.dx * 1e3])
            body[i] = torch.tensor([sc.params.body_mass, sc.params.body_inertia, sc.params.dt], dtype=torch.float64)
        sim = Simulator.batch(scs, device=dev)
        if lanes:
            sim.set_lanes(lanes)
        _relax(sim, relax_cycles, relax_steps)
        u = torch.stack([torch.as_tensor(sc.u_seq) for sc in scs]).to(dev)
        torch.cuda.synchronize(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        lg = sim.rollout(n_steps, u, log_stride=log_stride)
        e1.record(sim.stream)
        e1.synchronize()
        sph_seconds += e0.elapsed_time(e1) / 1e3
        st = sim.status()
        if st != 0:
            raise RuntimeError(f"rollouts of seeds {seeds[idx[0]]}..{seeds[idx[-1]]} raised status {st}")
        sl = slice(idx[0], idx[-1] + 1)
        feat[sl, :, 0] = lg["y"][:, :, 2]
        feat[sl, :, 1] = lg["y"][:, :, 5]
        feat[sl, :, 2] = lg["u"][:, :, 2]
        wrench[sl] = lg["wrench_mean"]
        y_all[sl] = lg["y"]
        u_all[sl] = u
        sim.close()
        if log is not None:
            log(f"rollouts {idx[-1] + 1}/{R} done ({sph_seconds:.1f} s of SPH so far)")
    return RolloutSet(feat, static, wrench, n_fluid, sph_seconds, n_steps, y_all, u_all, body, log_stride)


def norm_from(data: RolloutSet, n_static: int = N_STATIC) -> np.ndarray:
    """Mean and std of the inputs (theta, thetadot, torque, then the first
    n_static per-tank constants) and of the targets, as the
    2 (3 + n_static) + 6 numbers mlp_make_windows takes (n_static = 1: the
    fill ratio alone, the configured window)."""
    f = data.feat.reshape(-1, 3).double()
    st = data.static[:, :n_static].double()
    in_mean = torch.cat([f.mean(0), st.mean(0)])
    in_std = torch.cat([f.std(0), st.std(0)])
    w = data.wrench.reshape(-1, 3).double()
    out_mean, out_std = w.mean(0), w.std(0)
    v = torch.cat([in_mean, in_std.clamp_min(1e-12), out_mean, out_std.clamp_min(1e-12)])
    return v.cpu().numpy().astype(np.float32)


def _n_static(norm: np.ndarray) -> int:
    return (len(norm) - 12) // 2


def out_norm(norm: np.ndarray):
    """(output means [3], output stds [3]) of a norm vector."""
    k = 2 * (3 + _n_static(norm))
    return norm[k:k + 3], norm[k + 3:k + 6]


def windows(data: RolloutSet, norm: np.ndarray, with_targets: bool = True, stream=None):
    """(x [n, 128], y [n, 3]) standardised, built by the window kernel."""
    L = load()
    R, T, _ = data.feat.shape
    n = R * (T - WINDOW + 1)
    dev = data.feat.device
    x = torch.empty(n, WINDOW * 4, device=dev)
    y = torch.empty(n, 3, device=dev) if with_targets else None
    ns = _n_static(norm)
    stat = data.static[:, :ns].contiguous()
    nm = (C.c_float * len(norm))(*[float(v) for v in norm])
    st = torch.cuda.current_stream(dev) if stream is None else stream
    check(L.mlp_make_windows(C.c_void_p(data.feat.data_ptr()), C.c_void_p(stat.data_ptr()), ns,
                             C.c_void_p(data.wrench.data_ptr()) if with_targets else None, int(R), int(T),
                             WINDOW, nm, C.c_void_p(x.data_ptr()),
                             C.c_void_p(y.data_ptr()) if with_targets else None,
                             C.c_void_p(st.cuda_stream)), "mlp_make_windows")
    return x, y


def init_params(seed: int = 0) -> np.ndarray:
    """Fan-in uniform initialisation, packed in the C-ABI order."""
    from .mlp import DIMS, pack
    rng = np.random.default_rng(seed)
    params = []
    for i in range(len(DIMS) - 1):
        bound = 1.0 / math.sqrt(DIMS[i])
        params.append((rng.uniform(-bound, bound, (DIMS[i + 1], DIMS[i])),
                       rng.uniform(-bound, bound, DIMS[i + 1])))
    return pack(params)


def train(x: torch.Tensor, y: torch.Tensor, epochs: int = 10, batch: int = 4096, lr: float = 1e-3,
          seed: int = 0, lr_final: float = 1e-4, device="cuda:0", log=None) -> Mlp:
    """Adam on the mean squared error, shuffled minibatches, cosine-decayed lr."""
    net = Mlp(init_params(seed), max_batch=batch, device=device)
    n = x.shape[0]
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    gen = torch.Generator(device=x.device)
    gen.manual_seed(seed)
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device=x.device, generator=gen)
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            a = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * k / max(1, total - 1)))
            loss, _ = net.train_step(x.index_select(0, idx), y.index_select(0, idx), lr=a)
            k += 1
        if log is not None:
            log(f"epoch {ep + 1}/{epochs}: batch loss {float(loss.item()):.4e}")
    return net


def inference_net(net: Mlp, max_batch: int = 65536) -> Mlp:
    """A handle for large inference batches with the trained weights."""
    return Mlp(net.params().cpu().numpy(), max_batch=max_batch, device=net.device)


def predict(net: Mlp, x: torch.Tensor, batch: int = 65536) -> torch.Tensor:
    out = torch.empty(x.shape[0], 3, device=x.device)
    step = min(batch, net.max_batch)
    for b in range(0, x.shape[0], step):
        net.forward(x[b:b + step], out=out[b:b + step])
    return out


def nrmse(pred_std: torch.Tensor, y_std: torch.Tensor, norm: np.ndarray) -> np.ndarray:
    """Per-channel RMS(prediction - SPH) / RMS(SPH), in physical units."""
    om, osd = out_norm(norm)
    mean = torch.as_tensor(om, device=y_std.device)
    std = torch.as_tensor(osd, device=y_std.device)
    p = pred_std * std + mean
    t = y_std * std + mean
    err = torch.sqrt(((p - t) ** 2).mean(0))
    ref = torch.sqrt((t ** 2).mean(0))
    return (err / ref).cpu().numpy()


def noise_floor(a: RolloutSet, b: RolloutSet, first: int = WINDOW - 1) -> np.ndarray:
    """Per-channel RMS(wrench_b - wrench_a) / RMS(wrench_a) of two sets of
    rollouts of the same tanks and inputs that differ only in the initial
    jitter, over the samples a window's target can take (from index
    ``first`` on): how far SPH itself reproduces its wrench.  A predictor
    that knew the part common to both would reach about this / sqrt(2)
    against either set when the difference is independent noise."""
    wa = a.wrench[:, first:].reshape(-1, 3).double()
    wb = b.wrench[:, first:].reshape(-1, 3).double()
    err = torch.sqrt(((wb - wa) ** 2).mean(0))
    ref = torch.sqrt((wa ** 2).mean(0))
    return (err / ref).cpu().numpy()


def time_inference(net: Mlp, x: torch.Tensor, reps: int = 20) -> float:
    """Seconds per forward pass of the batch x (HIP events around reps
    back-to-back launches on the network's stream, after a warm-up); x must
    fit the handle's max_batch."""
    x = x.to(torch.float32).contiguous()
    out = torch.empty(x.shape[0], 3, device=x.device)
    net.forward(x, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(net.stream)
    for _ in range(reps):
        net.launch(x, out)
    e1.record(net.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


# The rigid-body channels a coupled run is judged on: r_x, r_y, theta,
# rdot_x, rdot_y, thetadot.
TRAJ_CHANNELS = ("r_x", "r_y", "theta", "rdot_x", "rdot_y", "thetadot")


def coupled(net: Mlp, data: RolloutSet, norm: np.ndarray, z_max: float = 6.0) -> dict:
    """The rollouts of `data` again, the rigid body driven by the network
    instead of SPH from sample WINDOW - 1 on (``mlp_coupled_rollout``): the
    first window and the state at the hand-over come from SPH's logs, the
    inputs are the same.  Returns the coupled run's logs, its flags and its
    GPU seconds (HIP events on the network's stream)."""
    ns = _n_static(norm)
    dev = net.device
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    e0.record(net.stream)
    res = net.coupled_rollout(norm, data.static[:, :ns], data.feat[:, :WINDOW], data.y[:, WINDOW - 1].double(),
                              data.u, data.body, data.log_stride, z_max=z_max, window=WINDOW)
    e1.record(net.stream)
    e1.synchronize()
    res["seconds"] = e0.elapsed_time(e1) / 1e3
    return res


def trajectory_nrmse(y: torch.Tensor, ref: RolloutSet, first: int = WINDOW) -> np.ndarray:
    """Per rigid-body channel (TRAJ_CHANNELS), RMS(y - SPH) / RMS(SPH - SPH
    at the hand-over) over the samples from `first` on: the error of a
    trajectory against SPH's, relative to the motion SPH made after the
    hand-over at sample WINDOW - 1."""
    y_ref = ref.y.double()
    d = (y[:, first:].double() - y_ref[:, first:]).reshape(-1, 6)
    m = (y_ref[:, first:] - y_ref[:, WINDOW - 1:WINDOW]).reshape(-1, 6)
    return (torch.sqrt((d ** 2).mean(0)) / torch.sqrt((m ** 2).mean(0))).cpu().numpy()


def constant_net(norm: np.ndarray, max_batch: int, device="cuda:0") -> Mlp:
    """A network whose output is the training-mean wrench for every window
    (all weights zero): the rigid body with the fluid's mean wrench, the
    baseline a coupled surrogate must beat."""
    from .mlp import N_PARAMS
    return Mlp(np.zeros(N_PARAMS, np.float32), max_batch=max_batch, device=device)


def coupled_or_sph(net: Mlp, data: RolloutSet, norm: np.ndarray, scenarios, z_max: float = 6.0,
                   relax=None) -> dict:
    """The surrogate with SPH as its fallback: the coupled run of every
    rollout, then the rollouts whose windows left the training range
    (MLP_FLAG_OUT_OF_RANGE) simulated again by SPH from the same start;
    their logs replace the coupled ones.  `scenarios` are the rollouts'
    workloads.Scenario objects (the SPH fallback needs the tanks), `relax`
    the relaxation applied before their forced steps, as for the data
    (cycles, steps).  Returns the merged y [R, T, 6] and wrench [R, T, 3],
    the flags and the indices that fell back."""
    res = coupled(net, data, norm, z_max)
    flags = res["flags"].cpu().numpy()
    back = [int(i) for i in np.nonzero(flags & 1)[0]]
    y, w = res["y"].clone(), res["wrench"].clone()
    if back:
        sim = Simulator.batch([scenarios[i] for i in back], device=net.device)
        if relax is not None:
            _relax(sim, *relax)
        lg = sim.rollout(data.sph_steps, data.u[back], log_stride=data.log_stride)
        y[back] = lg["y"]
        w[back] = lg["wrench_mean"]
        sim.close()
    return dict(y=y, wrench=w, flags=res["flags"], fell_back=back, seconds=res["seconds"])
