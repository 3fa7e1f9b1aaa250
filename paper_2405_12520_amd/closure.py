"""Training pipeline of the learned car-following closure.

1. Trajectories on the 10 x 10 grid network, in IDM mode with the trace on:
   the grid workload itself (20k vehicles, shortest-path demand over an
   hour), whose traffic is light, and two dense starts on the same network
   (18k and 9k vehicles pre-placed at random speeds, 600 steps each), which
   supply the congested states (short gaps at low speed, stop-and-go) that the
   light workload rarely reaches.  Every step yields, for each active
   vehicle, the 8 closure inputs and the IDM acceleration (the label).
   Steps are split into training and held-out sets by step index (every 10th
   step of each run is held out).
2. Input description: per-input mean and standard deviation for the
   normalisation, and the [0.1, 99.9] percentile range as the envelope
   outside which the simulator keeps IDM.
3. Training: Adam on mean squared error with random batches (indices drawn
   on the host), forward/backward through the project's kernels
   (moss_mlp_grad), in bfloat16 mode so that training sees the simulator's
   rounding.

The network's arithmetic (traces, forward, backward, Adam, inference) runs
in libmoss kernels; the input description and the error statistics are FP64
numpy on host copies.  torch only holds the device tensors.
"""
from __future__ import annotations

import os
import time
from typing import Dict

import numpy as np

from . import moss
from . import scenarios as S

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "data", "closure_grid10.npz")
MLP_PARAMS = moss.MLP_PARAMS


DENSE_STARTS = ((18000, 600), (9000, 600))    # (vehicles, steps) pre-placed on the grid


def _trace_run(sc, steps, k0, feats, labs, steps_idx, log, name):
    import torch
    sim = moss.Simulator(sc, trace=True)
    t0 = time.time()
    for k in range(steps):
        sim.step(1)
        f, y = sim.trace(device=True)
        if f.shape[0]:
            feats.append(f.clone())
            labs.append(y.clone())
            steps_idx.append(torch.full((f.shape[0],), k0 + k, dtype=torch.int32,
                                        device=f.device))
        if log and (k + 1) % 600 == 0:
            log(f"[closure] {name}: traced {k + 1} steps, "
                f"{sum(x.shape[0] for x in labs)} samples, {time.time() - t0:.1f} s")
    sim.close()


def collect(steps: int = 3600, n_veh: int = 20000, dense=DENSE_STARTS, log=print):
    """Traces the grid workload and the dense starts on the same network;
    returns device tensors (features, labels, step index) of all
    vehicle-steps.  Step indices of the runs follow one another, each run
    starting at a multiple of 10."""
    import torch
    feats, labs, steps_idx = [], [], []
    _trace_run(S.grid(10, n_veh), steps, 0, feats, labs, steps_idx, log, "grid workload")
    k0 = (steps + 9) // 10 * 10
    for nv, st in dense:
        _trace_run(S.grid_snapshot(10, nv), st, k0, feats, labs, steps_idx, log,
                   f"dense start {nv}")
        k0 += (st + 9) // 10 * 10
    return torch.cat(feats), torch.cat(labs), torch.cat(steps_idx)


LOG_INPUTS = (0, 4, 6)      # distances enter the network as ln(max(x, 0.5 m))


def describe(F) -> np.ndarray:
    """mean[8], inv_std[8] of the network inputs (distances log-transformed)
    and lo[8], hi[8] of the raw inputs (the envelope: 0.1 % and 99.9 %
    quantiles, linear interpolation).  Computed in FP64 with numpy on a host
    copy of the features."""
    f = F.cpu().numpy().astype(np.float64) if hasattr(F, "cpu") else np.asarray(F, np.float64)
    ft = f.copy()
    for q in LOG_INPUTS:
        ft[:, q] = np.log(np.maximum(ft[:, q], 0.5))
    mean = ft.mean(0)
    std = np.maximum(ft.std(0, ddof=1), 1e-3)
    # quantiles on every k-th row (at most about a million per input)
    step = max(1, f.shape[0] // 1_000_000)
    lohi = np.quantile(f[::step], [0.001, 0.999], axis=0)
    return np.concatenate([mean, 1.0 / std, lohi[0], lohi[1]]).astype(np.float32)


def he_init(seed: int) -> np.ndarray:
    """He-style uniform initialisation of the parameter vector (seeded)."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, 64 * 8) * np.sqrt(3.0 / 8), np.zeros(64),
             rng.uniform(-1, 1, 64 * 64) * np.sqrt(3.0 / 64), np.zeros(64),
             rng.uniform(-1, 1, 64) * np.sqrt(3.0 / 64), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def fit(F, Y, norm: np.ndarray, *, steps: int = 60000, batch: int = 4096, lr: float = 2e-3,
        seed: int = 0, bf16: bool = True, log=print):
    """Adam training on the GPU through moss_mlp_grad / moss_mlp_adam with a
    cosine-decayed learning rate, on the output limited as the simulator
    limits it; the last quarter of the steps (all of them unless bf16)
    rounds weights and activations to bfloat16 as the simulator does.
    Returns the FP32 master parameters."""
    import torch
    dev = F.device
    N = torch.from_numpy(norm).to(dev)
    th = torch.from_numpy(he_init(seed)).to(dev)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    rng = np.random.default_rng(seed)
    n = F.shape[0]
    t0 = time.time()
    block = 256                 # steps whose batch indices are copied at once
    for s in range(1, steps + 1):
        if (s - 1) % block == 0:
            k = min(block, steps - s + 1)
            idx_blk = torch.from_numpy(rng.integers(0, n, (k, batch), dtype=np.int32)).to(dev)
        idx = idx_blk[(s - 1) % block]
        q = bf16 and s > (3 * steps) // 4
        loss, g = moss.mlp_grad(F, Y, th, N, idx=idx, bf16=q, out_lo=-S.DEFAULT_PARAMS["b_max"],
                                out_hi=S.DEFAULT_PARAMS["a_max"])
        lr_s = lr * 0.5 * (1.0 + np.cos(np.pi * (s - 1) / steps)) + 1e-5
        moss.mlp_adam(th, m, v, g, s, lr=float(lr_s))
        if log and s % 10000 == 0:
            log(f"[closure] step {s}: batch loss {float(loss.item()):.4f} "
                f"({time.time() - t0:.1f} s)")
    return th.cpu().numpy()


def rms(F, Y, theta: np.ndarray, norm: np.ndarray, inside_only: bool = True) -> Dict[str, float]:
    """RMS error of the network (simulator inference path, the project's
    kernel) against the labels, over the samples inside the envelope (or
    all); the error arithmetic is FP64 numpy on host copies."""
    import torch
    dev = F.device
    pred = moss.mlp_predict(F, torch.from_numpy(theta).to(dev), torch.from_numpy(norm).to(dev))
    f = F.cpu().numpy()
    y = Y.cpu().numpy().astype(np.float64)
    p = pred.cpu().numpy().astype(np.float64)
    inside = np.all((f >= norm[16:24]) & (f <= norm[24:32]), axis=1)
    amax, bmax = S.DEFAULT_PARAMS["a_max"], S.DEFAULT_PARAMS["b_max"]
    e = np.clip(p, -bmax, amax) - y
    if inside_only:
        e = e[inside]
    return dict(rms=float(np.sqrt(np.mean(e * e))) if e.size else 0.0,
                inside=float(inside.mean()), n=int(e.shape[0]))


def build_closure(path: str = DEFAULT_PATH, *, steps_trace: int = 3600,
                  train_steps: int = 150000, log=print):
    """Full pipeline; writes theta and norm to path (npz) and returns them."""
    import torch
    F, Y, K = collect(steps_trace, log=log)
    held = (K % 10) == 9
    Ftr, Ytr = F[~held], Y[~held]
    norm = describe(Ftr)
    theta = fit(Ftr, Ytr, norm, steps=train_steps, log=log)
    ev = rms(F[held], Y[held], theta, norm)
    if log:
        log(f"[closure] held-out RMS {ev['rms']:.4f} m/s^2 on {ev['n']} samples, "
            f"{100 * ev['inside']:.2f} % inside the envelope")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, theta=theta, norm=norm, heldout_rms=ev["rms"], inside=ev["inside"])
    del torch
    return theta, norm, ev


def load(path: str = DEFAULT_PATH):
    z = np.load(path)
    return z["theta"].astype(np.float32), z["norm"].astype(np.float32)


if __name__ == "__main__":
    build_closure()
