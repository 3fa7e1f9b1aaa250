"""FP64 reference of the learned car-following closure -- TEST INFRASTRUCTURE.

The network is the small multilayer perceptron that replaces the IDM
acceleration inside the vehicle update when its inputs lie in the training
envelope: 8 normalised inputs -> 64 -> 64 -> 1 with GELU activations.
(The paper itself uses IDM only; the closure is this project's extension,
trained on trajectories the simulator produces, with IDM as label and
fallback.)

Parameter vector layout (float32, 4801 values):
    W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3[1]
BF16 mode rounds W1, W2, w3 and the hidden layer inputs (h1, h2) to bfloat16
(round to nearest even) before each product, and represents each network
input z as a pair of bfloat16 numbers, hi = bf16(z) and lo = bf16(z - hi)
(the difference in float32, where it is exact), so that the first layer sees
hi + lo: about 16 significant bits instead of 8.  Sums are exact here (FP64),
FP32 on the GPU.  Gradients in BF16 mode are those of the rounded network with
respect to the rounded weights (straight-through for the master weights).

GELU is the tanh form of Hendrycks & Gimpel (2016):
    g(x) = x/2 * (1 + tanh(sqrt(2/pi) * (x + 0.044715 x^3))).
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_H = 8, 64
SIZES = dict(W1=(N_H, N_IN), b1=(N_H,), W2=(N_H, N_H), b2=(N_H,), w3=(N_H,), b3=(1,))
N_PARAMS = sum(int(np.prod(s)) for s in SIZES.values())
K0 = math.sqrt(2.0 / math.pi)
K1 = 0.044715


LOG_INPUTS = (0, 4, 6)      # leader gap, red stop line, lane end: distances


def normalise(feat, norm):
    """Network input from the 8 raw inputs: the distances enter as
    ln(max(x, 0.5 m)), then z = (x' - mean) * inv_std (FP32 as the simulator
    computes it; the log in FP64 then rounded)."""
    f = np.asarray(feat, dtype=np.float32).copy()
    for q in LOG_INPUTS:
        f[:, q] = np.log(np.maximum(f[:, q].astype(np.float64), 0.5)).astype(np.float32)
    mean = np.asarray(norm[:8], np.float32)
    inv = np.asarray(norm[8:16], np.float32)
    return ((f - mean) * inv).astype(np.float32)


def unpack(theta):
    theta = np.asarray(theta)
    out, o = {}, 0
    for k, s in SIZES.items():
        n = int(np.prod(s))
        out[k] = theta[o:o + n].reshape(s)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in SIZES])


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def bf16x2(x):
    """A float32 value as the sum of two bfloat16 numbers (as float64)."""
    x32 = np.asarray(x, dtype=np.float32)
    hi = bf16(x32)
    lo = bf16((x32 - hi.astype(np.float32)).astype(np.float32))
    return hi + lo


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(K0 * (x + K1 * x ** 3)))


def gelu_grad(x):
    u = K0 * (x + K1 * x ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * K0 * (1.0 + 3.0 * K1 * x * x)


def init_params(seed: int):
    """He-style uniform initialisation (seeded)."""
    rng = np.random.default_rng(seed)
    p = dict(W1=rng.uniform(-1, 1, SIZES["W1"]) * math.sqrt(3.0 / N_IN),
             b1=np.zeros(N_H),
             W2=rng.uniform(-1, 1, SIZES["W2"]) * math.sqrt(3.0 / N_H),
             b2=np.zeros(N_H),
             w3=rng.uniform(-1, 1, SIZES["w3"]) * math.sqrt(3.0 / N_H),
             b3=np.zeros(1))
    return pack(p).astype(np.float32)


def forward(theta, z, bf16_mode=False):
    """Returns y [B] and the intermediate values for backward."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    z = np.asarray(z, dtype=np.float64)
    W1, W2, w3 = p["W1"], p["W2"], p["w3"]
    if bf16_mode:
        W1, W2, w3 = bf16(W1), bf16(W2), bf16(w3)
        z = bf16x2(z)
    a1 = z @ W1.T + p["b1"]
    h1 = gelu(a1)
    h1q = bf16(h1) if bf16_mode else h1
    a2 = h1q @ W2.T + p["b2"]
    h2 = gelu(a2)
    h2q = bf16(h2) if bf16_mode else h2
    y = h2q @ w3 + p["b3"][0]
    cache = dict(z=z, a1=a1, h1q=h1q, a2=a2, h2q=h2q, W1=W1, W2=W2, w3=w3)
    return y, cache


def loss_and_grad(theta, z, label, bf16_mode=False):
    """MSE loss and its gradient with respect to the parameter vector."""
    y, c = forward(theta, z, bf16_mode)
    label = np.asarray(label, dtype=np.float64)
    B = y.shape[0]
    r = y - label
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = {}
    g["w3"] = c["h2q"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, c["w3"])
    da2 = dh2 * gelu_grad(c["a2"])
    g["W2"] = da2.T @ c["h1q"]
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ c["W2"]
    da1 = dh1 * gelu_grad(c["a1"])
    g["W1"] = da1.T @ c["z"]
    g["b1"] = da1.sum(axis=0)
    return loss, pack(g)


def adam(theta, m, v, grad, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) in FP64; step counts from 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v
