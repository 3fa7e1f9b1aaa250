"""Pins of the FP64 MLP reference (test infrastructure) against mathematics
that does not come from it: central finite differences of the loss, the
exact erf form of GELU, bfloat16 rounding rules, and Adam's first step."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_tanh_form_close_to_erf_form():
    """The tanh form approximates x * Phi(x) (Hendrycks & Gimpel) to < 5e-4."""
    x = np.linspace(-8, 8, 4001)
    exact = 0.5 * x * (1 + np.array([math.erf(t / math.sqrt(2)) for t in x]))
    assert np.abs(mlp.gelu(x) - exact).max() < 5e-4


def test_gelu_grad_matches_finite_differences():
    x = np.linspace(-6, 6, 601)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(x)).max() < 1e-7


def test_bf16_rounding_rules():
    """Round to nearest with ties to even on the 16 dropped mantissa bits."""
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-9, 1.0 + 3 * 2**-9, -2.5, 3.14159265], np.float32)
    got = mlp.bf16(vals)
    assert got[0] == 1.0
    assert got[1] == 1.0 + 2**-7 or got[1] == 1.0  # representable step is 2^-7
    assert got[2] == 1.0                           # tie -> even (1.0)
    assert got[3] == 1.0 + 2**-7                   # tie -> even (mantissa ...1 -> ...10)
    assert got[4] == -2.5
    assert abs(got[5] - 3.140625) < 1e-12
    # every result is representable in 8 mantissa bits
    u = got.astype(np.float32).view(np.uint32)
    assert np.all((u & 0xFFFF) == 0)


def test_bf16_pair_inputs():
    """A network input as two bfloat16 numbers: exact for values that are
    already bfloat16, within 2^-16 relative otherwise (each part drops 8
    mantissa bits of what is left), and both parts representable."""
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(100000) * np.exp(rng.uniform(-6, 6, 100000))).astype(np.float32)
    got = mlp.bf16x2(x)
    assert np.all(np.abs(got - x.astype(np.float64)) <= 2.0**-16 * np.abs(x))
    b = mlp.bf16(x).astype(np.float32)
    assert np.array_equal(mlp.bf16x2(b), b.astype(np.float64))
    hi = mlp.bf16(x)
    lo = got - hi
    for part in (hi, lo):
        u = part.astype(np.float32).view(np.uint32)
        assert np.all((u & 0xFFFF) == 0)
    # about 8 more bits than one bfloat16: mean relative errors ~2^-17 vs ~2^-9
    rel = lambda y: np.mean(np.abs(y - x) / np.abs(x))
    assert rel(got) < 2.0**-7 * rel(hi)


def test_c_oracle_forward_equals_fp64_reference():
    """The C oracle's network (MLP mode) and the numpy reference implement
    the same rounded network: equal to FP64 summation-order differences."""
    from oracle import mlp_forward
    rng = np.random.default_rng(9)
    for k in range(5):
        th = mlp.init_params(30 + k)
        th[mlp.N_PARAMS - 65:mlp.N_PARAMS] = rng.normal(0, 0.3, 65).astype(np.float32)
        z = rng.normal(0, 1.5, (50, 8)).astype(np.float32)
        ref, _ = mlp.forward(th.astype(np.float64), z, bf16_mode=True)
        got = np.array([mlp_forward(th, z[i]) for i in range(z.shape[0])])
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_central_differences(seed):
    """Analytic gradient of the FP64 network equals central differences of
    the loss to 1e-6 relative (FP32 mode, i.e. no rounding)."""
    rng = np.random.default_rng(seed)
    theta = mlp.init_params(seed).astype(np.float64)
    z = rng.normal(size=(32, mlp.N_IN))
    lab = rng.normal(size=32)
    _, g = mlp.loss_and_grad(theta, z, lab)
    idx = rng.choice(mlp.N_PARAMS, size=60, replace=False)
    idx = np.concatenate([idx, [mlp.N_PARAMS - 1, 0]])   # include the biases' ends
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss_and_grad(tp, z, lab)[0] - mlp.loss_and_grad(tm, z, lab)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_adam_first_step_is_lr_times_sign():
    """With zero moments, Adam's bias-corrected first step is lr*g/(|g|+eps)."""
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t2, m, v = mlp.adam(theta, np.zeros(3), np.zeros(3), g, step=1, lr=1e-2)
    np.testing.assert_allclose(theta - t2, 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss_on_a_smooth_target():
    """A few hundred Adam steps fit a smooth function of the inputs (the
    training loop the GPU kernels implement)."""
    rng = np.random.default_rng(3)
    z = rng.normal(size=(512, mlp.N_IN))
    lab = np.tanh(z[:, 0]) - 0.5 * z[:, 1] * z[:, 2]
    theta = mlp.init_params(3).astype(np.float64)
    m = np.zeros_like(theta); v = np.zeros_like(theta)
    l0 = mlp.loss_and_grad(theta, z, lab)[0]
    for s in range(1, 301):
        l, g = mlp.loss_and_grad(theta, z, lab)
        theta, m, v = mlp.adam(theta, m, v, g, s, lr=3e-3)
    assert l < 0.1 * l0
