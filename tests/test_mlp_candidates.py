"""Pins of the oracle's admissible closure outputs (orc_mlp_candidates).

The closure's definition rounds hidden activations to bfloat16; an FP32
evaluation (sums in another order, GELU through exp2 and a reciprocal, the
logarithm of a distance within an ulp) may round an activation that lies
close to a bfloat16 boundary the other way.  The candidate list is the
network-mode parity tolerance, so it is pinned here on the CPU:

- its first entry is the oracle's own output, bit for bit the acceleration
  the oracle's network-mode step gives;
- every output of emulated FP32 evaluations (numpy float32, random
  summation orders, perturbed exp2, reciprocal and logarithm) lies within
  the output sum's rounding of some candidate, and some of those outputs are
  NOT the oracle's own value (so the check has teeth);
- a tie built by hand (a hidden unit placed on a rounding boundary) yields
  exactly the two roundings.
"""
import numpy as np
import pytest

from oracle import OracleSim, mlp_candidates, mlp_forward
from oracle import mlp as M
from paper_2405_12520_amd import closure
from paper_2405_12520_amd import scenarios as S

B_MAX, A_MAX = 9.0, 2.0


@pytest.fixture(scope="module")
def grid_inputs():
    theta, norm = closure.load(closure.DEFAULT_PATH)
    sc = S.grid_snapshot(10, 6000).with_params(mlp=dict(theta=theta, norm=norm))
    o = OracleSim(sc)
    o.step(1)
    f, use = o.mlp_inputs()
    dbg = o.debug()
    st = o.state()
    return theta, norm, f, use, dbg, st


def test_first_candidate_is_the_oracle_step(grid_inputs):
    theta, norm, f, use, dbg, st = grid_inputs
    ev = use == 1
    assert ev.mean() > 0.5
    out, cnt, info = mlp_candidates(theta, norm, f[ev], -B_MAX, A_MAX)
    assert (cnt >= 1).all()
    a_by_id = dict(zip(st["id"].tolist(), st["a"].tolist()))
    got = np.array([a_by_id.get(int(i), np.nan) for i in dbg["id"][ev]], np.float32)
    keep = ~np.isnan(got)
    assert keep.mean() > 0.99
    assert np.array_equal(out[keep, 0].astype(np.float32).view(np.uint32),
                          got[keep].view(np.uint32))


def _f32(x):
    return np.asarray(x, dtype=np.float32)


def _nudge(x, rng, k=1):
    """x moved by a random number of float32 ulps in [-k, k]."""
    x = _f32(x).copy()
    steps = rng.integers(-k, k + 1, size=x.shape)
    for s in range(1, k + 1):
        x = np.where(steps >= s, np.nextafter(x, _f32(np.inf)), x)
        x = np.where(steps <= -s, np.nextafter(x, _f32(-np.inf)), x)
    return x


def _gelu32(x, rng):
    """x / (1 + 2^(x (c0 + c1 x^2))) in float32, exp2 and reciprocal each off
    by up to one ulp."""
    c0 = _f32(-2.0 * M.K0 * 1.4426950408889634)
    c1 = _f32(-2.0 * M.K0 * M.K1 * 1.4426950408889634)
    xx = _f32(x * x)
    p = _f32(xx.astype(np.float64) * np.float64(c1) + np.float64(c0))
    with np.errstate(over="ignore"):
        e = _nudge(_f32(np.exp2(_f32(x * p).astype(np.float64))), rng)
        r = _nudge(_f32(1.0 / _f32(1.0 + e).astype(np.float64)), rng)
    return _f32(x * r)


def _sum32(bias, terms, order):
    """bias + sum of terms[..., k] in float32, added in the given order."""
    acc = _f32(bias).copy()
    for k in order:
        acc = _f32(acc + terms[..., k])
    return acc


def _emulated_fp32(theta, norm, f, rng):
    p = M.unpack(theta.astype(np.float32))
    W1 = _f32(M.bf16(p["W1"]))
    W2 = _f32(M.bf16(p["W2"]))
    w3 = _f32(M.bf16(p["w3"]))
    x = _f32(f).copy()
    for q in M.LOG_INPUTS:
        c = _f32(np.log(np.maximum(x[:, q].astype(np.float64), 0.5)))
        x[:, q] = _nudge(c, rng, k=1)
    z = _f32((x - _f32(norm[:8])) * _f32(norm[8:16]))
    hi = _f32(M.bf16(z))
    lo = _f32(M.bf16(_f32(z - hi)))
    zz = np.concatenate([hi, lo], axis=1)                        # [n, 16]
    t1 = _f32(zz[:, None, :] * np.concatenate([W1, W1], axis=1)[None])   # [n, 64, 16]
    a1 = _sum32(np.broadcast_to(_f32(p["b1"]), t1.shape[:2]), t1, rng.permutation(16))
    h1 = _f32(M.bf16(_gelu32(a1, rng)))
    t2 = _f32(h1[:, None, :] * W2[None])                         # [n, 64, 64]
    a2 = _sum32(np.broadcast_to(_f32(p["b2"]), t2.shape[:2]), t2, rng.permutation(64))
    h2 = _f32(M.bf16(_gelu32(a2, rng)))
    t3 = _f32(h2 * w3[None])
    y = _sum32(np.full(h2.shape[0], _f32(p["b3"][0])), t3, rng.permutation(64))
    return np.clip(y.astype(np.float64), -B_MAX, A_MAX)


def test_emulated_fp32_evaluations_are_candidates(grid_inputs):
    theta, norm, f, use, _, _ = grid_inputs
    fe = f[use == 1][:3000]
    out, cnt, info = mlp_candidates(theta, norm, fe, -B_MAX, A_MAX)
    rng = np.random.default_rng(17)
    off_nominal = 0
    for trial in range(6):
        y = _emulated_fp32(theta, norm, fe, rng)
        d = np.nanmin(np.abs(out - y[:, None]), axis=1)
        # the output layer's own FP32 sum: 67 u times the sum of |terms|
        assert d.max() < 1e-4, (trial, d.max(), int(np.argmax(d)))
        off_nominal += int((np.abs(y - out[:, 0]) > 1e-4).sum())
    # the emulations do land on other roundings than the oracle's own
    assert off_nominal > 0


def test_hand_built_tie_gives_both_roundings():
    """Hidden unit 0 of layer 1 sits on a bfloat16 rounding boundary (its
    pre-activation is a bias chosen by bisection so that GELU hits the
    midpoint between two bfloat16 numbers); layer 2 copies it to the output
    through unit 0.  The two candidates are the two roundings carried
    through; a unit far from any boundary adds none."""
    import math
    mid = 1.0 + 2.0 ** -8          # midpoint of bfloat16 1.0 and 1 + 2^-7
    lo, hi = 0.5, 2.0
    for _ in range(200):
        x = 0.5 * (lo + hi)
        if M.gelu(x) < mid:
            lo = x
        else:
            hi = x
    b1 = np.float32(x)
    p = {k: np.zeros(s) for k, s in M.SIZES.items()}
    p["b1"][0] = b1
    p["W2"][0, 0] = 1.0
    p["w3"][0] = 1.0
    theta = M.pack(p).astype(np.float32)
    norm = np.concatenate([np.zeros(8), np.ones(8), np.full(8, -1e9), np.full(8, 1e9)])
    f = np.full((1, 8), 10.0, np.float32)
    out, cnt, info = mlp_candidates(theta, norm.astype(np.float32), f, -100.0, 100.0)
    assert info[0, 0] == 1 and info[0, 3] == 0          # one tie, unit 0 of layer 1
    got = sorted(out[0, :cnt[0]])
    # unit 0 of layer 2 sees h1 = 1 or 1 + 2^-7 and outputs bf16(gelu(.)) of it
    want = sorted({M.bf16(np.float32(M.gelu(h))).item() for h in (1.0, 1.0 + 2.0 ** -7)})
    assert got == want, (got, want)
    # the oracle's own value is the rounding of its FP64 GELU
    h1 = M.bf16(np.float32(M.gelu(float(b1)))).item()
    assert out[0, 0] == M.bf16(np.float32(M.gelu(h1))).item()
    assert math.isclose(out[0, 0], mlp_forward(theta, np.zeros(8, np.float32)), rel_tol=0, abs_tol=0)
