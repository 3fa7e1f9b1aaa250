"""The gradient entry point that allocates nothing (moss_mlp_grad_static)
against the one that takes a caller's scratch (moss_mlp_grad).

Both run the same kernels, so the gradient and the loss must agree bit for
bit.  Two calls in a row on the library's static scratch, the first at the
largest batch it accepts and the second smaller, check that nothing of the
first call leaks into the second.  The loss is also held to the FP64
reference of the closure (oracle/mlp.py) at the tolerance of the workspace
entry point's own test.
"""
import sys

import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _features(rng, n):
    f = np.empty((n, 8), np.float32)
    f[:, 0] = rng.uniform(-2, 300, n)
    f[:, 1] = rng.uniform(0, 18, n)
    f[:, 2] = np.clip(f[:, 1] + rng.normal(0, 2, n), 0, 20)
    f[:, 3] = rng.uniform(8, 17, n)
    f[:, 4] = np.where(rng.random(n) < 0.3, rng.uniform(0, 300, n), 300.0)
    f[:, 5] = rng.uniform(-9, 2, n)
    f[:, 6] = rng.uniform(0, 300, n)
    f[:, 7] = rng.choice([11.11, 13.89, 16.67], n)
    return f


def _norm_for(f):
    ft = f.astype(np.float64).copy()
    for q in M.LOG_INPUTS:
        ft[:, q] = np.log(np.maximum(ft[:, q], 0.5))
    mean = ft.mean(0)
    inv = 1.0 / np.maximum(ft.std(0), 1e-3)
    lo = np.full(8, -1e9, np.float32)
    hi = np.full(8, 1e9, np.float32)
    return np.concatenate([mean, inv, lo, hi]).astype(np.float32)


@pytest.mark.parametrize("bf16", [True, False])
def test_static_scratch_gradient_equals_workspace_gradient(bf16):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_12520_amd import moss
    nmax = moss.MLP_STATIC_MAX_SAMPLES
    rng = np.random.default_rng(21)
    f = _features(rng, nmax + 500)
    nrm = _norm_for(f)
    lab = rng.normal(0, 1.5, f.shape[0]).astype(np.float32)
    th = M.init_params(5)
    F, Y = torch.from_numpy(f).cuda(), torch.from_numpy(lab).cuda()
    TH, N = torch.from_numpy(th).cuda(), torch.from_numpy(nrm).cuda()
    grad = torch.empty(moss.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    # first call: the largest batch, gathered through idx; second: smaller,
    # rows taken in order
    idx = torch.from_numpy(rng.permutation(f.shape[0])[:nmax].astype(np.int32)).cuda()
    cases = [("max batch via idx", dict(idx=idx), nmax),
             ("smaller batch in order", dict(), 1000)]
    for what, kw, n in cases:
        _say(f"mlp grad static vs workspace: {what}, n={n}, bf16={bf16}")
        Fn, Yn = (F, Y) if kw else (F[:n].contiguous(), Y[:n].contiguous())
        l_ws, g_ws = moss.mlp_grad(Fn, Yn, TH, N, bf16=bf16, **kw)
        moss.mlp_grad_static(Fn, Yn, TH, N, grad, loss, bf16=bf16, **kw)
        torch.cuda.synchronize()
        a, b = grad.cpu().numpy(), g_ws.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), \
            (what, int(np.sum(a != b)))
        assert loss.item() == l_ws.item(), (what, loss.item(), l_ws.item())
        rows = idx.cpu().numpy() if kw else np.arange(n)
        z = M.normalise(f[rows], nrm)
        ref_loss, _ = M.loss_and_grad(th.astype(np.float64), z, lab[rows], bf16_mode=bf16)
        tol = 2e-2 if bf16 else 1e-4
        assert abs(float(loss.item()) - ref_loss) <= tol * ref_loss, (what, loss.item(), ref_loss)


def test_static_scratch_rejects_a_batch_beyond_its_size():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_12520_amd import moss
    n = moss.MLP_STATIC_MAX_SAMPLES + 1
    F = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    Y = torch.zeros(n, dtype=torch.float32, device="cuda")
    TH = torch.zeros(moss.MLP_PARAMS, dtype=torch.float32, device="cuda")
    N = torch.zeros(moss.MLP_NORM, dtype=torch.float32, device="cuda")
    grad = torch.empty(moss.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    with pytest.raises(moss.MossError) as e:
        moss.mlp_grad_static(F, Y, TH, N, grad, loss)
    assert e.value.code == -1 and "at most" in str(e.value)
