"""The allocation-free MLP backward pass (fixed device scratch) against the
allocating one, through the C ABI: two calls in a row, the second with a
smaller batch, so that the second reads a scratch that still holds the
first call's deltas.  Both passes run the same kernels in the same order,
so the gradients must agree bit for bit; both are also checked against the
FP64 oracle at the FP32 bound of the MLP parity tests (1e-4 relative)."""
import numpy as np
import pytest
import torch

import paper_1808_03595_amd as pmg
from oracle import mlp

pytestmark = pytest.mark.gpu


def _case(gpu, nout, B, seed):
    rng = np.random.default_rng(seed)
    th = (mlp.glorot_init(nout, seed) + 0.05 * rng.normal(size=mlp.nparams(nout))).astype(np.float32)
    x = rng.uniform(0, 1, size=(B, 3)).astype(np.float32)
    dy = rng.normal(size=(B, nout)).astype(np.float32)
    dp = torch.as_tensor(th, device=gpu)
    dx = torch.as_tensor(x, device=gpu)
    y = torch.empty(B, nout, dtype=torch.float32, device=gpu)
    cache = torch.empty(B, 128 + nout, dtype=torch.float32, device=gpu)
    pmg.mlp_forward(dp, dx, y, cache, B, nout)
    return th, x, dy, dp, dx, cache


@pytest.mark.parametrize("nout", [4, 3])
def test_noalloc_backward_equals_allocating(gpu, nout):
    for B, seed in ((3000, 11), (129, 12)):   # second call smaller than the first
        th, x, dy, dp, dx, cache = _case(gpu, nout, B, seed)
        ddy = torch.as_tensor(dy, device=gpu)
        g_ref = torch.full((th.size,), float("nan"), dtype=torch.float32, device=gpu)
        g_new = torch.full((th.size,), float("nan"), dtype=torch.float32, device=gpu)
        pmg.mlp_backward(dp, dx, cache, ddy, g_ref, B, nout)
        pmg.mlp_backward_noalloc(dp, dx, cache, ddy, g_new, B, nout)
        torch.cuda.synchronize()
        a, b = g_ref.cpu().numpy(), g_new.cpu().numpy()
        assert np.isfinite(b).all()
        assert np.array_equal(a, b), (B, float(np.abs(a - b).max()))
        _, c64 = mlp.forward(th.astype(np.float64), x.astype(np.float64), nout)
        rg = mlp.backward(th.astype(np.float64), c64, dy.astype(np.float64), nout)
        assert np.linalg.norm(b - rg) <= 1e-4 * np.linalg.norm(rg)


def test_noalloc_backward_rejects_oversize(gpu):
    nout = 4
    th, x, dy, dp, dx, cache = _case(gpu, nout, 8, 0)
    g = torch.empty(th.size, dtype=torch.float32, device=gpu)
    big = (1 << 21) // (128 + nout) + 1
    with pytest.raises(pmg.PmgError) as e:
        pmg.mlp_backward_noalloc(dp, dx, cache, dp, g, big, nout)
    assert e.value.code == -4
