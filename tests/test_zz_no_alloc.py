"""The allocation-free gradient entry point against the workspace one.

lbm_mlp_grad_noalloc keeps the per-workgroup gradient partials in the
library's fixed device array instead of a caller workspace.  Through the C
ABI it must give the same loss and gradient as lbm_mlp_grad on the same
inputs (the same kernels and the same fixed-order reduction, so the results
are bitwise equal), on two calls in a row, the second with a smaller batch
(the array keeps the first call's contents), in both arithmetic modes.  A
batch above the stated maximum is rejected on the host.
"""
import numpy as np
import pytest

from paper_2403_11167_amd import inputs, lbm

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = np.stack([rng.integers(0, 2, n), rng.uniform(0.5, 0.95, n), rng.uniform(2, 8, n),
                  rng.uniform(0.5, 2, n)], axis=1).astype(np.float32)
    y = np.exp(rng.standard_normal((n, 4))).astype(np.float32)
    return x, y


@pytest.mark.parametrize("bf16", [False, True])
def test_noalloc_gradient_equals_workspace_gradient(bf16):
    import torch
    dev = torch.device("cuda:0")
    norm = lbm.MlpNorm.make([0.5, 0.725, 5.0, 1.25], [2.0, 2 / 0.45, 1 / 3, 2 / 1.5],
                            [0.0] * 4, [1.0] * 4)
    theta = torch.from_numpy(inputs.mlp_initial_params(3)).to(dev)
    # a full-size batch, then a smaller one drawn through an index list
    x, y = _data(lbm.MLP_NOALLOC_MAX_N, 21)
    xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    idx = torch.from_numpy(np.random.default_rng(5).permutation(lbm.MLP_NOALLOC_MAX_N)[:77]
                           .astype(np.int32)).to(dev)
    for call, (ix, n) in enumerate([(None, lbm.MLP_NOALLOC_MAX_N), (idx, 77)]):
        print(f"noalloc call {call}: n={n} bf16={bf16}", flush=True)
        l_ws, g_ws = lbm.mlp_grad(theta, norm, xd, yd, idx=ix, n=n, bf16=bf16)
        l_na, g_na = lbm.mlp_grad_noalloc(theta, norm, xd, yd, idx=ix, n=n, bf16=bf16)
        torch.cuda.synchronize()
        g_ws, g_na = g_ws.cpu().numpy(), g_na.cpu().numpy()
        assert np.isfinite(g_ws).all() and np.abs(g_ws).max() > 0
        assert np.array_equal(g_na, g_ws), float(np.abs(g_na - g_ws).max())
        assert float(l_na.cpu()[0]) == float(l_ws.cpu()[0])


def test_noalloc_rejects_batches_above_the_maximum():
    import torch
    dev = torch.device("cuda:0")
    norm = lbm.MlpNorm.make([0.0] * 4, [1.0] * 4, [0.0] * 4, [1.0] * 4)
    theta = torch.from_numpy(inputs.mlp_initial_params(3)).to(dev)
    n = lbm.MLP_NOALLOC_MAX_N + 1
    x, y = _data(n, 4)
    with pytest.raises(lbm.LbmError) as e:
        lbm.mlp_grad_noalloc(theta, norm, torch.from_numpy(x).to(dev),
                             torch.from_numpy(y).to(dev))
    assert e.value.status == lbm.ERR_WORKSPACE
