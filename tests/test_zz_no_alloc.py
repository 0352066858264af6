"""The surrogate prediction that allocates nothing (ij_mlp_predict_noalloc,
through the C ABI) against ij_mlp_predict on the same network and queries:
bit for bit the same mean and spread (the same kernels, the per-member
outputs in the library's fixed device array instead of a handle buffer), on
two calls in a row, the second with fewer queries, so that the second call
reads nothing the first left behind; sizes beyond the fixed array are
rejected before any device work."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

X_MEAN = np.array([90.0, 0.01, 1.5e-4, 1.5e-4, 1750.0, 1750.0, 1750.0])
X_STD = np.array([35.0, 0.004, 7e-5, 7e-5, 700.0, 700.0, 700.0])
Y_MEAN = np.array([20000.0, 0.01, 5000.0])
Y_STD = np.array([10000.0, 0.01, 3000.0])


def _queries(n, seed):
    u = W.uniform_array(seed, n * 7).reshape(n, 7)
    return (X_MEAN + X_STD * (2 * u - 1) * 1.7).astype(np.float32)


def test_predict_noalloc_matches_predict(gpu_lib):
    import torch
    L = gpu_lib
    members = 4
    net = L.MLP(members)
    net.set_scaling(X_MEAN, X_STD, Y_MEAN, Y_STD)
    for k in range(members):
        p = W.mlp_init(20 + k)
        p["b1"] = W.uniform_array(120 + k, 128, -0.2, 0.2)
        net.set_weights(k, p)
    for n, seed in ((100000, 5), (3001, 6)):   # the second call is smaller
        print("no-alloc prediction of", n, "queries", flush=True)
        x = torch.as_tensor(_queries(n, seed), device="cuda")
        mean_ref, spread_ref = net.predict(x)
        mean = torch.full((n, 4), float("nan"), device="cuda")
        spread = torch.full((n, 4), float("nan"), device="cuda")
        net.predict_into(x, mean, spread)
        torch.cuda.synchronize()
        assert torch.equal(mean, mean_ref) and torch.equal(spread, spread_ref), n
        assert bool(torch.isfinite(mean).all()) and bool((spread > 0).any())
    # beyond the fixed array: rejected, outputs untouched
    n_max = (1 << 21) // (members * 4)
    x = torch.zeros((n_max + 1, 7), device="cuda")
    mean = torch.zeros((n_max + 1, 4), device="cuda")
    spread = torch.zeros((n_max + 1, 4), device="cuda")
    with pytest.raises(L.LBMError) as e:
        net.predict_into(x, mean, spread)
    assert e.value.code == L.IJ_ERR_INVALID_ARG
    assert "scratch" in str(e.value)
    assert not bool(mean.any())
    # zero queries is a no-op
    e0 = torch.zeros((0, 7), device="cuda")
    net.predict_into(e0, torch.zeros((0, 4), device="cuda"), torch.zeros((0, 4), device="cuda"))
    net.close()
