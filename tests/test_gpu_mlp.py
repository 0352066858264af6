"""The surrogate network's matrix-core kernels against the FP64 reference
(oracle/mlp_oracle.py) through the C ABI: forward outputs, the loss and
its gradient per layer (bfloat16 products, float32 accumulation: within
2e-2 relative L2 per layer), training under the same initial weights and
minibatch order, and the ensemble mean and spread."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu

X_MEAN = np.array([90.0, 0.01, 1.5e-4, 1.5e-4, 1750.0, 1750.0, 1750.0])
X_STD = np.array([35.0, 0.004, 7e-5, 7e-5, 700.0, 700.0, 700.0])
Y_MEAN = np.array([20000.0, 0.01, 5000.0])
Y_STD = np.array([10000.0, 0.01, 3000.0])


def _data(n, seed):
    u = W.uniform_array(seed, n * 7).reshape(n, 7)
    x = X_MEAN + X_STD * (2 * u - 1) * 1.7
    y = np.zeros((n, 4))
    z = (x - X_MEAN) / X_STD
    y[:, 0] = Y_MEAN[0] + Y_STD[0] * np.tanh(z[:, 0] - 0.5 * z[:, 1] * z[:, 4])
    y[:, 1] = Y_MEAN[1] + Y_STD[1] * np.sin(z[:, 2] + z[:, 3])
    y[:, 2] = Y_MEAN[2] + Y_STD[2] * (0.3 * z[:, 5] - 0.2 * z[:, 6] ** 2)
    y[:, 3] = (z[:, 0] + z[:, 6] > 0.2).astype(float)
    return x.astype(np.float32).astype(np.float64), y.astype(np.float32).astype(np.float64)


def _params(seed):
    p = W.mlp_init(seed)
    p["b1"] = W.uniform_array(seed + 100, 128, -0.2, 0.2)
    p["b2"] = W.uniform_array(seed + 101, 128, -0.2, 0.2)
    p["b3"] = W.uniform_array(seed + 102, 4, -0.2, 0.2)
    return p


def _targets_n(y):
    t = y.copy()
    t[:, :3] = (y[:, :3] - Y_MEAN) / Y_STD
    return t


def _net(L, members=4):
    net = L.MLP(members)
    net.set_scaling(X_MEAN, X_STD, Y_MEAN, Y_STD)
    ps = [_params(10 + k) for k in range(members)]
    for k, p in enumerate(ps):
        net.set_weights(k, p)
    return net, ps


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n", [1, 37, 300])
def test_forward_matches_oracle(gpu_lib, n):
    net, ps = _net(gpu_lib)
    x, _ = _data(n, 3)
    mean, spread, mem = net.predict(x, members=True)
    mem = mem.cpu().numpy().astype(np.float64)
    outs = []
    for k, p in enumerate(ps):
        o, _ = M.forward(p, M.normalise(x, X_MEAN, X_STD))
        ref = np.concatenate([o[:, :3] * Y_STD + Y_MEAN, 1 / (1 + np.exp(-o[:, 3:]))], axis=1)
        outs.append(ref)
        for c in range(3):
            # bfloat16 operands: about 3 significant digits per product
            err = np.abs(mem[k, :, c] - ref[:, c]).max() / Y_STD[c]
            assert err < 3e-2, (k, c, err)
        assert np.abs(mem[k, :, 3] - ref[:, 3]).max() < 1e-2
    m_np, s_np = mem.mean(axis=0), mem.std(axis=0)
    assert np.allclose(mean.cpu().numpy(), m_np, rtol=1e-5, atol=1e-6 * np.abs(m_np).max())
    assert np.allclose(spread.cpu().numpy(), s_np, rtol=1e-3, atol=1e-5 * np.abs(m_np).max())
    net.close()


@pytest.mark.parametrize("n", [16, 200, 1024])
def test_gradients_match_oracle_per_layer(gpu_lib, n):
    net, ps = _net(gpu_lib)
    x, y = _data(n, 4)
    loss, grads = net.gradients(x, y)
    xn, t = M.normalise(x, X_MEAN, X_STD), _targets_n(y)
    for k, p in enumerate(ps):
        l_ref, g_ref = M.gradients(p, xn, t)
        assert loss[k] == pytest.approx(l_ref, rel=1e-2)
        for name in M.NAMES:
            e = rel(grads[k][name], g_ref[name])
            assert e < 2e-2, (k, name, e)
    net.close()


def test_training_follows_oracle(gpu_lib):
    n, steps, batch, lr = 2048, 300, 128, 2e-3
    net, ps = _net(gpu_lib, members=2)
    x, y = _data(n, 5)
    idx = np.stack([W.minibatch_order(40 + k, n, steps, batch) for k in range(2)])
    loss_gpu = net.train(x, y, idx, lr).cpu().numpy().astype(np.float64)
    xn, t = M.normalise(x, X_MEAN, X_STD), _targets_n(y)
    for k in range(2):
        p = {name: v.copy() for name, v in ps[k].items()}
        loss_ref = np.array(M.train(p, xn, t, idx[k], lr))
        assert loss_gpu[k, -30:].mean() < 0.5 * loss_gpu[k, :10].mean()
        # same trajectory within bfloat16 noise: the smoothed curves agree
        for a, b in [(0, 10), (100, 130), (270, 300)]:
            assert loss_gpu[k, a:b].mean() == pytest.approx(loss_ref[a:b].mean(), rel=0.1), (k, a)
        w = net.get_weights(k)
        o_gpu = net.predict(x[:256], members=True)[2].cpu().numpy()[k]
        o_ref, _ = M.forward(p, xn[:256])
        assert rel(o_gpu[:, :3], o_ref[:, :3] * Y_STD + Y_MEAN) < 0.1
        assert np.isfinite(pack := np.concatenate([w[nm].ravel() for nm in M.NAMES])).all()
    net.close()


def test_seeded_create_draws_the_published_generator(gpu_lib):
    """ij_mlp_create_seeded: member k holds, as float, the uniform draws of
    SplitMix64 started at seed + 1000 k (workloads.mlp_init, written from
    the generator's definition in Python), bit for bit."""
    seed = 4242
    net = gpu_lib.MLP(3, seed=seed)
    for k in range(3):
        got = net.get_weights(k)
        ref = W.mlp_init(seed + 1000 * k)
        for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
            assert np.array_equal(np.asarray(got[name]), ref[name].astype(np.float32).astype(np.float64)), (k, name)
    net.close()
