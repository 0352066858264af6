"""Pins of the FP64 surrogate network reference (oracle/mlp_oracle.py):
analytic gradients against central finite differences, GELU against the
normal distribution function, the first Adam step against its closed form,
the logistic loss against its direct form, and a fit that must succeed."""
import math

import numpy as np
import pytest
from scipy.stats import norm

import workloads as W
from oracle import mlp_oracle as M


def _data(n=24, seed=5):
    x = W.uniform_array(seed, n * 7, -2.0, 2.0).reshape(n, 7)
    t = np.zeros((n, 4))
    t[:, :3] = W.uniform_array(seed + 1, n * 3, -1.0, 1.0).reshape(n, 3)
    t[:, 3] = (W.uniform_array(seed + 2, n) > 0.5).astype(float)
    return x, t


def test_splitmix_array_matches_scalar_generator():
    r = W.SplitMix64(1234)
    ref = [r.next_u64() for _ in range(10)]
    assert [int(v) for v in W.splitmix64_array(1234, 10)] == ref
    assert [int(v) for v in W.splitmix64_array(1234, 4, offset=6)] == ref[6:]


def test_gelu_is_z_times_normal_cdf():
    z = np.linspace(-6, 6, 241)
    assert np.allclose(M.gelu(z), z * norm.cdf(z), rtol=0, atol=1e-15)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(z), fd, rtol=0, atol=1e-9)


def test_logistic_loss_matches_direct_form():
    o = np.array([[0.1, -0.2, 0.3, 1.7], [0.0, 0.5, -1.0, -2.3]])
    t = np.array([[0.0, 0.0, 0.0, 1.0], [0.5, 0.5, -1.0, 0.0]])
    s = 1.0 / (1.0 + np.exp(-o[:, 3]))
    bce = -np.mean(t[:, 3] * np.log(s) + (1 - t[:, 3]) * np.log(1 - s))
    mse = np.mean(np.sum((o[:, :3] - t[:, :3]) ** 2, axis=1) / 3.0)
    assert M.loss(o, t) == pytest.approx(mse + bce, rel=1e-14)


def test_gradients_match_central_differences():
    x, t = _data()
    p = W.mlp_init(11)
    p["b1"] = W.uniform_array(3, 128, -0.1, 0.1)
    p["b2"] = W.uniform_array(4, 128, -0.1, 0.1)
    p["b3"] = W.uniform_array(6, 4, -0.1, 0.1)
    _, g = M.gradients(p, x, t)
    # central differences: truncation ~ h^2 (third derivative) and round-off ~ 1e-16 |L| / h
    # are both ~1e-11 at h = 1e-5, well under the 1e-6 relative bar
    h = 1e-5
    rng = np.random.default_rng(0)
    for name in M.NAMES:
        flat = p[name].reshape(-1)
        idx = np.arange(flat.size) if flat.size <= 1024 else rng.choice(flat.size, 256, replace=False)
        an = g[name].reshape(-1)[idx]
        fd = np.zeros(len(idx))
        for j, i in enumerate(idx):
            old = flat[i]
            flat[i] = old + h
            lp = M.loss(M.forward(p, x)[0], t)
            flat[i] = old - h
            lm = M.loss(M.forward(p, x)[0], t)
            flat[i] = old
            fd[j] = (lp - lm) / (2 * h)
        assert np.linalg.norm(an - fd) <= 1e-6 * np.linalg.norm(fd), name
        assert np.abs(an - fd).max() <= 1e-6 * np.abs(fd).max(), name


def test_first_adam_step_closed_form():
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    opt = M.Adam(p, lr=0.01)
    opt.step(p, g)
    # bias-corrected moments after one step are g and g^2
    expect = np.array([1.0, -2.0, 3.0]) - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], expect, rtol=0, atol=1e-15)


def test_training_fits_a_smooth_target():
    n = 512
    x = W.uniform_array(21, n * 7, -1.0, 1.0).reshape(n, 7)
    t = np.zeros((n, 4))
    t[:, 0] = np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2]
    t[:, 1] = x[:, 3] - x[:, 4] ** 2
    t[:, 2] = np.tanh(x[:, 5] + x[:, 6])
    t[:, 3] = (x[:, 0] + x[:, 1] > 0).astype(float)
    p = W.mlp_init(2)
    order = W.minibatch_order(8, n, 300, 64)
    hist = M.train(p, x, t, order, lr=3e-3)
    assert np.mean(hist[-20:]) < 0.25 * np.mean(hist[:5])
