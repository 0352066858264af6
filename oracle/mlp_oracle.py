"""FP64 reference of the surrogate network: a multilayer perceptron 7 -> 128
-> 128 -> 4 with GELU activations, used to predict the droplet outputs of the
lattice Boltzmann model (breakup step, drop velocity, drop volume and the
satellite flag of the Results section) from its seven inputs.

TEST INFRASTRUCTURE ONLY: the slow, plain reference the GPU training and
inference kernels are checked against.  Only the test-suite and the
benchmark's CPU leg use it; it shares no code with the GPU library.

Everything is float64 numpy.  Conventions (also those of the GPU library):
  parameters  W1 [128, 7], b1 [128], W2 [128, 128], b2 [128], W3 [4, 128], b3 [4]
  inputs      x normalised as (x - x_mean) / x_std before the first layer
  outputs     o[0:3] regression outputs in normalised units (target
              (y - y_mean) / y_std), o[3] the logit of the satellite flag
  loss        L = mean_s (1/3) sum_{k<3} (o_k - t_k)^2
                + mean_s [softplus(o_3) - y_3 o_3]
  GELU        g(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2  (exact form)
  Adam        Kingma & Ba (2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
              p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SIZES = (7, 128, 128, 4)
N_REG = 3
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def normalise(x, x_mean, x_std):
    return (np.asarray(x, np.float64) - x_mean) / x_std


def forward(p: dict, xn: np.ndarray):
    """xn: [S, 7] normalised inputs.  Returns the outputs [S, 4] and the
    intermediate values the backward pass needs."""
    z1 = xn @ p["W1"].T + p["b1"]
    a1 = gelu(z1)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = gelu(z2)
    o = a2 @ p["W3"].T + p["b3"]
    return o, (xn, z1, a1, z2, a2)


def loss(o: np.ndarray, t: np.ndarray) -> float:
    """t: [S, 4]; t[:, :3] normalised regression targets, t[:, 3] in {0, 1}."""
    s = o.shape[0]
    reg = np.sum((o[:, :N_REG] - t[:, :N_REG]) ** 2) / (N_REG * s)
    z = o[:, N_REG]
    softplus = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))
    bce = np.sum(softplus - t[:, N_REG] * z) / s
    return float(reg + bce)


def loss_grad(o: np.ndarray, t: np.ndarray) -> np.ndarray:
    s = o.shape[0]
    d = np.zeros_like(o)
    d[:, :N_REG] = 2.0 * (o[:, :N_REG] - t[:, :N_REG]) / (N_REG * s)
    d[:, N_REG] = (1.0 / (1.0 + np.exp(-o[:, N_REG])) - t[:, N_REG]) / s
    return d


def backward(p: dict, cache, do: np.ndarray) -> dict:
    xn, z1, a1, z2, a2 = cache
    g = {}
    g["W3"] = do.T @ a2
    g["b3"] = do.sum(axis=0)
    dz2 = (do @ p["W3"]) * gelu_grad(z2)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * gelu_grad(z1)
    g["W1"] = dz1.T @ xn
    g["b1"] = dz1.sum(axis=0)
    return g


def gradients(p: dict, xn: np.ndarray, t: np.ndarray):
    o, cache = forward(p, xn)
    return loss(o, t), backward(p, cache, loss_grad(o, t))


class Adam:
    def __init__(self, p: dict, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in p.items()}
        self.v = {k: np.zeros_like(v) for k, v in p.items()}
        self.t = 0

    def step(self, p: dict, g: dict) -> None:
        self.t += 1
        for k in p:
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * g[k]
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * g[k] * g[k]
            mh = self.m[k] / (1.0 - self.b1 ** self.t)
            vh = self.v[k] / (1.0 - self.b2 ** self.t)
            p[k] = p[k] - self.lr * mh / (np.sqrt(vh) + self.eps)


def train(p: dict, xn: np.ndarray, t: np.ndarray, order: np.ndarray, lr: float) -> list:
    """Adam over the minibatches order[step] (index arrays); returns the
    loss of each step before its update."""
    opt = Adam(p, lr)
    hist = []
    for idx in order:
        l, g = gradients(p, xn[idx], t[idx])
        hist.append(l)
        opt.step(p, g)
    return hist
