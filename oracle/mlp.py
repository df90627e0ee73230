"""FP64 CPU oracle of the surrogate network: MLP forward, backward, MSE, Adam.

TEST INFRASTRUCTURE ONLY (same rule as ``oracle.pwfs``): used by the tests to
check the GPU kernels' forward activations, gradients and optimiser steps.

The paper has no learned component; the network is the learned-surrogate
form of the workload: modal coefficients -> hidden layers with GELU ->
slope map.  Everything here is the plain definition:

  z_l = a_{l-1} W_l + b_l,   a_l = gelu(z_l) for hidden layers, y = z_L;
  gelu(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2   (exact, not tanh);
  loss = sum((y - t)^2) / (B * n_out);
  Adam with bias correction (Kingma & Ba, Algorithm 1).

Weights are [fan_in][fan_out] (``y = x W``), biases [fan_out].
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

_SQRT1_2 = 1.0 / math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(x: np.ndarray) -> np.ndarray:
    return 0.5 * x * (1.0 + erf(x * _SQRT1_2))


def gelu_grad(x: np.ndarray) -> np.ndarray:
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x * _SQRT1_2)) + x * _INV_SQRT_2PI * np.exp(-0.5 * x * x)


def forward(params, x):
    """params = [(W1, b1), ..., (WL, bL)].  Returns (y, cache)."""
    a = np.asarray(x, np.float64)
    cache = {"a": [a], "z": []}
    L = len(params)
    for l, (W, b) in enumerate(params):
        z = a @ np.asarray(W, np.float64) + np.asarray(b, np.float64)
        cache["z"].append(z)
        a = gelu(z) if l < L - 1 else z
        cache["a"].append(a)
    return a, cache


def mse(y, t):
    """Returns (loss, dL/dy)."""
    y = np.asarray(y, np.float64)
    t = np.asarray(t, np.float64)
    n = y.size
    d = y - t
    return float((d * d).sum() / n), 2.0 * d / n


def backward(params, cache, dy):
    """Gradients [(dW1, db1), ...] of the loss given dL/dy."""
    L = len(params)
    grads = [None] * L
    g = np.asarray(dy, np.float64)
    for l in range(L - 1, -1, -1):
        W = np.asarray(params[l][0], np.float64)
        if l < L - 1:
            g = g * gelu_grad(cache["z"][l])
        a_prev = cache["a"][l]
        grads[l] = (a_prev.T @ g, g.sum(axis=0))
        g = g @ W.T
    return grads


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One Adam update of parameter p at step t (t >= 1).  Returns (p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    if weight_decay:
        g = g + weight_decay * p
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

