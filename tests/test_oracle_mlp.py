"""Pins of the FP64 network oracle: GELU values, finite-difference gradients,
Adam's closed-form first step."""

import math

import numpy as np
import pytest

from oracle import mlp as M


def test_gelu_known_values():
    # x Phi(x): Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707 (normal table)
    x = np.array([0.0, 1.0, -1.0, 8.0, -8.0])
    g = M.gelu(x)
    assert g[0] == 0.0
    assert abs(g[1] - 0.8413447460685429) < 1e-15
    assert abs(g[2] + 0.15865525393145707) < 1e-15
    assert abs(g[3] - 8.0) < 1e-12 and abs(g[4]) < 1e-12


def test_gelu_grad_finite_difference():
    x = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.abs(fd - M.gelu_grad(x)).max() < 1e-8


def _params(sizes, seed):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((i, o)) / math.sqrt(i), rng.standard_normal(o) * 0.1)
            for i, o in zip(sizes[:-1], sizes[1:])]


def test_backward_matches_central_differences():
    sizes = [7, 11, 9, 5]
    P = _params(sizes, 1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((6, 7))
    t = rng.standard_normal((6, 5))
    y, cache = M.forward(P, x)
    _, dy = M.mse(y, t)
    G = M.backward(P, cache, dy)
    h = 1e-6

    def loss(PP):
        return M.mse(M.forward(PP, x)[0], t)[0]

    worst = 0.0
    for l in range(len(P)):
        for which in (0, 1):
            arr = P[l][which]
            it = np.nditer(arr, flags=["multi_index"])
            for _ in it:
                i = it.multi_index
                keep = arr[i]
                arr[i] = keep + h
                lp = loss(P)
                arr[i] = keep - h
                lm = loss(P)
                arr[i] = keep
                fd = (lp - lm) / (2 * h)
                worst = max(worst, abs(fd - G[l][which][i]) / max(1e-3, abs(fd)))
    assert worst < 1e-6


def test_input_gradient_by_finite_difference():
    """The chain through the first layer (dL/dx = g W1^T) also matches."""
    P = _params([4, 6, 3], 3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 4))
    t = rng.standard_normal((2, 3))
    y, cache = M.forward(P, x)
    _, dy = M.mse(y, t)
    # recompute dL/dx by hand from the oracle's pieces
    g = dy @ P[1][0].T * M.gelu_grad(cache["z"][0])
    dx = g @ P[0][0].T
    h = 1e-6
    for i in range(2):
        for j in range(4):
            xp = x.copy(); xp[i, j] += h
            xm = x.copy(); xm[i, j] -= h
            fd = (M.mse(M.forward(P, xp)[0], t)[0] - M.mse(M.forward(P, xm)[0], t)[0]) / (2 * h)
            assert abs(fd - dx[i, j]) < 1e-8


def test_mse_zero_and_scale():
    y = np.arange(6.0).reshape(2, 3)
    assert M.mse(y, y)[0] == 0.0
    l, d = M.mse(y + 1.0, y)
    assert l == 1.0 and np.allclose(d, 2.0 / 6)


@pytest.mark.parametrize("lr", [1e-3, 0.1])
def test_adam_first_step_closed_form(lr):
    """At t = 1 the bias corrections give m_hat = g, v_hat = g^2, so the step
    is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = M.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr)
    assert np.allclose(p1 - p, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_converges_to_lr_steps():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so each step moves by lr * sign(g) (to 1e-8 relative)."""
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -3.0])
    m = np.zeros(2); v = np.zeros(2)
    for t in range(1, 6):
        p_new, m, v = M.adam_step(p, g, m, v, t, 0.01)
        assert np.allclose(p_new - p, -0.01 * np.sign(g), rtol=1e-7)
        p = p_new
