"""Pins for the oracle MLP: finite differences, GELU values, Adam's first step."""
import math

import numpy as np

from oracle import mlp


def test_gelu_values():
    assert mlp.gelu(np.array(0.0)) == 0.0
    # Phi(1) = 0.841344746068543 (standard normal CDF, tabulated value).
    assert abs(mlp.gelu(np.array(1.0)) - 0.841344746068543) < 1e-14
    assert abs(mlp.gelu(np.array(-1.0)) - (-1 + 0.841344746068543)) < 1e-14
    assert abs(mlp.gelu_grad(np.array(0.0)) - 0.5) < 1e-15
    x = np.linspace(-4, 4, 81)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8


def test_backward_matches_central_differences():
    sizes = [6, 9, 7, 5]
    params = mlp.init_params(sizes, seed=3)
    g = np.random.default_rng(1)
    for p in params[1::2]:
        p[:] = g.normal(scale=0.3, size=p.shape)
    X = g.normal(size=(4, sizes[0]))
    T = g.normal(size=(4, sizes[-1]))
    w = g.uniform(0.2, 1.0, size=sizes[-1])
    Y, cache = mlp.forward(params, X)
    grads = mlp.backward(params, cache, Y, T, w)
    h = 1e-6
    for p, gr in zip(params, grads):
        flat = p.reshape(-1)
        gflat = gr.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 11)):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(params, X)[0], T, w)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(params, X)[0], T, w)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[idx]) <= 1e-7 * max(1e-3, abs(fd)), (idx, fd, gflat[idx])


def test_adam_first_step_closed_form():
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -4.0, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    lr = 1e-2
    new_p, m1, v1 = mlp.adam_step(p, g, m, v, t=1, lr=lr)
    # After one step mhat = g and vhat = g^2, so the update is lr * g / (|g| + eps).
    assert np.allclose(new_p[0], p[0] - lr * g[0] / (np.abs(g[0]) + 1e-8), rtol=0, atol=1e-15)


def test_training_reduces_loss():
    sizes = [8, 16, 16, 6]
    params = mlp.init_params(sizes, seed=0)
    g = np.random.default_rng(2)
    X = g.uniform(-1, 1, size=(32, 8))
    T = np.tanh(X[:, :6] * 0.5) * 0.1
    w = mlp.loss_weights(8, 6) * 0 + 1.0
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    l0 = mlp.loss(mlp.forward(params, X)[0], T, w)
    for t in range(1, 201):
        Y, cache = mlp.forward(params, X)
        grads = mlp.backward(params, cache, Y, T, w)
        params, m, v = mlp.adam_step(params, grads, m, v, t, lr=3e-3)
    l1 = mlp.loss(mlp.forward(params, X)[0], T, w)
    assert l1 < 0.05 * l0
    assert math.isfinite(l1)
