"""FP64 reference of the moment-extrapolation MLP (forward, backward, Adam).

Test infrastructure only (see the package docstring).

The network maps the first K_in Chebyshev moments of a DOS to the next K_out
moments:  Z1 = X W1 + b1, A1 = gelu(Z1), Z2 = A1 W2 + b2, A2 = gelu(Z2),
Y = A2 W3 + b3, with the exact GELU gelu(x) = x Phi(x), Phi the standard
normal CDF (computed with erf).  The loss is the kernel-weighted mean squared
error  L = (1/(B K_out)) sum_{b,j} (w_j (Y_bj - T_bj))^2  with w_j the Jackson
factor of moment K_in + j in an expansion of K_in + K_out moments, so that the
loss is the Chebyshev-weighted L2 error of the damped DOS tail.  The paper has
no learned component; this part is specified by the network shape alone, and
its numerics are pinned by finite differences in the tests.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from . import kpm


def gelu(x):
    return x * 0.5 * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    phi = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * phi


def loss_weights(k_in: int, k_out: int) -> np.ndarray:
    return kpm.jackson(k_in + k_out)[k_in:]


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    Z1 = X @ W1 + b1
    A1 = gelu(Z1)
    Z2 = A1 @ W2 + b2
    A2 = gelu(Z2)
    Y = A2 @ W3 + b3
    return Y, (X, Z1, A1, Z2, A2)


def loss(Y, T, w):
    B, K = Y.shape
    return float(np.sum((w[None, :] * (Y - T)) ** 2) / (B * K))


def backward(params, cache, Y, T, w):
    """Gradients of ``loss`` with respect to (W1, b1, W2, b2, W3, b3)."""
    W1, b1, W2, b2, W3, b3 = params
    X, Z1, A1, Z2, A2 = cache
    B, K = Y.shape
    dY = 2.0 * (w[None, :] ** 2) * (Y - T) / (B * K)
    dW3 = A2.T @ dY
    db3 = dY.sum(axis=0)
    dA2 = dY @ W3.T
    dZ2 = dA2 * gelu_grad(Z2)
    dW2 = A1.T @ dZ2
    db2 = dZ2.sum(axis=0)
    dA1 = dZ2 @ W2.T
    dZ1 = dA1 * gelu_grad(Z1)
    dW1 = X.T @ dZ1
    db1 = dZ1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015), returns new (params, m, v)."""
    new_p, new_m, new_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = beta1 * mm + (1.0 - beta1) * g
        vv = beta2 * vv + (1.0 - beta2) * g * g
        mhat = mm / (1.0 - beta1 ** t)
        vhat = vv / (1.0 - beta2 ** t)
        new_p.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        new_m.append(mm)
        new_v.append(vv)
    return new_p, new_m, new_v


def init_params(sizes, seed: int):
    """Deterministic He-uniform-like initialisation (numpy Generator; tests only)."""
    g = np.random.default_rng(seed)
    params = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        lim = math.sqrt(3.0 / fan_in)
        params.append(g.uniform(-lim, lim, size=(fan_in, fan_out)))
        params.append(np.zeros(fan_out))
    return params
