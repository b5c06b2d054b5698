"""GPU MLP kernels vs the FP64 oracle on identical weights and inputs.

Tolerances (full 256 -> 1024 -> 1024 -> 1792 network, batch 64):
* FP32 forward (FP32 MFMA): relative Frobenius error <= 1e-5 (FP32 rounding of
  sums of up to 1024 products).
* FP32 gradients: relative Frobenius error <= 1e-4 per parameter tensor.
* BF16-operand forward: relative Frobenius error <= 2e-2 (8-bit mantissas;
  errors ~ 2^-9 per operand, partially averaged over the sums).
"""
import numpy as np
import pytest

from oracle import kpm as okpm
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_05194_amd import kpm
    return kpm


def _data(B, n_in, n_out, seed=0):
    g = np.random.default_rng(seed)
    # Moment-like inputs: decaying amplitudes with random signs, mu_0 = 1.
    n = np.arange(n_in)
    X = g.normal(size=(B, n_in)) * np.exp(-n / 80.0)[None, :] * 0.3
    X[:, 0] = 1.0
    T = g.normal(size=(B, n_out)) * 0.01
    w = okpm.jackson(n_in + n_out)[n_in:]
    return X.astype(np.float32), T.astype(np.float32), w.astype(np.float32)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_forward_and_gradients_match_oracle(K):
    import torch
    net = K.MLP(256, 1024, 1792, seed=11)
    params = net.get_params()
    # Non-zero biases so that every term of the backward pass is exercised.
    g = np.random.default_rng(3)
    params = [p if p.ndim == 2 else (g.normal(size=p.shape) * 0.05).astype(np.float32) for p in params]
    net.set_params(params)
    X, T, w = _data(64, 256, 1792)
    xd, td, wd = (torch.tensor(a, device="cuda") for a in (X, T, w))
    y = net.forward(xd).cpu().numpy()
    p64 = [p.astype(np.float64) for p in params]
    Y, cache = omlp.forward(p64, X.astype(np.float64))
    e_f = rel(y, Y)
    print("forward fp32 rel err", e_f)
    assert e_f <= 1e-5
    grads, loss = net.gradients(xd, td, wd)
    L = omlp.loss(Y, T.astype(np.float64), w.astype(np.float64))
    G = omlp.backward(p64, cache, Y, T.astype(np.float64), w.astype(np.float64))
    assert abs(loss - L) <= 1e-5 * L
    for name, gg, GG in zip(["W1", "b1", "W2", "b2", "W3", "b3"], grads, G):
        e = rel(gg, GG)
        print(f"grad {name}: rel err {e:.2e}")
        assert e <= 1e-4
    yb = net.forward(xd, bf16=True).cpu().numpy()
    e_b = rel(yb, Y)
    print("forward bf16 rel err", e_b)
    assert e_b <= 2e-2
    net.close()


def test_ragged_shapes(K):
    """Layer sizes that are not multiples of the 64 x 64 tile."""
    import torch
    net = K.MLP(37, 70, 29, seed=2)
    params = net.get_params()
    X, T, w = _data(13, 37, 29, seed=5)
    y = net.forward(torch.tensor(X, device="cuda")).cpu().numpy()
    Y, cache = omlp.forward([p.astype(np.float64) for p in params], X.astype(np.float64))
    assert rel(y, Y) <= 1e-5
    grads, _ = net.gradients(*(torch.tensor(a, device="cuda") for a in (X, T, w)))
    G = omlp.backward([p.astype(np.float64) for p in params], cache, Y, T.astype(np.float64), w.astype(np.float64))
    for gg, GG in zip(grads, G):
        assert rel(gg, GG) <= 1e-4
    net.close()


def test_adam_step_matches_oracle_and_overfits(K):
    import torch
    net = K.MLP(64, 128, 96, seed=4)
    p0 = net.get_params()
    X, T, w = _data(32, 64, 96, seed=9)
    xd, td, wd = (torch.tensor(a, device="cuda") for a in (X, T, w))
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    net.train_step(xd, td, wd, lr=1e-3, loss_out=loss)
    p1 = net.get_params()
    p64 = [p.astype(np.float64) for p in p0]
    Y, cache = omlp.forward(p64, X.astype(np.float64))
    G = omlp.backward(p64, cache, Y, T.astype(np.float64), w.astype(np.float64))
    ref, _, _ = omlp.adam_step(p64, G, [np.zeros_like(p) for p in p64], [np.zeros_like(p) for p in p64], 1, 1e-3)
    for a, b, g, p in zip(p1, ref, G, p64):
        # The first Adam step moves each parameter by lr * g / (|g| + eps) ~ lr sign(g):
        # compare where the gradient is clearly non-zero (elsewhere FP32 and FP64 may
        # disagree on the sign of a vanishing gradient), and bound every step by lr.
        big = np.abs(g) > 1e-3 * np.max(np.abs(g))
        assert np.max(np.abs(a - b)[big]) <= 2e-5
        assert np.max(np.abs(a - p)) <= 1e-3 * (1 + 1e-3)
    l0 = float(loss.item())
    for _ in range(300):
        net.train_step(xd, td, wd, lr=1e-3, loss_out=loss)
    l1 = float(loss.item())
    print("overfit loss", l0, "->", l1)
    assert l1 < 0.01 * l0
    net.close()
