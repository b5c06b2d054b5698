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


def test_fit_scaling_matches_standardised_oracle(K):
    """After fit_scaling the network maps x -> (x - mean)/sd, y' -> mean + sd y', and
    trains on standardised targets with weights w * sd (population statistics;
    a constant column gets sd 1)."""
    import torch
    net = K.MLP(48, 64, 40, seed=3)
    params = net.get_params()
    X, T, w = _data(50, 48, 40, seed=12)          # column 0 is constant (mu_0 = 1)
    X[:, 5] += 3.0
    T = (T * 7.0 + 0.2).astype(np.float32)
    xd, td, wd = (torch.tensor(a, device="cuda") for a in (X, T, w))
    net.fit_scaling(xd, td)
    X64, T64 = X.astype(np.float64), T.astype(np.float64)
    mx, sx = X64.mean(0), X64.std(0)
    mt, st = T64.mean(0), T64.std(0)
    assert sx[0] == 0.0
    sx[sx == 0.0] = 1.0
    p64 = [p.astype(np.float64) for p in params]
    Yn, cache = omlp.forward(p64, (X64 - mx) / sx)
    y = net.forward(xd).cpu().numpy()
    assert rel(y, mt + st * Yn) <= 1e-5
    Tn, wn = (T64 - mt) / st, w.astype(np.float64) * st
    grads, loss = net.gradients(xd, td, wd)
    L = omlp.loss(Yn, Tn, wn)
    assert abs(loss - L) <= 1e-5 * L
    for gg, GG in zip(grads, omlp.backward(p64, cache, Yn, Tn, wn)):
        assert rel(gg, GG) <= 1e-4
    net.close()


def test_acceptance_rules(K):
    from paper_1910_05194_amd import extrapolate as ex
    E = np.linspace(-0.99, 0.99, 256)
    good = np.zeros((1, 32))
    good[0, 0] = 1.0
    good[0, 2] = 0.2                               # smooth positive DOS
    assert ex.accept(good, -1.0, 1.0, E)[0]
    assert not ex.accept(good, -1.0, 1.0, E, overlap=[1.5], overlap_tol=1.0)[0]
    assert ex.accept(good, -1.0, 1.0, E, overlap=[0.5], overlap_tol=1.0)[0]
    nan = good.copy()
    nan[0, 7] = np.nan
    assert not ex.accept(nan, -1.0, 1.0, E)[0]
    big = good.copy()
    big[0, 3] = 1.5                                # |mu_n| <= 1 holds for any DOS
    assert not ex.accept(big, -1.0, 1.0, E)[0]
    neg = good.copy()
    neg[0, 2] = -1.0                               # rho ~ 1 - 2 g_2 T_2(x) < 0 near the band edges
    assert not ex.accept(neg, -1.0, 1.0, E)[0]


def test_learned_extrapolation_gains_over_truncation_and_falls_back(K):
    """A network trained on recursion moments of random disordered lattices beats
    plain truncation on held-out lattices; rejected tables come from the full
    recursion.

    Small version of the learned-extrapolation workload: 256^2-cell lattices
    (orders up to 256 do not wrap around the torus), 64 -> 192 moments, hidden
    width 256.  Training: 384 lattices, R = 8; evaluation: 8 held-out lattices,
    R = 32, DOS error E = sum|rho - rho_full| / sum|rho_full| on 512 midpoints.
    """
    from paper_1910_05194_amd import extrapolate as ex
    import workload as wl
    n_in, M, n_chk = 64, 256, 32
    train = [wl.mlp_training_lattice(i, L=256) for i in range(384)]
    mu = ex.generate_moments(train, M, 8, 11, batch=64)
    net = K.MLP(n_in, 256, M - n_in, seed=5)
    ex.train(net, mu, epochs=120, batch=64, lr=1e-3)
    evl = [wl.mlp_training_lattice(i, L=256, seed=777) for i in range(8)]
    full = ex.generate_moments(evl, M, 32, 3, batch=64)
    tables, ok, ov = ex.learned_moments(net, evl, 32, 3, n_check=n_chk, z_tol=np.inf, neg_tol=np.inf)
    assert all(ok)
    # Every computed order is kept; the network only fills the rest.
    assert np.array_equal(tables[:, :n_in + n_chk], full[:, :n_in + n_chk])
    e_tr, e_ml = [], []
    for i, L in enumerate(evl):
        E = wl.energy_grid(L.e_min, L.e_max, 512)
        rf = K.reconstruct_jackson(full[i], E, L.e_min, L.e_max)
        e_tr.append(ex.dos_error(K.reconstruct_jackson(full[i, :n_in + n_chk], E, L.e_min, L.e_max), rf))
        e_ml.append(ex.dos_error(K.reconstruct_jackson(tables[i], E, L.e_min, L.e_max), rf))
    gain = np.mean(e_tr) / np.mean(e_ml)
    print(f"E_trunc({n_in + n_chk}) {np.mean(e_tr):.4f}  E_mlp {np.mean(e_ml):.4f}  gain {gain:.2f}  overlap {np.round(ov, 3)}")
    assert gain > 1.2
    # Rejecting everything hands every lattice to the full recursion (same vectors).
    fb, ok0, _ = ex.learned_moments(net, evl, 32, 3, n_check=n_chk, z_tol=0.0)
    assert not any(ok0)
    assert np.array_equal(fb, full)
    net.close()


def test_kernel_factors_match_oracle(K):
    """kpm_kernel_factors against the oracle's Jackson and Lorentz kernels:
    whole expansions and slices (the learned path's loss weights are the slice
    n_in .. M-1 of a 2048-moment Jackson kernel), host and device outputs."""
    import torch
    for M in (1, 7, 256, 2048):
        assert np.max(np.abs(K.kernel_factors(M) - okpm.jackson(M))) <= 1e-14
        assert np.max(np.abs(K.kernel_factors(M, kernel=1, lam=4.0) - okpm.lorentz(M, 4.0))) <= 1e-14
    g = K.kernel_factors(2048, n0=256, count=1792)
    assert np.max(np.abs(g - okpm.jackson(2048)[256:])) <= 1e-14
    gd = K.kernel_factors(2048, n0=256, count=1792, out_device="cuda").cpu().numpy()
    assert np.array_equal(gd, g)
    assert np.array_equal(omlp.loss_weights(256, 1792), okpm.jackson(2048)[256:])
    for bad in (dict(n0=2040, count=16), dict(n0=-1, count=4), dict(kernel=1, lam=0.0), dict(kernel=3)):
        with pytest.raises(K.KPMError):
            K.kernel_factors(2048, **bad)


def test_rel_error_and_eval_loss_match_oracle(K):
    """kpm_mlp_rel_error and kpm_mlp_noise_z (the overlap measures of the
    acceptance check) and kpm_mlp_eval_loss (the validation loss) against the same quantities
    computed from the FP64 oracle's forward pass on the same weights: the
    FP32 forward's relative error is <= 1e-5 (see above), so both agree to
    ~1e-5 relative; with the fitted standardisation as well."""
    import torch
    net = K.MLP(256, 1024, 1792, seed=5)
    params = net.get_params()
    X, T, w = _data(48, 256, 1792, seed=9)
    xd, td, wd = (torch.tensor(a, device="cuda") for a in (X, T, w))
    p64 = [p.astype(np.float64) for p in params]
    Y, _ = omlp.forward(p64, X.astype(np.float64))
    n_cmp = 64
    ref = (Y[:, :n_cmp] + np.random.default_rng(2).normal(size=(48, n_cmp)) * 1e-2)
    wc = w[:n_cmp].astype(np.float64)
    want = np.sqrt(np.sum((wc * (Y[:, :n_cmp] - ref)) ** 2, 1)) / np.sqrt(np.sum((wc * ref) ** 2, 1))
    got = net.rel_error(xd, torch.tensor(ref, device="cuda"), wd[:n_cmp], bf16=False).cpu().numpy()
    print("rel_error max rel dev", np.max(np.abs(got - want) / want))
    assert np.max(np.abs(got - want) / want) <= 1e-3
    # kpm_mlp_noise_z: the same deviation over the per-row noise times ||w||.
    noise = np.random.default_rng(3).uniform(1e-4, 1e-2, 48)
    want_z = np.sqrt(np.sum((wc * (Y[:, :n_cmp] - ref)) ** 2, 1)) / (noise * np.sqrt(np.sum(wc ** 2)))
    got_z = net.noise_z(xd, torch.tensor(ref, device="cuda"), torch.tensor(noise, device="cuda"), wd[:n_cmp],
                        bf16=False).cpu().numpy()
    print("noise_z max rel dev", np.max(np.abs(got_z - want_z) / want_z))
    assert np.max(np.abs(got_z - want_z) / want_z) <= 1e-3
    L = omlp.loss(Y, T.astype(np.float64), w.astype(np.float64))
    got_l = float(net.eval_loss(xd, td, wd).item())
    print("eval_loss", got_l, "oracle", L)
    assert abs(got_l - L) <= 1e-4 * L
    # With standardisation: eval_loss equals the loss of forward() in original units.
    net.fit_scaling(xd, td)
    y = net.forward(xd).cpu().numpy().astype(np.float64)
    L2 = omlp.loss(y, T.astype(np.float64), w.astype(np.float64))
    assert abs(float(net.eval_loss(xd, td, wd).item()) - L2) <= 1e-6 * L2
    net.close()
