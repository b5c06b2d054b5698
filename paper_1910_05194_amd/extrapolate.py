"""Learned extrapolation of Chebyshev moments (orchestration of libkpm calls).

Every numerical step runs in libkpm: the training moments come from the
Chebyshev recursion (``Plan``), the network is trained by the library's MFMA
GEMM / GELU / loss / Adam kernels (``MLP.train_step``), inference is the BF16
MFMA forward, and DOS curves come from the Jackson reconstruction kernel.
This module only batches lattices, shuffles mini-batches and applies the
acceptance checks that decide when to fall back to the full recursion.

The network maps mu_0..mu_{n_in-1} of a DOS (rescaled units of its own
lattice) to mu_{n_in}..mu_{n_in+n_out-1}; the loss weights are the Jackson
factors of an (n_in + n_out)-moment expansion, so the loss is the
kernel-weighted L2 error of the predicted part of the damped DOS series.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

from . import kpm


def generate_moments(lattices: Sequence, num_moments: int, num_random: int, vector_seed: int,
                     precision: int = kpm.FP32, batch: int = 256, device="cuda") -> np.ndarray:
    """Mean moments [len(lattices), num_moments] from the recursion, batched per lattice kind."""
    import torch

    class _P:
        pass

    out = np.zeros((len(lattices), num_moments))
    by_kind = {}
    for i, L in enumerate(lattices):
        by_kind.setdefault(int(L.kind), []).append(i)
    for kind, idx in by_kind.items():
        for c0 in range(0, len(idx), batch):
            chunk = idx[c0:c0 + batch]
            par = _P()
            par.num_moments, par.num_random, par.vector_seed = num_moments, num_random, vector_seed
            par.precision, par.start, par.sites = precision, kpm.START_RANDOM_PHASE, None
            plan = kpm.Plan([lattices[i] for i in chunk], par)
            mean = torch.zeros((len(chunk), num_moments), dtype=torch.float64, device=device)
            plan.run(None, mean)
            plan.close()
            out[chunk] = mean.cpu().numpy()
    return out


def loss_weights(n_in: int, n_out: int, device=None):
    """Jackson factors g_n of an (n_in + n_out)-moment expansion for n = n_in .. n_in+n_out-1
    (kpm_kernel_factors; numpy, or a float64 tensor on device)."""
    return kpm.kernel_factors(n_in + n_out, n0=n_in, count=n_out, kernel=0, out_device=device)


def train(net: "kpm.MLP", mu: np.ndarray, epochs: int, batch: int = 256, lr: float = 1e-3,
          val_frac: float = 0.1, seed: int = 0, device="cuda", log=None, standardise: bool = True) -> dict:
    """Adam with a cosine learning-rate schedule on moment tables mu [n, n_in + n_out].

    With standardise=True the network works on per-order standardised moments
    (statistics of the training split, fitted by the library), which keeps the
    tiny high-order targets from being swamped by the output layer's scale.
    """
    import torch
    n_in, n_out = net.n_in, net.n_out
    assert mu.shape[1] >= n_in + n_out
    g = np.random.default_rng(seed)
    perm = g.permutation(mu.shape[0])
    n_val = max(1, int(val_frac * mu.shape[0]))
    val, tr = perm[:n_val], perm[n_val:]
    X = torch.tensor(mu[:, :n_in], dtype=torch.float32, device=device)
    T = torch.tensor(mu[:, n_in:n_in + n_out], dtype=torch.float32, device=device)
    w = loss_weights(n_in, n_out, device=device).to(torch.float32)
    loss = torch.zeros(1, dtype=torch.float64, device=device)
    if standardise:
        ti = torch.tensor(tr, device=device)
        net.fit_scaling(X[ti].contiguous(), T[ti].contiguous())
    steps_per_epoch = max(1, len(tr) // batch)
    total = epochs * steps_per_epoch
    hist = {"train": [], "val": [], "val_idx": val}
    step = 0
    for ep in range(epochs):
        order = g.permutation(tr)
        acc = 0.0
        for s in range(steps_per_epoch):
            idx = torch.tensor(order[s * batch:(s + 1) * batch], device=device)
            lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * step / total))
            net.train_step(X[idx].contiguous(), T[idx].contiguous(), w, lr_t, loss_out=loss)
            acc += float(loss.item()) if s == steps_per_epoch - 1 else 0.0
            step += 1
        vi = torch.tensor(val, device=device)
        vloss = float(net.eval_loss(X[vi], T[vi], w).item())
        hist["train"].append(acc)
        hist["val"].append(vloss)
        if log:
            log(f"[mlp] epoch {ep + 1}/{epochs}: train loss {acc:.3e}, val loss {vloss:.3e}")
    return hist


def extrapolate(net: "kpm.MLP", mu_head, bf16: bool = True):
    """Full moment tables [n, n_in + n_out]: the given head followed by the network's prediction."""
    import torch
    x = torch.as_tensor(mu_head, dtype=torch.float32, device="cuda")[:, :net.n_in].contiguous()
    y = net.forward(x, bf16=bf16)
    return torch.cat([torch.as_tensor(mu_head, dtype=torch.float64, device="cuda")[:, :net.n_in],
                      y.to(torch.float64)], dim=1)


def overlap_error(net: "kpm.MLP", mu_head, n_check: int = 64, bf16: bool = True) -> np.ndarray:
    """Kernel-weighted relative error of the network on orders n_in .. n_in+n_check-1.

    mu_head [n, >= n_in + n_check] holds moments the recursion computed; the
    network sees only the first n_in and its prediction of the next n_check is
    compared with the computed ones:  ||g (mu_hat - mu)|| / ||g mu|| over that
    window, with g the Jackson factors of the full expansion.
    """
    import torch
    mu_head = np.asarray(mu_head, dtype=np.float64)
    n_in = net.n_in
    assert mu_head.shape[1] >= n_in + n_check and n_check <= net.n_out
    x = torch.as_tensor(mu_head[:, :n_in], dtype=torch.float32, device="cuda").contiguous()
    ref = torch.as_tensor(mu_head[:, n_in:n_in + n_check], dtype=torch.float64, device="cuda").contiguous()
    g = loss_weights(n_in, net.n_out, device="cuda")[:n_check].to(torch.float32)
    return net.rel_error(x, ref, g, bf16=bf16).cpu().numpy()


def stat_noise(lattices: Sequence, num_random: int) -> np.ndarray:
    """Upper bound 1/sqrt(N R) of the standard error of mean moments from R
    random-phase vectors on a lattice of N orbitals (the bound of
    kpm_mlp_noise_z; vacancies leave fewer active orbitals, N (1 - p), which
    raises it by 1/sqrt(1 - p))."""
    return np.array([1.0 / math.sqrt(L.L1 * L.L2 * L.n_orb_cell * num_random) for L in lattices])


def overlap_z(net: "kpm.MLP", mu_head, noise, n_check: int = 64, bf16: bool = True) -> np.ndarray:
    """Kernel-weighted RMS deviation of the network's prediction on orders
    n_in .. n_in+n_check-1 from the moments the recursion computed, in units of
    those moments' statistical error (``stat_noise``): about 1 when the
    prediction agrees with the recursion within its noise, larger when the
    network is off by more than the recursion can resolve."""
    import torch
    mu_head = np.asarray(mu_head, dtype=np.float64)
    n_in = net.n_in
    assert mu_head.shape[1] >= n_in + n_check and n_check <= net.n_out
    x = torch.as_tensor(mu_head[:, :n_in], dtype=torch.float32, device="cuda").contiguous()
    ref = torch.as_tensor(mu_head[:, n_in:n_in + n_check], dtype=torch.float64, device="cuda").contiguous()
    nz = torch.as_tensor(np.asarray(noise, dtype=np.float64), device="cuda").contiguous()
    g = loss_weights(n_in, net.n_out, device="cuda")[:n_check].to(torch.float32)
    return net.noise_z(x, ref, nz, g, bf16=bf16).cpu().numpy()


def fit_acceptance(net: "kpm.MLP", mu_val, n_check: int = 64, factor: float = 2.0) -> float:
    """Acceptance threshold on the overlap error: factor x its 99th percentile on held-out tables."""
    e = overlap_error(net, mu_val, n_check)
    return float(factor * np.percentile(e, 99))


def accept(mu_full, e_min: float, e_max: float, energies, overlap=None, overlap_tol: float = np.inf,
           neg_tol: float = 0.02) -> List[bool]:
    """Acceptance checks of extrapolated tables [n, M].

    A table passes when it is finite with |mu_n| <= 1, its Jackson DOS dips
    below zero by at most neg_tol of its maximum (the damped series of true
    moments is non-negative), and, if given, its overlap error (prediction
    against recursion moments just past the network's input) is at most
    overlap_tol.  Tables that fail go back to the full recursion.
    """
    import torch
    ok = []
    en = torch.as_tensor(energies, dtype=torch.float64, device="cuda")
    for i in range(mu_full.shape[0]):
        row = torch.as_tensor(mu_full[i], dtype=torch.float64, device="cuda")
        if not bool(torch.isfinite(row).all()) or float(row.abs().max()) > 1.0 + 1e-6:
            ok.append(False)
            continue
        if overlap is not None and not (float(overlap[i]) <= overlap_tol):
            ok.append(False)
            continue
        rho = kpm.reconstruct_jackson(row.contiguous(), en, e_min, e_max)
        ok.append(float(rho.min()) >= -neg_tol * float(rho.abs().max()))
    return ok


def splice(net: "kpm.MLP", mu_head, bf16: bool = True) -> np.ndarray:
    """Full tables [n, n_in + n_out]: the computed head (all of it) followed by the
    network's prediction for the orders past it."""
    import torch
    mu_head = np.asarray(mu_head, dtype=np.float64)
    n_in, M = net.n_in, net.n_in + net.n_out
    x = torch.as_tensor(mu_head[:, :n_in], dtype=torch.float32, device="cuda").contiguous()
    y = net.forward(x, bf16=bf16).to(torch.float64).cpu().numpy()
    out = np.concatenate([mu_head[:, :n_in], y], axis=1)
    h = min(mu_head.shape[1], M)
    out[:, :h] = mu_head[:, :h]
    return out


def learned_moments(net: "kpm.MLP", lattices: Sequence, num_random: int, vector_seed: int, n_check: int = 64,
                    z_tol: float = 3.0, neg_tol: float = 0.05, n_energies: int = 1024, batch: int = 64):
    """Moment tables [n, n_in + n_out] from the truncated recursion plus the network,
    with the full recursion as fallback.

    The recursion computes n_in + n_check moments per lattice; the network
    extends each table; a table is kept when it passes ``accept`` (the
    network's deviation from the n_check computed orders, ``overlap_z`` in
    units of their statistical error, at most z_tol; a Jackson DOS on
    n_energies midpoints that is non-negative within neg_tol; |mu_n| <= 1);
    the lattices that fail are recomputed by the full recursion.  The random
    vectors are keyed by a lattice's place in its batch, so a fallback for
    every lattice reproduces the full run exactly, while a partial one draws
    fresh vectors for the rejected lattices.  Returns (tables, accepted flags,
    overlap z).
    """
    M = net.n_in + net.n_out
    head = generate_moments(lattices, net.n_in + n_check, num_random, vector_seed, batch=batch)
    ov = overlap_z(net, head, stat_noise(lattices, num_random), n_check)
    out = splice(net, head)
    ok = []
    for i, L in enumerate(lattices):
        E = L.e_min + (np.arange(n_energies) + 0.5) * (L.e_max - L.e_min) / n_energies
        ok.append(accept(out[i:i + 1], L.e_min, L.e_max, E, overlap=ov[i:i + 1], overlap_tol=z_tol,
                         neg_tol=neg_tol)[0])
    bad = [i for i, a in enumerate(ok) if not a]
    if bad:
        out[bad] = generate_moments([lattices[i] for i in bad], M, num_random, vector_seed, batch=batch)
    return out, ok, ov


def dos_error(rho, rho_ref) -> float:
    """E_DOS = sum_k |rho - rho_ref| / sum_k |rho_ref| on a common energy grid."""
    rho = np.asarray(rho)
    rho_ref = np.asarray(rho_ref)
    return float(np.sum(np.abs(rho - rho_ref)) / np.sum(np.abs(rho_ref)))
