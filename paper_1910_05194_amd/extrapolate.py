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


def loss_weights(n_in: int, n_out: int) -> np.ndarray:
    """Jackson factors g_n of an (n_in + n_out)-moment expansion for n = n_in .. n_in+n_out-1."""
    M = n_in + n_out
    n = np.arange(n_in, M, dtype=np.float64)
    q = math.pi / (M + 1)
    return ((M - n + 1) * np.cos(q * n) + np.sin(q * n) / math.tan(q)) / (M + 1)


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
    w = torch.tensor(loss_weights(n_in, n_out), dtype=torch.float32, device=device)
    loss = torch.zeros(1, dtype=torch.float64, device=device)
    if standardise:
        ti = torch.tensor(tr, device=device)
        net.fit_scaling(X[ti].contiguous(), T[ti].contiguous())
    steps_per_epoch = max(1, len(tr) // batch)
    total = epochs * steps_per_epoch
    hist = {"train": [], "val": []}
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
        yv = net.forward(X[vi].contiguous()).cpu().numpy().astype(np.float64)
        vloss = float(np.mean(((yv - mu[val, n_in:n_in + n_out]) * loss_weights(n_in, n_out)[None, :]) ** 2))
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


def accept(mu_full, e_min: float, e_max: float, energies, tol: float = 1e-3) -> List[bool]:
    """Acceptance checks of an extrapolated table: |mu_n| <= 1 and a non-negative Jackson DOS."""
    import torch
    ok = []
    en = torch.as_tensor(energies, dtype=torch.float64, device="cuda")
    for i in range(mu_full.shape[0]):
        row = mu_full[i]
        if not bool(torch.isfinite(row).all()) or float(row.abs().max()) > 1.0 + 1e-6:
            ok.append(False)
            continue
        rho = kpm.reconstruct_jackson(row.contiguous(), en, e_min, e_max)
        ok.append(float(rho.min()) >= -tol * float(rho.abs().max()))
    return ok


def dos_error(rho, rho_ref) -> float:
    """E_DOS = sum_k |rho - rho_ref| / sum_k |rho_ref| on a common energy grid."""
    rho = np.asarray(rho)
    rho_ref = np.asarray(rho_ref)
    return float(np.sum(np.abs(rho - rho_ref)) / np.sum(np.abs(rho_ref)))
