"""Rank-2 conductivity moments Gamma_nm and the T=0 longitudinal conductivity (FP64).

Test infrastructure only (see the package docstring).

Paper passages followed:
* eq. generalized velocity and the definition that follows it: the operator
  used in Gamma is h~^a = (i hbar) h^a = [r^a, H], which is anti-Hermitian.
* eq. Gammanm (rank 2, alpha, beta single directions):
      Gamma_nm = Tr[ h~^a T_n(H~)/(1+d_n0)  h~^b T_m(H~)/(1+d_m0) ] / N,
  with the trace taken stochastically (Sec. 2(c)):  <r| h~^a T_n h~^b T_m |r>
  = <L_n | R_m>  with  L_n = T_n(H~)(-h~^a r)  (h~^a is anti-Hermitian) and
  R_m = h~^b T_m(H~) r.  Here every <L_n|R_m> is a plain inner product.
* eq. delta_function_cheb_expansion with the first-order Kubo formula (eq. cond
  1st order) at T=0 and omega -> 0, keeping only the Fermi-surface term
  (Kubo-Greenwood).  Reading used (the paper prints the Kubo-Bastin form and
  leaves the T=0 longitudinal reduction to KITE-tools):
      sigma_xx(E) = -(pi e^2/(hbar Omega)) Tr[h~ d(E-H) h~ d(E-H)]
                  = -2 pi^2 (e^2/h) (N/Omega) (1/de-^2) sum_nm g_n g_m D_n(eps) D_m(eps) Re Gamma_nm,
  D_n(eps) = 2 T_n(eps)/(pi sqrt(1-eps^2)), Omega = L1 L2 * cell area.
  The absolute prefactor is parity unpinned (no worked value in the paper);
  the Gamma -> sigma algebra is pinned against an eigenbasis sum in the tests.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import kpm, lattice


def velocity(model: lattice.Model, direction: int) -> sp.csr_matrix:
    return model.hx if direction == 0 else model.hy


def gamma_nm(Ht: sp.csr_matrix, ha: sp.csr_matrix, hb: sp.csr_matrix, vectors: np.ndarray, M: int,
             n_idx=None, m_idx=None) -> np.ndarray:
    """Gamma_nm averaged over the given start vectors, for orders n in n_idx, m in m_idx.

    Returns complex [len(n_idx), len(m_idx)] in the eq. Gammanm normalisation
    (includes 1/(1+d_n0) (1+d_m0) and 1/(R N)).
    """
    R, N = vectors.shape
    n_idx = np.arange(M) if n_idx is None else np.asarray(n_idx)
    m_idx = np.arange(M) if m_idx is None else np.asarray(m_idx)
    n_need = int(n_idx.max()) + 1
    m_need = int(m_idx.max()) + 1
    n_pos = {int(n): k for k, n in enumerate(n_idx)}
    m_pos = {int(m): k for k, m in enumerate(m_idx)}
    G = np.zeros((len(n_idx), len(m_idx)), dtype=complex)
    for r in range(R):
        xi = vectors[r]
        Lstore = np.zeros((len(n_idx), N), dtype=complex)
        for n, Ln in enumerate(kpm.chebyshev_vectors(Ht, -(ha @ xi), n_need)):
            if n in n_pos:
                Lstore[n_pos[n]] = Ln
        for m, Tm in enumerate(kpm.chebyshev_vectors(Ht, xi, m_need)):
            if m in m_pos:
                Rm = hb @ Tm
                for k in range(len(n_idx)):
                    G[k, m_pos[m]] += np.vdot(Lstore[k], Rm)
    dn = np.where(n_idx == 0, 2.0, 1.0)
    dm = np.where(m_idx == 0, 2.0, 1.0)
    return G / (R * N) / dn[:, None] / dm[None, :]


def cond_gamma(lat, par, model=None, vectors=None, n_idx=None, m_idx=None):
    """Gamma for a lattice and CondParams-like ``par`` with random-phase vectors."""
    if model is None:
        model = lattice.build(lat)
    Ht = kpm.rescale(model.H, lat.e_min, lat.e_max)
    if vectors is None:
        vectors = kpm.random_phase_vectors(model, par.num_random, par.vector_seed, 0)
    ha = velocity(model, par.alpha)
    hb = velocity(model, par.beta)
    return gamma_nm(Ht, ha, hb, vectors, par.num_moments, n_idx, m_idx), model


def sigma_from_gamma(gamma: np.ndarray, energies_ev: np.ndarray, e_min: float, e_max: float,
                     n_orbitals: int, area_nm2: float, kernel=None) -> np.ndarray:
    """sigma_xx(E) in units of e^2/h from a full [M, M] Gamma (reading stated in the module docstring)."""
    M = gamma.shape[0]
    g = kpm.jackson(M) if kernel is None else kernel
    de_p = 0.5 * (e_max + e_min)
    de_m = 0.5 * (e_max - e_min)
    eps = (np.asarray(energies_ev, dtype=np.float64) - de_p) / de_m
    out = np.zeros(eps.shape)
    inside = np.abs(eps) < 1.0
    e_in = eps[inside]
    T = kpm.chebyshev_t(M, e_in)
    D = 2.0 * T / (np.pi * np.sqrt(1.0 - e_in ** 2))      # Delta_n(eps), [M, K]
    W = g[:, None] * D                                      # g_n Delta_n(eps)
    s = np.einsum("nk,nm,mk->k", W, gamma.real, W)
    out[inside] = -2.0 * np.pi ** 2 * (n_orbitals / area_nm2) / de_m ** 2 * s
    return out
