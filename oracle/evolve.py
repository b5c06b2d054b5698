"""Wave-packet time evolution (FP64) -- TEST INFRASTRUCTURE ONLY.

Paper passages followed (Sec. 4, the spintronics example):
* The time-evolution operator U(dt) = exp(-i H dt / hbar) of a time-independent
  Hamiltonian and its expansion in Chebyshev polynomials of the rescaled
  Hamiltonian (Tal-Ezer and Kosloff): with H = de- H~ + de+ (eqs. rescalingH /
  rescalingE),
      U(dt) = exp(-i de+ dt / hbar) sum_n (2 - d_n0) c_n T_n(H~),
      c_n = (-i)^n J_n(de- dt / hbar).
  Reading used: the paper prints c_n = (-1)^n J_n.  The Jacobi-Anger expansion
  exp(-i x cos th) = J_0(x) + 2 sum_{n>=1} (-i)^n J_n(x) cos(n th) gives (-i)^n;
  with real coefficients the series is a real function of H~ and not unitary.
  The tests pin the series against the dense matrix exponential.
* The initial Gaussian wave packet
      psi(0, r) = exp(-|r - r_c|^2 / (2 sigma^2)) sum_j exp(i k_j . r) spinor_j,
  spinor_j a vector over the orbitals of one cell (sublattice-major, then
  spin).  Reading used: the printed exponent is garbled; sigma is read as the
  standard deviation of the envelope, r_c = c1 a1 + c2 a2 for the centre cell
  (c1, c2).  The packet is zero on vacant sites and normalised to 1.
* The observables: <sigma_{x,y,z}> (hbar/2 units), the mean position <x>, <y>
  and the mean square position <x^2>, <y^2> (nm, nm^2), each divided by the
  norm <psi|psi>, which is reported too.  Positions are r = n1 a1 + n2 a2 + tau_s
  for the cell indices 0 <= n1 < L1, 0 <= n2 < L2 (meaningful while the packet
  stays away from the periodic seam).
"""
from __future__ import annotations

import numpy as np
from scipy import special

from . import kpm, lattice

HBAR_EV_FS = 0.6582119569509067   # hbar in eV fs (exact in the 2019 SI: h / (2 pi e))


def orbital_positions(lat, model: lattice.Model) -> np.ndarray:
    """Cartesian position (nm) of every active orbital, [n_active, 2]."""
    a1, a2, tau, _ = lattice._geometry(lat.kind)
    per_cell = model.n_sub * model.n_spin
    o = model.orb_index
    cell = o // per_cell
    s = (o // model.n_spin) % model.n_sub
    n1, n2 = cell % lat.L1, cell // lat.L1
    return n1[:, None] * a1[None, :] + n2[:, None] * a2[None, :] + np.array(tau)[s]


def gaussian_wavepacket(lat, model: lattice.Model, k_vectors, spinors, width_nm: float, center_cells) -> np.ndarray:
    """The normalised Gaussian packet of the block comment, [n_active] complex.
    k_vectors [n_k, 2] in 1/nm, spinors [n_k, n_sub * n_spin] complex."""
    a1, a2, _, _ = lattice._geometry(lat.kind)
    r = orbital_positions(lat, model)
    rc = center_cells[0] * a1 + center_cells[1] * a2
    env = np.exp(-np.sum((r - rc) ** 2, axis=1) / (2.0 * width_nm ** 2))
    comp = model.orb_index % (model.n_sub * model.n_spin)
    psi = np.zeros(model.n_active, dtype=np.complex128)
    for k, sp in zip(np.atleast_2d(k_vectors), np.atleast_2d(spinors)):
        psi += np.exp(1j * (r @ np.asarray(k, dtype=np.float64))) * np.asarray(sp, dtype=np.complex128)[comp]
    psi *= env
    return psi / np.linalg.norm(psi)


def bessel_coefficients(M: int, x: float) -> np.ndarray:
    """(2 - d_n0) (-i)^n J_n(x) for n < M."""
    n = np.arange(M)
    return np.where(n == 0, 1.0, 2.0) * (-1j) ** n * special.jv(n, x)


def propagate(Ht, psi: np.ndarray, coef: np.ndarray, phase: complex) -> np.ndarray:
    """phase * sum_n coef_n T_n(H~) psi with the three-term recursion of eq. e6."""
    out = coef[0] * psi
    if coef.size == 1:
        return phase * out
    v_prev, v = psi, Ht @ psi
    out = out + coef[1] * v
    for n in range(2, coef.size):
        v_prev, v = v, 2.0 * (Ht @ v) - v_prev
        out = out + coef[n] * v
    return phase * out


def step_operator(lat, model: lattice.Model, dt_fs: float, M: int):
    """(H~, coefficients, global phase) of one time step dt (fs) with M terms."""
    d_plus, d_minus = (lat.e_max + lat.e_min) / 2.0, (lat.e_max - lat.e_min) / 2.0
    Ht = kpm.rescale(model.H, lat.e_min, lat.e_max)
    coef = bessel_coefficients(M, d_minus * dt_fs / HBAR_EV_FS)
    return Ht, coef, np.exp(-1j * d_plus * dt_fs / HBAR_EV_FS)


def observables(lat, model: lattice.Model, psi: np.ndarray) -> np.ndarray:
    """[norm, <x>, <y>, <x^2>, <y^2>, <sx>, <sy>, <sz>] of one state (spinless lattices:
    zero spin).  The spin pairs are found through the global orbital index."""
    r = orbital_positions(lat, model)
    p = np.abs(psi) ** 2
    norm = float(np.sum(p))
    out = [norm] + [float(np.sum(f * p)) / norm for f in (r[:, 0], r[:, 1], r[:, 0] ** 2, r[:, 1] ** 2)]
    if model.n_spin == 2:
        full = np.zeros(model.site_active.size * 2, dtype=np.complex128)
        full[model.orb_index] = psi
        up, dn = full[0::2], full[1::2]
        z = np.sum(np.conj(up) * dn)
        out += [2.0 * z.real / norm, 2.0 * z.imag / norm, float(np.sum(np.abs(up) ** 2 - np.abs(dn) ** 2)) / norm]
    else:
        out += [0.0, 0.0, 0.0]
    return np.array(out)


def evolve(lat, model: lattice.Model, psi0: np.ndarray, dt_fs: float, M: int, n_points: int):
    """psi at t = (n_points - 1) dt and the observables at t_k = k dt, k < n_points
    ([n_points, 8])."""
    Ht, coef, phase = step_operator(lat, model, dt_fs, M)
    psi = np.asarray(psi0, dtype=np.complex128)
    obs = [observables(lat, model, psi)]
    for _ in range(1, n_points):
        psi = propagate(Ht, psi, coef, phase)
        obs.append(observables(lat, model, psi))
    return psi, np.array(obs)
