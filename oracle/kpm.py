"""Chebyshev moments of the DOS/LDOS and their Jackson-damped reconstruction (FP64).

Test infrastructure only (see the package docstring).

Paper passages followed:
* eqs. rescalingH / rescalingE: H~ = (H - de+)/de-, eps = (E - de+)/de-,
  de+- = (E_max +- E_min)/2.
* eq. e6: T_0 = 1, T_1 = X, T_{n+1} = 2 X T_n - T_{n-1}.
* Sec. 2(c), stochastic trace: Tr A / N ~ (1/R) sum_r <r|A|r>/N with white-noise
  |r>; here random phases xi = exp(2 pi i u).  Moments are taken directly as
  mu_n^(r) = <r|T_n(H~)|r>/N, one inner product per order (no doubling).
* eqs. e7, delta_function_cheb_expansion: the DOS per unit eps is
  (1/(pi sqrt(1-eps^2))) [mu_0 + 2 sum_{n>=1} mu_n T_n(eps)] when
  mu_n = Tr T_n(H~)/N.  (The factor printed in eqs. sss and e8 is the
  reciprocal of the one these two equations require; this oracle follows
  e4/e7/delta_function_cheb_expansion.)
* Sec. 2(a) KPM damping mu_n -> g_n mu_n with the Jackson kernel, which the
  paper cites (Weisse et al., Rev. Mod. Phys. 78, 275 (2006)) but does not
  print:  g_n = [(M-n+1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))]/(M+1);
  or with the Lorentz kernel the paper prints, sinh(lam (1 - n/M))/sinh(lam).
* eqs. green_function_cheb_expansion(b): the CPGF expansion of the resolvent,
  coefficients -2 sigma i exp(-sigma i n arccos(eps + i sigma eta)) /
  sqrt(1 - (eps + i sigma eta)^2) times T_n(H~)/(1 + delta_n0).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import lattice, rng


def rescale(H: sp.csr_matrix, e_min: float, e_max: float) -> sp.csr_matrix:
    de_p = 0.5 * (e_max + e_min)
    de_m = 0.5 * (e_max - e_min)
    N = H.shape[0]
    return ((H - de_p * sp.identity(N, dtype=H.dtype, format="csr")) / de_m).tocsr()


def random_phase_vectors(model: lattice.Model, R: int, vector_seed: int, lat_index: int = 0) -> np.ndarray:
    """xi_{r,o} = exp(2 pi i u), u from stream (PHASE, seed, lat_index, r), counter = global orbital."""
    out = np.empty((R, model.n_active), dtype=complex)
    for r in range(R):
        u = rng.uniform(rng.stream_key(rng.PHASE, vector_seed, lat_index, r), model.orb_index.astype(np.uint64))
        out[r] = np.exp(2j * np.pi * u)
    return out


def site_vectors(model: lattice.Model, orbitals) -> np.ndarray:
    """Basis vectors |i> for global orbital indices (LDOS start vectors)."""
    pos = {int(o): k for k, o in enumerate(model.orb_index)}
    out = np.zeros((len(orbitals), model.n_active), dtype=complex)
    for r, o in enumerate(orbitals):
        if int(o) not in pos:
            raise ValueError(f"orbital {o} is vacant or out of range")
        out[r, pos[int(o)]] = 1.0
    return out


def chebyshev_vectors(Ht: sp.csr_matrix, v0: np.ndarray, M: int):
    """Yield v_n = T_n(H~) v0 for n = 0..M-1 (eq. e6 applied to a vector)."""
    v_prev = v0
    yield v_prev
    if M == 1:
        return
    v = Ht @ v0
    yield v
    for _ in range(2, M):
        v_next = 2.0 * (Ht @ v) - v_prev
        v_prev, v = v, v_next
        yield v


def moments(Ht: sp.csr_matrix, vectors: np.ndarray, M: int, norm: float) -> np.ndarray:
    """Per-vector complex moments mu_n^(r) = <r|T_n(H~)|r>/norm, shape [R, M]."""
    R = vectors.shape[0]
    mu = np.empty((R, M), dtype=complex)
    for r in range(R):
        xi = vectors[r]
        for n, vn in enumerate(chebyshev_vectors(Ht, xi, M)):
            mu[r, n] = np.vdot(xi, vn) / norm
    return mu


def dos_moments(lat, par, lat_index: int = 0, model=None):
    """Moments for one lattice and DosParams-like ``par``.

    Returns (mu_per_vector [R, M] real, mu_mean [M], model).  The imaginary parts
    of the per-vector moments vanish for a Hermitian H and are checked.
    """
    if model is None:
        model = lattice.build(lat)
    Ht = rescale(model.H, lat.e_min, lat.e_max)
    if par.start == 1:
        vecs = site_vectors(model, par.sites)
        norm = 1.0
    else:
        vecs = random_phase_vectors(model, par.num_random, par.vector_seed, lat_index)
        norm = float(model.n_active)
    mu = moments(Ht, vecs, par.num_moments, norm)
    imag = np.max(np.abs(mu.imag)) if mu.size else 0.0
    if imag > 1e-10 * max(1, par.num_moments):
        raise AssertionError(f"moments have an imaginary part {imag}")
    mu_r = mu.real.copy()
    return mu_r, mu_r.mean(axis=0), model


def honeycomb_kspace_moments(L1: int, L2: int, t: float, e_min: float, e_max: float, M: int) -> np.ndarray:
    """Exact mu_n = Tr T_n(H~)/N of the clean nearest-neighbour honeycomb torus.

    The Bloch energies of the two-band model with the bonds A(n) - B(n + d),
    d in {(0,0), (1,-1), (0,-1)}, are +-|t| |1 + exp(i(k1 - k2)) + exp(-i k2)|,
    k_j = 2 pi m_j / L_j; the trace is the average of T_n over both bands
    (eq. e4 with the rescaling of Sec. 2(a)), evaluated by the Chebyshev
    recurrence on the k-grid.  A closed walk must take at least 2 min(L1, L2)
    hops to wind around the torus, so these moments equal those of any larger
    torus (and of the infinite lattice) for n < 2 min(L1, L2).
    """
    k1 = 2.0 * np.pi * np.arange(L1) / L1
    k2 = 2.0 * np.pi * np.arange(L2) / L2
    K1, K2 = np.meshgrid(k1, k2, indexing="ij")
    e = np.abs(t) * np.abs(1.0 + np.exp(1j * (K1 - K2)) + np.exp(-1j * K2)).ravel()
    d_plus, d_minus = (e_max + e_min) / 2.0, (e_max - e_min) / 2.0
    mu = np.zeros(M)
    for x in ((e - d_plus) / d_minus, (-e - d_plus) / d_minus):
        t_prev = np.ones_like(x)
        t_cur = x.copy()
        mu[0] += 1.0
        if M > 1:
            mu[1] += t_cur.mean()
        for n in range(2, M):
            t_prev, t_cur = t_cur, 2.0 * x * t_cur - t_prev
            mu[n] += t_cur.mean()
    return mu / 2.0


def jackson(M: int) -> np.ndarray:
    """Jackson kernel g_n, n = 0..M-1 (Weisse et al. 2006, the kernel the paper cites)."""
    n = np.arange(M, dtype=np.float64)
    q = np.pi / (M + 1)
    return ((M - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (M + 1)


def lorentz(M: int, lam: float) -> np.ndarray:
    """Lorentz kernel g_n = sinh(lam (1 - n/M)) / sinh(lam), n = 0..M-1 (Sec. 2(a),
    KPM damping); a delta peak becomes a Lorentzian of width ~ lam/M."""
    n = np.arange(M, dtype=np.float64)
    return np.sinh(lam * (1.0 - n / M)) / np.sinh(lam)


def cpgf_green(mu: np.ndarray, energies_ev: np.ndarray, e_min: float, e_max: float, eta_ev: float) -> np.ndarray:
    """(1/N) Tr 1/(E - H + i eta) per eV from moments mu_n = Tr T_n(H~)/N: the CPGF
    expansion of the retarded resolvent (eqs. green_function_cheb_expansion and
    green_function_cheb_expansionb, sigma = +), with eps = (E - de+)/de- and the
    broadening rescaled the same way, eta~ = eta / de-.  numpy's principal
    branches of arccos and sqrt are those of the printed coefficients for
    eta > 0 (the terms decay like exp(-n Im(-arccos z)))."""
    mu = np.asarray(mu, dtype=np.float64)
    d_plus, d_minus = (e_max + e_min) / 2.0, (e_max - e_min) / 2.0
    z = (np.asarray(energies_ev, dtype=np.float64) - d_plus) / d_minus + 1j * (eta_ev / d_minus)
    theta = np.arccos(z)
    root = np.sqrt(1.0 - z * z)
    out = np.zeros(z.shape, dtype=np.complex128)
    for n in range(mu.size):
        g_n = -2.0j * np.exp(-1j * n * theta) / root
        out += g_n * mu[n] / (2.0 if n == 0 else 1.0)
    return out / d_minus


def cpgf_dos(mu: np.ndarray, energies_ev: np.ndarray, e_min: float, e_max: float, eta_ev: float) -> np.ndarray:
    """rho(E) = -(1/pi) Im (1/N) Tr G^+(E), per eV per orbital (Lorentzian-broadened DOS)."""
    return -np.imag(cpgf_green(mu, energies_ev, e_min, e_max, eta_ev)) / np.pi


def chebyshev_t(n_max: int, x: np.ndarray) -> np.ndarray:
    """T_n(x) for n = 0..n_max-1 by the scalar recursion (eq. e3); shape [n_max, len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    T = np.empty((n_max, x.size))
    T[0] = 1.0
    if n_max > 1:
        T[1] = x
    for n in range(2, n_max):
        T[n] = 2.0 * x * T[n - 1] - T[n - 2]
    return T


def dos(mu: np.ndarray, energies_ev: np.ndarray, e_min: float, e_max: float, kernel=None) -> np.ndarray:
    """rho(E) per eV per orbital from moments mu_n = Tr T_n(H~)/N (eqs. e7, delta expansion).

    rho(E) = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(eps)] / (pi sqrt(1 - eps^2) de-).
    Energies outside the open interval (E_min, E_max) give 0.
    """
    M = mu.shape[-1]
    g = jackson(M) if kernel is None else kernel
    de_p = 0.5 * (e_max + e_min)
    de_m = 0.5 * (e_max - e_min)
    eps = (np.asarray(energies_ev, dtype=np.float64) - de_p) / de_m
    inside = np.abs(eps) < 1.0
    out = np.zeros(eps.shape)
    e_in = eps[inside]
    T = chebyshev_t(M, e_in)
    coef = g * mu
    coef = coef.copy()
    coef[1:] *= 2.0
    out[inside] = (coef @ T) / (np.pi * np.sqrt(1.0 - e_in ** 2) * de_m)
    return out
