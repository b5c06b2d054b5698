"""Conductivity (FP64): the rank-2 and rank-1 Gamma moments, the T = 0 longitudinal
(Kubo-Greenwood) conductivity, the Kubo-Bastin DC (Hall) and optical conductivities
at any temperature, the single-shot Fermi-surface conductivity, and their
eigenstate and k-space references.

Test infrastructure only (see the package docstring).  The sections below cite
the passages each part follows.

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
             n_idx=None, m_idx=None, with_bound: bool = False, progress=None):
    """Gamma_nm averaged over the given start vectors, for orders n in n_idx, m in m_idx.

    Returns complex [len(n_idx), len(m_idx)] in the eq. Gammanm normalisation
    (includes 1/(1+d_n0) (1+d_m0) and 1/(R N)).  With with_bound it also
    returns B_nm, the same normalisation of sum_r sum_k (|Re L_nk| + |Im L_nk|)
    (|Re R_mk| + |Im R_mk|): the sum of the magnitudes of the real products
    that make up Re and Im of Gamma_nm, the scale of a rounding-error bound
    for an approximate evaluation of the same inner products.  progress, if
    given, is called with a short message after each chain.
    """
    R, N = vectors.shape
    n_idx = np.arange(M) if n_idx is None else np.asarray(n_idx)
    m_idx = np.arange(M) if m_idx is None else np.asarray(m_idx)
    n_need = int(n_idx.max()) + 1
    m_need = int(m_idx.max()) + 1
    n_pos = {int(n): k for k, n in enumerate(n_idx)}
    m_pos = {int(m): k for k, m in enumerate(m_idx)}
    G = np.zeros((len(n_idx), len(m_idx)), dtype=complex)
    B = np.zeros((len(n_idx), len(m_idx)))
    for r in range(R):
        xi = vectors[r]
        Lstore = np.zeros((len(n_idx), N), dtype=complex)
        for n, Ln in enumerate(kpm.chebyshev_vectors(Ht, -(ha @ xi), n_need)):
            if n in n_pos:
                Lstore[n_pos[n]] = Ln
        if progress:
            progress(f"vector {r}: L chain done")
        Labs = np.abs(Lstore.real) + np.abs(Lstore.imag) if with_bound else None
        for m, Tm in enumerate(kpm.chebyshev_vectors(Ht, xi, m_need)):
            if m in m_pos:
                Rm = hb @ Tm
                for k in range(len(n_idx)):
                    G[k, m_pos[m]] += np.vdot(Lstore[k], Rm)
                if with_bound:
                    B[:, m_pos[m]] += Labs @ (np.abs(Rm.real) + np.abs(Rm.imag))
        if progress:
            progress(f"vector {r}: R chain done")
    dn = np.where(n_idx == 0, 2.0, 1.0)
    dm = np.where(m_idx == 0, 2.0, 1.0)
    norm = (R * N) * dn[:, None] * dm[None, :]
    if with_bound:
        return G / norm, B / norm
    return G / norm


def cond_gamma(lat, par, model=None, vectors=None, n_idx=None, m_idx=None, with_bound: bool = False,
               progress=None):
    """Gamma for a lattice and CondParams-like ``par`` with random-phase vectors
    (with_bound: (Gamma, B) as gamma_nm returns them, and the model)."""
    if model is None:
        model = lattice.build(lat)
    Ht = kpm.rescale(model.H, lat.e_min, lat.e_max)
    if vectors is None:
        vectors = kpm.random_phase_vectors(model, par.num_random, par.vector_seed, 0)
    ha = velocity(model, par.alpha)
    hb = velocity(model, par.beta)
    return gamma_nm(Ht, ha, hb, vectors, par.num_moments, n_idx, m_idx, with_bound, progress), model


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


# ---------------------------------------------------------------------------
# Kubo-Bastin (Fermi sea) conductivity, in particular the Hall conductivity.
#
# Paper passages followed:
# * eq. cond 1st order: first-order response with f(eps), the delta function
#   and the retarded/advanced resolvents.  Its static limit is the Kubo-Bastin
#   form (reading used, stated because the paper prints Lambda_nm(omega) with
#   a 1/omega prefactor and leaves omega -> 0 to KITE-tools):
#     sigma_ab(mu) = (i e^2 hbar / Omega) int d eps f(eps)
#                    Tr[ v_a delta(eps-H) v_b dG^R/d eps - v_a dG^A/d eps v_b delta(eps-H) ],
#   v = h~/(i hbar), h~ = [r, H]; f the Fermi function at chemical potential
#   mu and temperature T (f = theta(mu - eps) at T = 0).
# * eq. delta_function_cheb_expansion (Delta_n) and eqs.
#   green_function_cheb_expansion(b) (CPGF g_n^{R,A} at broadening eta) for
#   the two factors, and eq. Gammanm for the trace: in rescaled units
#     sigma_ab(mu)/(e^2/h) = Re{ -2 pi i (N/Omega)/de-^2 int_{-1}^{1} d eps f(eps)
#         sum_nm Gamma_nm [Delta_n(eps) g'^R_m(eps) - g'^A_n(eps) Delta_m(eps)] },
#   g' = d g / d eps.  This is the Lambda_nm contraction of eq.
#   conductivity_1st_order for a static field.
# * The energy integrals with f (here and in the optical conductivity) run in
#   theta, eps = cos theta, over Q equal cells of [0, pi]: the integrand apart
#   from f at each cell's midpoint, times the cell's occupation weight
#   int_cell f(cos theta) d theta.  At T = 0 that weight is the covered length
#   of the cell inside [theta_mu, pi]; at T > 0 it is a midpoint sum over
#   FERMI_SUB equal sub-cells (reading used: the paper gives no quadrature).
# ---------------------------------------------------------------------------

FERMI_SUB = 32


def fermi(eps_ev, mu_ev: float, kT_ev: float) -> np.ndarray:
    """Fermi-Dirac occupation 1/(1 + exp((eps - mu)/kT)) (kT in eV; kT = 0: the
    step theta(mu - eps), 1/2 at eps = mu)."""
    e = np.asarray(eps_ev, dtype=np.float64)
    if kT_ev == 0.0:
        return np.where(e < mu_ev, 1.0, np.where(e > mu_ev, 0.0, 0.5))
    x = (e - mu_ev) / kT_ev
    ex = np.exp(-np.abs(x))
    return np.where(x > 0, ex / (1.0 + ex), 1.0 / (1.0 + ex))


def occupation_weights(n_theta: int, mu_ev: float, kT_ev: float, e_min: float, e_max: float) -> np.ndarray:
    """int_cell f(cos theta) d theta for the n_theta equal theta-cells of [0, pi]
    (energies rescaled with the spectrum bounds), per the reading above."""
    d_plus, d_minus = (e_max + e_min) / 2.0, (e_max - e_min) / 2.0
    h = np.pi / n_theta
    th = (np.arange(n_theta) + 0.5) * h
    if kT_ev == 0.0:
        mut = (mu_ev - d_plus) / d_minus
        th_mu = 0.0 if mut >= 1.0 else (np.pi if mut <= -1.0 else float(np.arccos(mut)))
        return np.clip(th + h / 2.0 - np.maximum(th - h / 2.0, th_mu), 0.0, h)
    sub = th[:, None] - h / 2.0 + (np.arange(FERMI_SUB)[None, :] + 0.5) * (h / FERMI_SUB)
    return fermi(d_plus + d_minus * np.cos(sub), mu_ev, kT_ev).sum(axis=1) * (h / FERMI_SUB)

def _eigen(model):
    E, U = np.linalg.eigh(model.H.toarray())
    return E, U


def gamma_nm_exact(model: lattice.Model, e_min: float, e_max: float, M: int, alpha: int, beta: int) -> np.ndarray:
    """Gamma_nm (eq. Gammanm) as an exact trace, in the eigenbasis of H (dense):
        Tr[h~^a T_n(H~) h~^b T_m(H~)] = sum_ab (h~^a)_ab T_n(e_b) (h~^b)_ba T_m(e_a),
    divided by N (1+d_n0)(1+d_m0).  [M, M] complex."""
    E, U = _eigen(model)
    A = U.conj().T @ velocity(model, alpha).toarray() @ U
    B = U.conj().T @ velocity(model, beta).toarray() @ U
    d_plus, d_minus = (e_max + e_min) / 2.0, (e_max - e_min) / 2.0
    T = kpm.chebyshev_t(M, (E - d_plus) / d_minus).T          # [state, n]
    W = A * B.T                                                # W[a, b] = A_ab B_ba
    G = T.T @ W.T @ T                                          # [n, m] = sum_ab T_n(e_b) W_ab T_m(e_a)
    G = G / E.size
    G[0, :] /= 2.0
    G[:, 0] /= 2.0
    return G


def sigma_kubo_eigen(model: lattice.Model, mu_ev: float, alpha: int = 0, beta: int = 1, kT_ev: float = 0.0) -> float:
    """The Kubo-Bastin Fermi-sea conductivity at eta -> 0 in units of e^2/h,
    summed over eigenstates (the definition, evaluated directly):
        sigma_ab = Re{ (-2 pi i / Omega) sum_{a, b: E_a != E_b} f_a [P_ab - P_ba] / (E_a - E_b)^2 },
        P_ab = (h~^a)_ab (h~^b)_ba,  Omega = L1 L2 * cell area,  f = fermi(E, mu, kT).
    Pairs of occupied states cancel, so at T = 0 the sum runs over E_a < mu <= E_b.
    For a = x, b = y this is (4 pi/Omega) sum f_a Im[(h~^x)_ab (h~^y)_ba]/(E_a - E_b)^2
    (the diagonal terms of the Bastin integral cancel between its two parts; the
    Fermi-surface terms it adds at finite eta vanish with eta for a != b)."""
    E, U = _eigen(model)
    A = U.conj().T @ velocity(model, alpha).toarray() @ U
    B = U.conj().T @ velocity(model, beta).toarray() @ U
    f = (E < mu_ev).astype(np.float64) if kT_ev == 0.0 else fermi(E, mu_ev, kT_ev)
    P = A * B.T                                   # P_ab = A_ab B_ba
    dE = E[:, None] - E[None, :]
    off = np.abs(dE) > 1e-9 * max(1.0, float(np.max(np.abs(E))))
    den = np.where(off, dE, 1.0) ** 2
    n_cells = model.site_active.size // model.n_sub
    omega = n_cells * model.cell_area
    return float(np.real(-2j * np.pi / omega * np.sum(np.where(off, f[:, None] * (P - P.T) / den, 0.0))))


def sigma_bastin_eigen(model: lattice.Model, mu_ev: float, eta_ev: float, alpha: int = 0, beta: int = 1,
                       kT_ev: float = 0.0) -> float:
    """The Kubo-Bastin formula of the block comment above at finite broadening eta
    and temperature, evaluated on the eigenstates (what the Gamma/Lambda route
    tends to as M grows): the delta function picks E_b (first term) or E_a (second),
    and the derivative of the broadened resolvent is -1/(eps - E + i eta)^2, so
        sigma_ab = Re{ (-2 pi i / Omega) sum_ab P_ab (f_a - f_b) / (E_a - E_b - i eta)^2 },
    P_ab = (h~^a)_ab (h~^b)_ba, f = fermi(E, mu, kT).  eta -> 0 gives sigma_kubo_eigen."""
    E, U = _eigen(model)
    A = U.conj().T @ velocity(model, alpha).toarray() @ U
    B = U.conj().T @ velocity(model, beta).toarray() @ U
    f = fermi(E, mu_ev, kT_ev)
    P = A * B.T
    den = (E[:, None] - E[None, :] - 1j * eta_ev) ** 2
    n_cells = model.site_active.size // model.n_sub
    omega = n_cells * model.cell_area
    return float(np.real(-2j * np.pi / omega * np.sum(P * (f[:, None] - f[None, :]) / den)))


def cpgf_derivative(M: int, eps: np.ndarray, eta: float, sign: int) -> np.ndarray:
    """d g_n^{sign,eta}(eps) / d eps for n < M (eq. green_function_cheb_expansionb,
    rescaled units): with z = eps + i sign eta, theta = arccos z, s = sqrt(1 - z^2),
        g_n = -2 sign i exp(-sign i n theta) / s,
        g_n' = -2 sign i exp(-sign i n theta) [sign i n / s^2 + z / s^3]
    (d theta/dz = -1/s, d(1/s)/dz = z/s^3).  [len(eps), M]."""
    z = np.asarray(eps, dtype=np.float64) + 1j * sign * eta
    theta = np.arccos(z)
    s = np.sqrt(1.0 - z * z)
    n = np.arange(M, dtype=np.float64)
    e = np.exp(-sign * 1j * np.outer(theta, n))
    return -2.0 * sign * 1j * e * (sign * 1j * n[None, :] / (s * s)[:, None] + (z / s ** 3)[:, None])


def sigma_bastin(gamma: np.ndarray, energies_ev, e_min: float, e_max: float, eta_ev: float,
                 orbitals_per_nm2: float, n_theta: int, kT_ev: float = 0.0) -> np.ndarray:
    """Kubo-Bastin conductivity (e^2/h) at chemical potentials ``energies_ev`` and
    temperature kT_ev (eV) from a full [M, M] Gamma (formula in the block comment
    above).

    The energy integral is taken in theta (eps = cos theta, so Delta_n d eps =
    (2/pi) cos(n theta) d theta): the integrand at the midpoints of n_theta equal
    cells of [0, pi] times each cell's occupation weight."""
    gamma = np.asarray(gamma, dtype=np.complex128)
    M = gamma.shape[0]
    d_plus, d_minus = (e_max + e_min) / 2.0, (e_max - e_min) / 2.0
    eta = eta_ev / d_minus
    h = np.pi / n_theta
    th = (np.arange(n_theta) + 0.5) * h
    eps = np.cos(th)
    D = 2.0 * np.cos(np.outer(th, np.arange(M))) / np.pi       # Delta_n(eps) sin(theta), [q, n]
    gR = cpgf_derivative(M, eps, eta, +1)                      # [q, m]
    gA = cpgf_derivative(M, eps, eta, -1)                      # [q, n]
    F = np.sum((D @ gamma) * gR, axis=1) - np.sum((gA @ gamma) * D, axis=1)
    pref = -2j * np.pi * orbitals_per_nm2 / d_minus ** 2
    out = []
    for mu in np.atleast_1d(np.asarray(energies_ev, dtype=np.float64)):
        w = occupation_weights(n_theta, mu, kT_ev, e_min, e_max)
        out.append(float(np.real(pref * np.sum(F * w))))
    return np.array(out)


# ---------------------------------------------------------------------------
# Clean periodic lattices in k space (independent of the real-space builder's
# matrices; the same geometry and eq. HQAHE terms): Bloch Hamiltonian,
# velocity i dH/dk, the Kubo sum on the k grid of an L1 x L2 torus, and the
# Chern number of the occupied bands by the lattice link-variable method
# (Fukui, Hatsugai and Suzuki, J. Phys. Soc. Jpn. 74, 1674 (2005)).
# ---------------------------------------------------------------------------

def bloch(lat, k, periodic_gauge: bool = False):
    """(H(k), hx(k), hy(k)) of a clean honeycomb lattice (spinful or not): for a
    bond from j (cell n + d) to i (cell n), H(k)[i, j] += h_ij exp(-i k.d_ij) with
    d_ij = r_i - r_j, and h~^a(k) the same sum weighted by (d_ij)_a (= i dH/dk_a).
    periodic_gauge drops the sublattice offsets from the phase (H(k + G) = H(k))."""
    a1, a2, tau, bonds = lattice._geometry(lat.kind)
    n_spin = 2 if lat.kind == lattice.HONEYCOMB_SPIN else 1
    n = len(tau) * n_spin
    H = np.zeros((n, n), dtype=complex)
    hx = np.zeros((n, n), dtype=complex)
    hy = np.zeros((n, n), dtype=complex)
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    sy = np.array([[0, -1j], [1j, 0]], dtype=complex)
    for (si, sj, d1, d2) in bonds:
        cell = d1 * a1 + d2 * a2
        dvec = tau[si] - (cell + tau[sj])
        ph = np.exp(-1j * np.dot(k, -cell if periodic_gauge else dvec))
        dhat = dvec / np.linalg.norm(dvec)
        for s in range(n_spin):
            for s2 in range(n_spin):
                hop = lat.t if s == s2 else 0.0
                if n_spin == 2:
                    hop = hop + (2j / 3.0) * lat.rashba * (sx[s, s2] * dhat[1] - sy[s, s2] * dhat[0])
                i, j = si * n_spin + s, sj * n_spin + s2
                for (Mx, w) in ((H, 1.0), (hx, dvec[0]), (hy, dvec[1])):
                    Mx[i, j] += w * hop * ph
                    Mx[j, i] += np.conj(w * hop * ph) * (1.0 if Mx is H else -1.0)
    if n_spin == 2:
        H += np.diag([lat.exchange if (q % 2) == 0 else -lat.exchange for q in range(n)])
    return H, hx, hy


def _recip(lat):
    a1, a2, _, _ = lattice._geometry(lat.kind)
    A = np.column_stack([a1, a2])
    Bm = 2.0 * np.pi * np.linalg.inv(A).T
    return Bm[:, 0], Bm[:, 1], abs(a1[0] * a2[1] - a1[1] * a2[0])


def sigma_kubo_kgrid(lat, mu_ev: float, alpha: int = 0, beta: int = 1) -> float:
    """sigma_ab of sigma_kubo_eigen for the clean L1 x L2 torus, summed over its
    allowed wave vectors k = (m1 b1 / L1 + m2 b2 / L2) with the Bloch matrices."""
    b1, b2, area = _recip(lat)
    tot = 0.0 + 0.0j
    for m1 in range(lat.L1):
        for m2 in range(lat.L2):
            k = m1 * b1 / lat.L1 + m2 * b2 / lat.L2
            H, hx, hy = bloch(lat, k)
            E, U = np.linalg.eigh(H)
            A = U.conj().T @ (hx if alpha == 0 else hy) @ U
            B = U.conj().T @ (hx if beta == 0 else hy) @ U
            occ = np.nonzero(E < mu_ev)[0]
            emp = np.nonzero(E >= mu_ev)[0]
            P_ab = A[np.ix_(occ, emp)] * B[np.ix_(emp, occ)].T
            P_ba = A[np.ix_(emp, occ)].T * B[np.ix_(occ, emp)]
            tot += np.sum((P_ab - P_ba) / (E[occ][:, None] - E[emp][None, :]) ** 2)
    return float(np.real(-2j * np.pi / (lat.L1 * lat.L2 * area) * tot))


def chern_number(lat, n_occ: int, n_k: int) -> float:
    """Chern number of the n_occ lowest bands on an n_k x n_k grid by the link
    variables U_a(k) = det <u(k)|u(k + a)> (periodic gauge); the result is an
    integer whenever the grid resolves the Berry curvature."""
    b1, b2, _ = _recip(lat)
    vecs = np.empty((n_k, n_k), dtype=object)
    for i in range(n_k):
        for j in range(n_k):
            H, _, _ = bloch(lat, i * b1 / n_k + j * b2 / n_k, periodic_gauge=True)
            vecs[i, j] = np.linalg.eigh(H)[1][:, :n_occ]
    def link(u, v):
        d = np.linalg.det(u.conj().T @ v)
        return d / abs(d)
    total = 0.0
    for i in range(n_k):
        for j in range(n_k):
            ip, jp = (i + 1) % n_k, (j + 1) % n_k
            f = link(vecs[i, j], vecs[ip, j]) * link(vecs[ip, j], vecs[ip, jp]) / (
                link(vecs[i, jp], vecs[ip, jp]) * link(vecs[i, j], vecs[i, jp]))
            total += np.angle(f)
    return total / (2.0 * np.pi)


# ---------------------------------------------------------------------------
# Optical conductivity sigma_ab(omega) (eq. cond 1st order with the
# rank-1 and rank-2 Gamma of eq. Gammanm and the Lambda_n, Lambda_nm(omega)
# that follow it, combined as in eq. conductivity_1st_order):
#   sigma_ab(w)/(e^2/h) = (-2 pi i (N/Omega) / E_w) [ sum_n Gamma_n^{ab} L_n
#                          + (1/de-) sum_nm Gamma_nm^{a,b} L_nm(w) ],
#   L_n = int_{-1}^{1} d eps f(eps) Delta_n(eps),
#   L_nm(w) = int_{-1}^{1} d eps f(eps) [g^R_n(eps + w~) Delta_m(eps) + Delta_n(eps) g^A_m(eps - w~)],
# f the Fermi function at chemical potential mu and temperature T, E_w = hbar omega in eV, w~ = E_w/de-, g^{R,A} the CPGF coefficients at
# broadening eta (rescaled, hbar = 1), Gamma in eV nm^2 (rank 1) and eV^2 nm^2
# (rank 2).  The energy integrals use the theta quadrature of sigma_bastin.
# ---------------------------------------------------------------------------

def velocity2(model: lattice.Model, a: int, b: int) -> sp.csr_matrix:
    return model.h2[(min(a, b), max(a, b))]


def gamma_n(Ht: sp.csr_matrix, h2: sp.csr_matrix, vectors: np.ndarray, M: int) -> np.ndarray:
    """Rank-1 Gamma_n^{ab} averaged over the start vectors [R, N]:
    (1/(R N)) sum_r <T_n(H~) r | h~^{ab} r> / (1 + d_n0)."""
    R, N = vectors.shape
    G = np.zeros(M, dtype=complex)
    for r in range(R):
        u = h2 @ vectors[r]
        for n, vn in enumerate(kpm.chebyshev_vectors(Ht, vectors[r], M)):
            G[n] += np.vdot(vn, u)
    G /= R * N
    G[0] /= 2.0
    return G


def cond_gamma1(lat, par, model=None):
    """Gamma_n^{ab} for a lattice and CondParams-like ``par`` (random-phase vectors)."""
    if model is None:
        model = lattice.build(lat)
    Ht = kpm.rescale(model.H, lat.e_min, lat.e_max)
    vectors = kpm.random_phase_vectors(model, par.num_random, par.vector_seed, 0)
    return gamma_n(Ht, velocity2(model, par.alpha, par.beta), vectors, par.num_moments), model


def gamma_n_exact(model: lattice.Model, e_min: float, e_max: float, M: int, a: int, b: int) -> np.ndarray:
    """Rank-1 Gamma_n^{ab} as an exact trace: sum_a (h~^{ab})_aa T_n(e_a) / (N (1 + d_n0))."""
    E, U = _eigen(model)
    C = np.real(np.einsum("ia,ij,ja->a", U.conj(), velocity2(model, a, b).toarray(), U))
    d_plus, d_minus = (e_max + e_min) / 2.0, (e_max - e_min) / 2.0
    G = kpm.chebyshev_t(M, (E - d_plus) / d_minus) @ C / E.size
    G = G.astype(complex)
    G[0] /= 2.0
    return G


def cpgf_coefficients(M: int, z: np.ndarray, sign: int) -> np.ndarray:
    """g_n^{sign}(z) = -2 sign i exp(-sign i n arccos z) / sqrt(1 - z^2) for n < M (eq.
    green_function_cheb_expansionb with z = eps + i sign eta; principal branches).
    [len(z), M]."""
    z = np.asarray(z, dtype=np.complex128)
    theta = np.arccos(z)
    s = np.sqrt(1.0 - z * z)
    return -2.0 * sign * 1j * np.exp(-sign * 1j * np.outer(theta, np.arange(M))) / s[:, None]


def sigma_optical(gamma_nm: np.ndarray, gamma_n: np.ndarray, omegas_ev, mu_ev: float, e_min: float, e_max: float,
                  eta_ev: float, orbitals_per_nm2: float, n_theta: int, kT_ev: float = 0.0) -> np.ndarray:
    """Complex sigma_ab(omega) in e^2/h at chemical potential mu and temperature kT_ev
    (formula in the block comment above).  Quadrature in theta as in sigma_bastin."""
    gamma_nm = np.asarray(gamma_nm, dtype=np.complex128)
    gamma_n = np.asarray(gamma_n, dtype=np.complex128)
    M = gamma_nm.shape[0]
    d_plus, d_minus = (e_max + e_min) / 2.0, (e_max - e_min) / 2.0
    eta = eta_ev / d_minus
    h = np.pi / n_theta
    th = (np.arange(n_theta) + 0.5) * h
    eps = np.cos(th)
    D = 2.0 * np.cos(np.outer(th, np.arange(M))) / np.pi                   # [q, n]
    w = occupation_weights(n_theta, mu_ev, kT_ev, e_min, e_max)
    lam_n = D.T @ w                                                         # Lambda_n
    out = []
    for Ew in np.atleast_1d(np.asarray(omegas_ev, dtype=np.float64)):
        wt = Ew / d_minus
        gR = cpgf_coefficients(M, eps + wt + 1j * eta, +1)                 # g^R_m(eps + w~)
        gA = cpgf_coefficients(M, eps - wt - 1j * eta, -1)                 # g^A_m(eps - w~)
        # sum_nm G_nm [gR_n D_m + D_n gA_m] = sum_n D_n sum_m (gA_m G_nm + gR_m G_mn)
        F = np.sum(D * (gA @ gamma_nm.T + gR @ gamma_nm), axis=1)
        para = np.sum(F * w) / d_minus
        out.append(-2j * np.pi * orbitals_per_nm2 / Ew * (np.dot(gamma_n, lam_n) + para))
    return np.array(out)


def sigma_optical_eigen(model: lattice.Model, omegas_ev, mu_ev: float, eta_ev: float, a: int, b: int,
                        kT_ev: float = 0.0) -> np.ndarray:
    """The same sigma_ab(omega) evaluated on the eigenstates (the definition with the
    resolvents broadened by eta and the delta function exact):
      (-2 pi i/(Omega E_w)) [ sum_a f_a C_aa + sum_ab A_ab B_ba ( f_a/(E_a - E_b + E_w + i eta)
                                                             + f_b/(E_b - E_a - E_w - i eta) ) ],
    A, B, C = h~^a, h~^b, h~^{ab} in the eigenbasis, f = fermi(E, mu, kT) (theta(mu - E) at T = 0)."""
    E, U = _eigen(model)
    A = U.conj().T @ velocity(model, a).toarray() @ U
    B = U.conj().T @ velocity(model, b).toarray() @ U
    C = np.real(np.einsum("ia,ij,ja->a", U.conj(), velocity2(model, a, b).toarray(), U))
    f = (E < mu_ev).astype(np.float64) if kT_ev == 0.0 else fermi(E, mu_ev, kT_ev)
    P = A * B.T
    dE = E[:, None] - E[None, :]
    n_cells = model.site_active.size // model.n_sub
    omega = n_cells * model.cell_area
    out = []
    for Ew in np.atleast_1d(np.asarray(omegas_ev, dtype=np.float64)):
        para = np.sum(P * (f[:, None] / (dE + Ew + 1j * eta_ev) + f[None, :] / (-dE - Ew - 1j * eta_ev)))
        out.append(-2j * np.pi / (omega * Ew) * (np.dot(f, C) + para))
    return np.array(out)


def _bloch_many(lat, kpts: np.ndarray, a: int, b: int):
    """H(k), h~^a(k), h~^b(k), h~^{ab}(k) for many wave vectors [Nk, 2] of a clean
    honeycomb lattice (the bond sums of ``bloch`` and ``_bloch2``, vectorised over k)."""
    a1, a2, tau, bonds = lattice._geometry(lat.kind)
    n_spin = 2 if lat.kind == lattice.HONEYCOMB_SPIN else 1
    n = len(tau) * n_spin
    Nk = kpts.shape[0]
    H, Ha, Hb, H2 = (np.zeros((Nk, n, n), dtype=complex) for _ in range(4))
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    sy = np.array([[0, -1j], [1j, 0]], dtype=complex)
    for (si, sj, d1, d2) in bonds:
        dvec = tau[si] - (d1 * a1 + d2 * a2 + tau[sj])
        ph = np.exp(-1j * (kpts @ dvec))
        dhat = dvec / np.linalg.norm(dvec)
        for s in range(n_spin):
            for s2 in range(n_spin):
                hop = lat.t if s == s2 else 0.0
                if n_spin == 2:
                    hop = hop + (2j / 3.0) * lat.rashba * (sx[s, s2] * dhat[1] - sy[s, s2] * dhat[0])
                i, j = si * n_spin + s, sj * n_spin + s2
                for (Mx, w, sgn) in ((H, 1.0, 1.0), (Ha, dvec[a], -1.0), (Hb, dvec[b], -1.0),
                                     (H2, dvec[a] * dvec[b], 1.0)):
                    Mx[:, i, j] += w * hop * ph
                    Mx[:, j, i] += sgn * np.conj(w * hop * ph)
    if n_spin == 2:
        H += np.diag([lat.exchange if (q % 2) == 0 else -lat.exchange for q in range(n)])[None]
    return H, Ha, Hb, H2


def sigma_optical_kgrid(lat, omegas_ev, mu_ev: float, eta_ev: float, a: int, b: int) -> np.ndarray:
    """sigma_optical_eigen for the clean L1 x L2 torus from its Bloch states; the
    second-order operator in k space is sum d^a d^b h exp(-i k.d) (= -d^2 H/dk_a dk_b)."""
    b1, b2, area = _recip(lat)
    Ews = np.atleast_1d(np.asarray(omegas_ev, dtype=np.float64))
    tot = np.zeros(Ews.size, dtype=complex)
    m1, m2 = np.meshgrid(np.arange(lat.L1), np.arange(lat.L2), indexing="ij")
    kall = np.outer(m1.ravel() / lat.L1, b1) + np.outer(m2.ravel() / lat.L2, b2)
    for c0 in range(0, kall.shape[0], 20000):
        H, Ha, Hb, H2 = _bloch_many(lat, kall[c0:c0 + 20000], a, b)
        E, U = np.linalg.eigh(H)
        Uh = np.conj(np.swapaxes(U, 1, 2))
        A = Uh @ Ha @ U
        B = Uh @ Hb @ U
        C = np.real(np.einsum("kia,kij,kja->ka", U.conj(), H2, U))
        f = (E < mu_ev).astype(np.float64)
        P = A * np.swapaxes(B, 1, 2)
        dE = E[:, :, None] - E[:, None, :]
        for i, Ew in enumerate(Ews):
            tot[i] += np.sum(f * C) + np.sum(P * (f[:, :, None] / (dE + Ew + 1j * eta_ev)
                                                   + f[:, None, :] / (-dE - Ew - 1j * eta_ev)))
    return -2j * np.pi / (lat.L1 * lat.L2 * area * Ews) * tot


def _bloch2(lat, k, a: int, b: int):
    """k-space matrix of [r^a, [r^b, H]] for a clean honeycomb lattice (hopping terms only)."""
    a1, a2, tau, bonds = lattice._geometry(lat.kind)
    n_spin = 2 if lat.kind == lattice.HONEYCOMB_SPIN else 1
    n = len(tau) * n_spin
    Hm = np.zeros((n, n), dtype=complex)
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    sy = np.array([[0, -1j], [1j, 0]], dtype=complex)
    for (si, sj, d1, d2) in bonds:
        dvec = tau[si] - (d1 * a1 + d2 * a2 + tau[sj])
        ph = np.exp(-1j * np.dot(k, dvec))
        dhat = dvec / np.linalg.norm(dvec)
        w = dvec[a] * dvec[b]
        for s in range(n_spin):
            for s2 in range(n_spin):
                hop = lat.t if s == s2 else 0.0
                if n_spin == 2:
                    hop = hop + (2j / 3.0) * lat.rashba * (sx[s, s2] * dhat[1] - sy[s, s2] * dhat[0])
                i, j = si * n_spin + s, sj * n_spin + s2
                Hm[i, j] += w * hop * ph
                Hm[j, i] += np.conj(w * hop * ph)
    return Hm


# ---------------------------------------------------------------------------
# Single-shot Fermi-surface DC conductivity (Sec. 3(b) large-scale section:
# the 'single-shot' evaluation that avoids the double recursion of eq.
# Gammanm).  Reading used: the T = 0 Kubo-Greenwood conductivity with the
# Lorentzian-broadened delta function of the CPGF resolvent,
#   sigma_ab(E)/(e^2/h) = -2 pi^2 (1/Omega) Tr[h~^a d_eta(E-H) h~^b d_eta(E-H)],
#   d_eta(E-H) = -(1/pi) Im G^R(E + i eta) = (1/de-) sum_n c_n(E) T_n(H~)/(1+d_n0),
#   c_n(E) = -Im g_n(z~)/pi (eq. green_function_cheb_expansionb, z~ = eps + i eta~),
# with the stochastic trace: for each random vector r,
#   a = d_eta h~^a r,  b = h~^b d_eta r,  Tr[...] ~ -(1/R) sum_r <a|b>
# (h~^a is anti-Hermitian), i.e. two Chebyshev recursions per vector that
# serve every energy (O(K M N) work for K energies).
# ---------------------------------------------------------------------------

def singleshot_coefficients(M: int, energies_ev, e_min: float, e_max: float, eta_ev: float) -> np.ndarray:
    """c_n(E_k) / (de- (1 + d_n0)): the expansion of d_eta(E - H) in T_n(H~).  [K, M]."""
    d_plus, d_minus = (e_max + e_min) / 2.0, (e_max - e_min) / 2.0
    z = (np.atleast_1d(np.asarray(energies_ev, dtype=np.float64)) - d_plus) / d_minus + 1j * eta_ev / d_minus
    c = -np.imag(cpgf_coefficients(M, z, +1)) / np.pi / d_minus
    c[:, 0] /= 2.0
    return c


def sigma_singleshot(model: lattice.Model, e_min: float, e_max: float, energies_ev, eta_ev: float, M: int,
                     vectors: np.ndarray, a: int = 0, b: int = 0) -> np.ndarray:
    """Single-shot sigma_ab(E) in e^2/h with the given start vectors [R, N] (formula above)."""
    Ht = kpm.rescale(model.H, e_min, e_max)
    C = singleshot_coefficients(M, energies_ev, e_min, e_max, eta_ev)      # [K, M]
    K = C.shape[0]
    R = vectors.shape[0]
    ha, hb = velocity(model, a), velocity(model, b)
    acc = np.zeros(K)
    for r in range(R):
        xi = vectors[r]
        A = np.zeros((K, xi.size), dtype=complex)
        for n, vn in enumerate(kpm.chebyshev_vectors(Ht, ha @ xi, M)):
            A += C[:, n][:, None] * vn[None, :]
        Bd = np.zeros((K, xi.size), dtype=complex)
        for n, vn in enumerate(kpm.chebyshev_vectors(Ht, xi, M)):
            Bd += C[:, n][:, None] * vn[None, :]
        for k in range(K):
            acc[k] += np.real(np.vdot(A[k], hb @ Bd[k]))
    n_cells = model.site_active.size // model.n_sub
    return 2.0 * np.pi ** 2 / (n_cells * model.cell_area) * acc / R


def sigma_kubo_greenwood_eigen(model: lattice.Model, energies_ev, eta_ev: float, a: int = 0, b: int = 0) -> np.ndarray:
    """-2 pi^2 (1/Omega) sum_ab (h~^a)_ab d_eta(E - E_b) (h~^b)_ba d_eta(E - E_a) on the eigenstates,
    d_eta(x) = eta / (pi (x^2 + eta^2)): the definition the single-shot series converges to."""
    E, U = _eigen(model)
    A = U.conj().T @ velocity(model, a).toarray() @ U
    B = U.conj().T @ velocity(model, b).toarray() @ U
    P = A * B.T
    n_cells = model.site_active.size // model.n_sub
    out = []
    for e in np.atleast_1d(np.asarray(energies_ev, dtype=np.float64)):
        dl = eta_ev / (np.pi * ((e - E) ** 2 + eta_ev ** 2))
        out.append(float(np.real(-2.0 * np.pi ** 2 / (n_cells * model.cell_area) * np.sum(P * dl[None, :] * dl[:, None]))))
    return np.array(out)


def sigma_kubo_greenwood_kgrid(lat, energies_ev, eta_ev: float, a: int = 0, b: int = 0) -> np.ndarray:
    """sigma_kubo_greenwood_eigen for the clean L1 x L2 torus from its Bloch states."""
    b1, b2, area = _recip(lat)
    m1, m2 = np.meshgrid(np.arange(lat.L1), np.arange(lat.L2), indexing="ij")
    kall = np.outer(m1.ravel() / lat.L1, b1) + np.outer(m2.ravel() / lat.L2, b2)
    Es = np.atleast_1d(np.asarray(energies_ev, dtype=np.float64))
    tot = np.zeros(Es.size)
    for c0 in range(0, kall.shape[0], 20000):
        H, Ha, Hb, _ = _bloch_many(lat, kall[c0:c0 + 20000], a, b)
        E, U = np.linalg.eigh(H)
        Uh = np.conj(np.swapaxes(U, 1, 2))
        P = (Uh @ Ha @ U) * np.swapaxes(Uh @ Hb @ U, 1, 2)
        for i, e in enumerate(Es):
            dl = eta_ev / (np.pi * ((e - E) ** 2 + eta_ev ** 2))
            tot[i] += np.real(np.sum(P * dl[:, None, :] * dl[:, :, None]))
    return -2.0 * np.pi ** 2 / (lat.L1 * lat.L2 * area) * tot
