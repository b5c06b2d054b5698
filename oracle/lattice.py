"""Explicit sparse tight-binding Hamiltonians, built bond by bond (FP64, eV).

Test infrastructure only (see the package docstring).

Paper passages followed:
* Sec. 3(a): a periodic hopping is one value plus an integer cell offset; the
  oracle expands every such pattern into explicit matrix entries.
* Sec. 3(d) honeycomb listing: lattice vectors, sublattice positions and the
  three A-B hoppings with offsets (0,0), (1,-1), (0,-1).
* Sec. 4, eq. HQAHE: hopping t, Rashba term (2i/3) lambda_R (s x d_ij)_z with
  d_ij the unit vector from site j to site i, exchange Delta_ex s_z (+ on spin
  up, - on spin down), spin-independent disorder V.
* Sec. 4 (magnetic field): Peierls substitution on a periodic lattice; the
  flux per cell must be commensurate with the torus (flux * L1 integer).
  The gauge is the Landau gauge A = phi (0, s1) in fractional coordinates, so a
  hop from site j to site i picks up exp(2 pi i phi (s1_i + s1_j)/2 (s2_i - s2_j)),
  evaluated with the unwrapped image of the neighbour (no seam term).
* Sec. 3(a)/Sec. 4 structural disorder: a vacancy removes the site's orbitals
  and every bond touching them.
* eq. generalized velocity: h^a = [r^a, H] (in eV nm, i.e. (i hbar) times the
  velocity), evaluated with bond vectors so that it is well defined on a torus.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import rng

HONEYCOMB = 0
HONEYCOMB_SPIN = 1
SQUARE = 2

A_HC = 0.24595          # nm, honeycomb lattice constant
ACC_HC = 0.142          # nm, carbon-carbon distance used for the sublattice positions
A_SQ = 0.24595          # nm, square lattice constant


@dataclass
class Model:
    """A built model restricted to its active (non-vacant) orbitals."""
    H: sp.csr_matrix          # physical Hamiltonian (eV), active orbitals only
    hx: sp.csr_matrix         # [x, H] (eV nm), same index space
    hy: sp.csr_matrix         # [y, H] (eV nm)
    h2: dict                  # [a, [b, H]] (eV nm^2) for (a, b) in (0, 0), (0, 1), (1, 1)
    orb_index: np.ndarray     # global orbital index of each active orbital
    site_active: np.ndarray   # bool per site (cell*n_sub + s)
    onsite: np.ndarray        # V per site (eV), before removal
    n_sub: int
    n_spin: int
    cell_area: float          # nm^2

    @property
    def n_active(self) -> int:
        return int(self.orb_index.size)


def _geometry(kind):
    if kind in (HONEYCOMB, HONEYCOMB_SPIN):
        a1 = np.array([A_HC, 0.0])
        a2 = np.array([A_HC / 2.0, A_HC * np.sqrt(3.0) / 2.0])
        tau = [np.array([0.0, -ACC_HC / 2.0]), np.array([0.0, ACC_HC / 2.0])]
        # Bonds listed as (sub_i, sub_j, d1, d2): the hop from j at cell n+d to i at cell n.
        bonds = [(0, 1, 0, 0), (0, 1, 1, -1), (0, 1, 0, -1)]
    elif kind == SQUARE:
        a1 = np.array([A_SQ, 0.0])
        a2 = np.array([0.0, A_SQ])
        tau = [np.array([0.0, 0.0])]
        bonds = [(0, 0, 1, 0), (0, 0, 0, 1)]
    else:
        raise ValueError(f"unknown lattice kind {kind}")
    return a1, a2, tau, bonds


def _fractional(a1, a2, r):
    """Coordinates (s1, s2) of a Cartesian point r in the (a1, a2) basis."""
    B = np.column_stack([a1, a2])
    return np.linalg.solve(B, r)


def disorder_arrays(lat):
    """Per-site Anderson potential V (eV) and active mask, from the SplitMix64 streams.

    V_site = W (u - 1/2) with u from stream (ANDERSON, disorder_seed), counter = site;
    a site is removed iff u' < p with u' from stream (VACANCY, disorder_seed).
    Both spins of a site share V and its vacancy (eq. HQAHE disorder term).
    """
    n_sub = 2 if lat.kind in (HONEYCOMB, HONEYCOMB_SPIN) else 1
    n_sites = lat.L1 * lat.L2 * n_sub
    sites = np.arange(n_sites, dtype=np.uint64)
    if lat.anderson_w != 0.0:
        u = rng.uniform(rng.stream_key(rng.ANDERSON, lat.disorder_seed), sites)
        V = lat.anderson_w * (u - 0.5)
    else:
        V = np.zeros(n_sites)
    if lat.vacancy_p > 0.0:
        u = rng.uniform(rng.stream_key(rng.VACANCY, lat.disorder_seed), sites)
        active = ~(u < lat.vacancy_p)
    else:
        active = np.ones(n_sites, dtype=bool)
    return V, active


def build(lat) -> Model:
    """Assemble H, [x,H], [y,H] as explicit CSR matrices for lattice ``lat``.

    ``lat`` has the fields of ``workload.Lattice``.
    """
    kind = lat.kind
    L1, L2 = lat.L1, lat.L2
    if L1 < 2 or L2 < 2:
        raise ValueError("L1, L2 >= 2 required")
    a1, a2, tau, bonds = _geometry(kind)
    n_sub = len(tau)
    n_spin = 2 if kind == HONEYCOMB_SPIN else 1
    if lat.flux != 0.0:
        if kind == SQUARE:
            raise ValueError("flux on the square lattice is not supported")
        q = lat.flux * L1
        if abs(q - round(q)) > 1e-9:
            raise ValueError("flux * L1 must be an integer on a torus")
    if lat.rashba != 0.0 and kind != HONEYCOMB_SPIN:
        raise ValueError("Rashba coupling needs the spinful lattice")
    exchange = getattr(lat, "exchange", 0.0)
    if exchange != 0.0 and kind != HONEYCOMB_SPIN:
        raise ValueError("the exchange field needs the spinful lattice")
    N = L1 * L2 * n_sub * n_spin

    n1, n2 = np.meshgrid(np.arange(L1), np.arange(L2), indexing="xy")
    n1 = n1.ravel().astype(np.int64)
    n2 = n2.ravel().astype(np.int64)
    cell = n2 * L1 + n1

    rows, cols, vals, dxs, dys = [], [], [], [], []

    tau_frac = [_fractional(a1, a2, tv) for tv in tau]
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    sy = np.array([[0, -1j], [1j, 0]], dtype=complex)

    for (si, sj, d1, d2) in bonds:
        # site i at cell n (sublattice si); site j at the unwrapped image n + d.
        m1 = n1 + d1
        m2 = n2 + d2
        cell_j = (m2 % L2) * L1 + (m1 % L1)
        site_i = cell * n_sub + si
        site_j = cell_j * n_sub + sj
        r_i = np.outer(n1, a1) + np.outer(n2, a2) + tau[si]
        r_j = np.outer(m1, a1) + np.outer(m2, a2) + tau[sj]
        dvec = r_i - r_j                      # bond vector from j to i (nm)
        # Peierls phase of the hop j -> i (Landau gauge, fractional coordinates).
        if lat.flux != 0.0:
            s1_i = n1 + tau_frac[si][0]
            s2_i = n2 + tau_frac[si][1]
            s1_j = m1 + tau_frac[sj][0]
            s2_j = m2 + tau_frac[sj][1]
            theta = 2.0 * np.pi * lat.flux * 0.5 * (s1_i + s1_j) * (s2_i - s2_j)
            phase = np.exp(1j * theta)
        else:
            phase = np.ones(cell.size, dtype=complex)
        if n_spin == 1:
            hij = lat.t * phase
            pairs = [(site_i, site_j, hij)]
        else:
            dhat = dvec / np.linalg.norm(dvec, axis=1)[:, None]
            pairs = []
            for s in range(2):
                for s2 in range(2):
                    rash = (2j / 3.0) * lat.rashba * (sx[s, s2] * dhat[:, 1] - sy[s, s2] * dhat[:, 0])
                    hop = (lat.t if s == s2 else 0.0) + rash
                    pairs.append((site_i * 2 + s, site_j * 2 + s2, hop * phase))
        for (oi, oj, h) in pairs:
            # H_ij and its Hermitian partner H_ji.
            rows += [oi, oj]
            cols += [oj, oi]
            vals += [h, np.conj(h)]
            dxs += [dvec[:, 0], -dvec[:, 0]]
            dys += [dvec[:, 1], -dvec[:, 1]]

    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    dxs = np.concatenate(dxs)
    dys = np.concatenate(dys)

    V, site_active = disorder_arrays(lat)
    orb_site = np.arange(N) // n_spin
    diag = V[orb_site]
    if n_spin == 2:
        # s_z = +1 on spin up (orbital 2 site), -1 on spin down (2 site + 1).
        diag = diag + exchange * (1.0 - 2.0 * (np.arange(N) % 2))

    H = sp.coo_matrix((np.concatenate([vals, diag.astype(complex)]),
                       (np.concatenate([rows, np.arange(N)]), np.concatenate([cols, np.arange(N)]))),
                      shape=(N, N)).tocsr()
    hx = sp.coo_matrix((dxs * vals, (rows, cols)), shape=(N, N)).tocsr()
    hy = sp.coo_matrix((dys * vals, (rows, cols)), shape=(N, N)).tocsr()
    # Second-order operator [r^a, [r^b, H]]_ij = d^a_ij d^b_ij H_ij (eq. generalized velocity, n = 2).
    dd = {(0, 0): dxs * dxs, (0, 1): dxs * dys, (1, 1): dys * dys}
    h2 = {ab: sp.coo_matrix((w * vals, (rows, cols)), shape=(N, N)).tocsr() for ab, w in dd.items()}

    orb_active = site_active[orb_site]
    idx = np.nonzero(orb_active)[0]
    if idx.size < N:
        H = H[idx][:, idx].tocsr()
        hx = hx[idx][:, idx].tocsr()
        hy = hy[idx][:, idx].tocsr()
        h2 = {ab: m[idx][:, idx].tocsr() for ab, m in h2.items()}
    cell_area = abs(a1[0] * a2[1] - a1[1] * a2[0])
    return Model(H=H, hx=hx, hy=hy, h2=h2, orb_index=idx, site_active=site_active, onsite=V,
                 n_sub=n_sub, n_spin=n_spin, cell_area=cell_area)


def gershgorin(H: sp.csr_matrix) -> float:
    """max_i sum_j |H_ij|: a bound on the spectral radius."""
    return float(np.max(np.asarray(abs(H).sum(axis=1)).ravel()))
