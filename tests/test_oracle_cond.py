"""Pins for the oracle's Gamma_nm tensor and sigma_xx reconstruction."""
import numpy as np
import pytest

import workload as wl
from oracle import cond, kpm, lattice


def _cheb_dense(Ht, n):
    lam, U = np.linalg.eigh(Ht)
    return (U * np.cos(n * np.arccos(np.clip(lam, -1, 1)))[None, :]) @ U.conj().T


def test_gamma00_clean_graphene_closed_form():
    """Gamma_00^xx = Tr[h h]/(4N) = -a^2 t^2 / 8 for clean NN graphene (exact trace)."""
    t = -2.7
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=6, L2=6, t=t)
    m = lattice.build(lat)
    # Basis vectors scaled by sqrt(N) so that <r|r> = N as for random phases: then
    # (1/(R N)) sum_r <r|A|r> is exactly Tr A / N.
    vecs = np.sqrt(m.n_active) * np.eye(m.n_active, dtype=complex)
    Ht = kpm.rescale(m.H, lat.e_min, lat.e_max)
    G = cond.gamma_nm(Ht, m.hx, m.hx, vecs, 2, n_idx=[0], m_idx=[0])
    assert abs(G[0, 0] - (-(wl.A_HONEYCOMB ** 2) * t ** 2 / 8)) < 1e-12
    Gy = cond.gamma_nm(Ht, m.hy, m.hy, vecs, 2, n_idx=[0], m_idx=[0])
    # y components of the three bond vectors: a_cc (vertical bond) and a_cc - a sqrt(3)/2
    # (twice, the oblique bonds; -a_cc/2 for an exactly regular hexagon).
    acc, a = wl.ACC_HONEYCOMB, wl.A_HONEYCOMB
    sum_dy2 = acc ** 2 + 2 * (acc - a * np.sqrt(3) / 2) ** 2
    assert abs(Gy[0, 0] - (-sum_dy2 * t ** 2 / 4)) < 1e-12


@pytest.mark.parametrize("lat", [
    wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=4, L2=3, t=-2.7, rashba=0.3, flux=1 / 4, anderson_w=0.7,
               disorder_seed=2),
    wl.Lattice(kind=wl.HONEYCOMB, L1=5, L2=4, t=-2.7, anderson_w=1.0, vacancy_p=0.1, disorder_seed=5),
])
@pytest.mark.parametrize("ab", [(0, 0), (0, 1), (1, 1)])
def test_gamma_per_vector_matches_dense_products(lat, ab):
    M, R = 12, 2
    par = wl.CondParams(num_moments=M, num_random=R, vector_seed=77, alpha=ab[0], beta=ab[1])
    G, m = cond.cond_gamma(lat, par)
    Ht = kpm.rescale(m.H, lat.e_min, lat.e_max).toarray()
    ha = cond.velocity(m, ab[0]).toarray()
    hb = cond.velocity(m, ab[1]).toarray()
    vecs = kpm.random_phase_vectors(m, R, 77)
    T = [_cheb_dense(Ht, n) for n in range(M)]
    N = m.n_active
    ref = np.zeros((M, M), dtype=complex)
    for r in range(R):
        v = vecs[r]
        for n in range(M):
            left = v.conj() @ ha @ T[n] @ hb
            for mm in range(M):
                ref[n, mm] += left @ (T[mm] @ v)
    d = np.where(np.arange(M) == 0, 2.0, 1.0)
    ref = ref / (R * N) / d[:, None] / d[None, :]
    assert np.max(np.abs(G - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def _exact_gamma(lat, M, alpha=0, beta=0):
    m = lattice.build(lat)
    vecs = np.sqrt(m.n_active) * np.eye(m.n_active, dtype=complex)
    Ht = kpm.rescale(m.H, lat.e_min, lat.e_max)
    G = cond.gamma_nm(Ht, cond.velocity(m, alpha), cond.velocity(m, beta), vecs, M)
    return G, m


def test_exact_gamma_is_hermitian_for_equal_directions():
    lat = wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=3, L2=3, t=-2.7, rashba=0.3, flux=1 / 3, anderson_w=1.0,
                     disorder_seed=4)
    G, _ = _exact_gamma(lat, 10)
    assert np.max(np.abs(G - G.conj().T)) < 1e-13


def test_sigma_from_gamma_matches_eigenbasis_kubo_greenwood():
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=4, L2=4, t=-2.7, anderson_w=1.5, disorder_seed=8)
    M = 32
    G, m = _exact_gamma(lat, M)
    E = np.linspace(-7.5, 7.5, 41)
    area = lat.L1 * lat.L2 * m.cell_area
    sig = cond.sigma_from_gamma(G, E, lat.e_min, lat.e_max, m.n_active, area)
    # Eigenbasis: -(pi e^2/(hbar Omega)) sum_ij |h'_ij|^2 dJ(E,l_i) dJ(E,l_j) with
    # dJ(E, l) = (1/de-) sum_n g_n Delta_n(eps) T_n(l)/(1+d_n0); 1/hbar = 2 pi/h.
    Ht = kpm.rescale(m.H, lat.e_min, lat.e_max).toarray()
    lam, U = np.linalg.eigh(Ht)
    hp = U.conj().T @ m.hx.toarray() @ U
    de_m = 0.5 * (lat.e_max - lat.e_min)
    g = kpm.jackson(M)
    n = np.arange(M)
    ref = []
    for e in E:
        eps = e / de_m
        Dn = 2 * np.cos(n * np.arccos(eps)) / (np.pi * np.sqrt(1 - eps ** 2))
        coef = g * Dn / np.where(n == 0, 2.0, 1.0)
        dJ = (np.cos(np.outer(n, np.arccos(lam))).T @ coef) / de_m
        tr = np.sum(dJ[:, None] * (hp * hp.T) * dJ[None, :])     # Tr[h dJ h dJ]
        ref.append(-(np.pi * 2 * np.pi / area) * tr.real)
    ref = np.array(ref)
    assert np.max(np.abs(sig - ref)) < 1e-10 * np.max(np.abs(ref))
    assert np.all(ref > -1e-12 * np.max(np.abs(ref)))


def test_sigma_xx_equals_sigma_yy_on_c3_symmetric_torus():
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=6, L2=6, t=-2.7)
    M = 24
    Gx, m = _exact_gamma(lat, M, 0, 0)
    Gy, _ = _exact_gamma(lat, M, 1, 1)
    E = np.linspace(-7, 7, 29)
    area = lat.L1 * lat.L2 * m.cell_area
    sx = cond.sigma_from_gamma(Gx, E, lat.e_min, lat.e_max, m.n_active, area)
    sy = cond.sigma_from_gamma(Gy, E, lat.e_min, lat.e_max, m.n_active, area)
    # The paper's a and a_cc differ from an exact regular hexagon by ~1e-5 relative.
    assert np.max(np.abs(sx - sy)) < 1e-4 * np.max(np.abs(sx))
