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


def test_gamma_magnitude_sum_matches_dense_products():
    """The with_bound output B_nm: the same Gamma as without it, and B equal to
    the sum over vectors and orbitals of (|Re L_n| + |Im L_n|)(|Re R_m| + |Im R_m|)
    with L_n = T_n(H~)(-h^a r), R_m = h^b T_m(H~) r built from dense
    eigen-decomposition Chebyshev matrices; B dominates |Re Gamma| and |Im Gamma|."""
    lat = wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=4, L2=3, t=-2.7, rashba=0.3, flux=1 / 4, anderson_w=0.7,
                     vacancy_p=0.08, disorder_seed=2)
    M, R = 9, 2
    par = wl.CondParams(num_moments=M, num_random=R, vector_seed=31, alpha=0, beta=1)
    G0, m = cond.cond_gamma(lat, par)
    (G, B), _ = cond.cond_gamma(lat, par, model=m, with_bound=True)
    assert np.array_equal(G, G0)
    Ht = kpm.rescale(m.H, lat.e_min, lat.e_max).toarray()
    ha, hb = m.hx.toarray(), m.hy.toarray()
    vecs = kpm.random_phase_vectors(m, R, 31)
    T = [_cheb_dense(Ht, n) for n in range(M)]
    ref = np.zeros((M, M))
    for r in range(R):
        v = vecs[r]
        for n in range(M):
            Ln = T[n] @ (-(ha @ v))
            for mm in range(M):
                Rm = hb @ (T[mm] @ v)
                ref[n, mm] += np.sum((np.abs(Ln.real) + np.abs(Ln.imag)) * (np.abs(Rm.real) + np.abs(Rm.imag)))
    d = np.where(np.arange(M) == 0, 2.0, 1.0)
    ref = ref / (R * m.n_active) / d[:, None] / d[None, :]
    assert np.max(np.abs(B - ref)) <= 1e-12 * np.max(ref)
    assert np.all(B >= np.abs(G.real)) and np.all(B >= np.abs(G.imag))


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


# --- Kubo-Bastin / Hall conductivity (eq. cond 1st order, static limit) -----

T_HOP = -2.7


def _qahe(L, W=0.0, seed=0, exchange=0.4 * abs(T_HOP), rashba=0.3 * abs(T_HOP)):
    """The paper's QAHE model (eq. HQAHE, Fig. qahe): lambda_R = 0.3 t, Delta_ex = 0.4 t."""
    return wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=L, L2=L, t=T_HOP, rashba=rashba, exchange=exchange,
                      anderson_w=W, disorder_seed=seed, e_min=-10.0, e_max=10.0)


def test_qahe_real_space_spectrum_equals_bloch_bands():
    """The real-space builder (with the exchange term) and the k-space Bloch matrices
    are separate code: on a clean 6 x 6 torus the eigenvalues must coincide."""
    lat = _qahe(6)
    m = lattice.build(lat)
    e_real = np.sort(np.linalg.eigvalsh(m.H.toarray()))
    b1, b2, _ = cond._recip(lat)
    e_k = np.sort(np.concatenate([np.linalg.eigvalsh(cond.bloch(lat, i * b1 / 6 + j * b2 / 6)[0])
                                  for i in range(6) for j in range(6)]))
    assert np.max(np.abs(e_real - e_k)) < 1e-12


@pytest.mark.parametrize("L", [6, 9])
def test_kubo_real_space_equals_k_space(L):
    """sigma_xy from the dense real-space eigenstates = the same Kubo sum over the
    torus's Bloch states (independent matrices); L = 6, 9 give 0.614 and 1.633."""
    lat = _qahe(L)
    a = cond.sigma_kubo_eigen(lattice.build(lat), 0.0)
    b = cond.sigma_kubo_kgrid(lat, 0.0)
    assert abs(a - b) < 1e-10 * abs(b)
    assert abs(a - {6: 0.6135722646, 9: 1.6330226427}[L]) < 1e-8


def test_qahe_plateau_is_two_e2_over_h():
    """The clean QAHE insulator has Chern number 2 (paper: sigma_xy = 2 e^2/h in the
    gap).  The link-variable Chern number is an exact integer (+-2 by orientation),
    and the Kubo sum on a 120 x 120 torus equals -C to 1e-6 at the gap centre and
    off-centre inside the gap (E = +-0.3 eV; the gap is |E| < 0.62 eV)."""
    lat = _qahe(6)
    C = cond.chern_number(lat, 2, 24)
    assert abs(C - round(C)) < 1e-9 and abs(round(C)) == 2
    big = _qahe(120)
    for mu in (0.0, 0.3, -0.3):
        s = cond.sigma_kubo_kgrid(big, mu)
        assert abs(s - (-round(C))) < 1e-6, (mu, s)


def test_hall_vanishes_without_exchange_and_flips_with_it():
    """Rashba alone keeps time reversal: sigma_xy = 0 (checked at E = 50 meV, off the
    degenerate Dirac level of the gapless model).  Delta_ex -> -Delta_ex flips the
    sign of sigma_xy."""
    assert abs(cond.sigma_kubo_kgrid(_qahe(30, exchange=0.0), 0.05)) < 1e-12
    s_p = cond.sigma_kubo_kgrid(_qahe(30), 0.0)
    s_m = cond.sigma_kubo_kgrid(_qahe(30, exchange=-0.4 * abs(T_HOP)), 0.0)
    assert abs(s_p + s_m) < 1e-10 and abs(s_p) > 1.9


def test_gamma_exact_matches_dense_chebyshev_products():
    """gamma_nm_exact (eigenbasis sum) against Tr[h~x T_n h~y T_m]/N/((1+d_n0)(1+d_m0))
    with dense T_n(H~) matrices, on a disordered QAHE model with a vacancy."""
    lat = _qahe(3, W=1.5, seed=3)
    lat = lat.replace(vacancy_p=0.1, disorder_seed=5)
    m = lattice.build(lat)
    M = 9
    G = cond.gamma_nm_exact(m, lat.e_min, lat.e_max, M, 0, 1)
    Ht = kpm.rescale(m.H, lat.e_min, lat.e_max).toarray()
    hx, hy = m.hx.toarray(), m.hy.toarray()
    N = m.n_active
    for n in range(M):
        Tn = _cheb_dense(Ht, n)
        for mm in range(M):
            ref = np.trace(hx @ Tn @ hy @ _cheb_dense(Ht, mm)) / N / ((2 if n == 0 else 1) * (2 if mm == 0 else 1))
            assert abs(G[n, mm] - ref) < 1e-11 * max(1.0, abs(ref)), (n, mm)


def test_cpgf_derivative_matches_finite_differences():
    """cpgf_derivative against a central difference of the printed coefficients
    g_n = -2 s i exp(-s i n arccos z)/sqrt(1 - z^2), z = eps + i s eta."""
    eps = np.array([-0.83, -0.2, 0.0, 0.37, 0.9])
    eta, h, M = 0.01, 1e-6, 40
    for sign in (1, -1):
        def g(e):
            z = e + 1j * sign * eta
            n = np.arange(M)
            return -2 * sign * 1j * np.exp(-sign * 1j * np.outer(np.arccos(z), n)) / np.sqrt(1 - z * z)[:, None]
        fd = (g(eps + h) - g(eps - h)) / (2 * h)
        an = cond.cpgf_derivative(M, eps, eta, sign)
        assert np.max(np.abs(fd - an)) < 1e-6 * np.max(np.abs(an))


def test_bastin_spectral_converges_to_eigenstate_kubo():
    """The Gamma/Lambda route (sigma_bastin on the exact Gamma^xy, M = 4096,
    eta = 50 meV) reproduces the eigenstate Kubo sum of the same 6 x 6 torus
    (0.6136 e^2/h) to 1e-3; at M = 512 it is 2 % off (truncation)."""
    lat = _qahe(6)
    m = lattice.build(lat)
    exact = cond.sigma_kubo_eigen(m, 0.0)
    opn = m.n_active / (36 * m.cell_area)
    G = cond.gamma_nm_exact(m, lat.e_min, lat.e_max, 4096, 0, 1)
    s = cond.sigma_bastin(G, [0.0], lat.e_min, lat.e_max, 0.05, opn, 8192)[0]
    assert abs(s - exact) < 1e-3 * abs(exact), (s, exact)
    s512 = cond.sigma_bastin(G[:512, :512], [0.0], lat.e_min, lat.e_max, 0.05, opn, 1024)[0]
    assert 0.005 < abs(s512 - exact) / abs(exact) < 0.05


def test_bastin_both_directions_converge_on_a_disordered_model():
    """Disordered 4 x 4 QAHE model (W = 1 eV), Gamma^yx = (Gamma^xy)^T exactly.  At
    M = 4096, eta = 30 meV the spectral sigma_xy and sigma_yx match the eigenstate
    Kubo sums (+-0.8173 e^2/h at three Fermi energies) to 0.5 %; the symmetric part
    sigma_xy + sigma_yx, a truncation and broadening effect of the finite series
    (4 % at M = 256), is below 1e-3."""
    lat = _qahe(4, W=1.0, seed=9)
    m = lattice.build(lat)
    opn = m.n_active / (16 * m.cell_area)
    E = [-0.4, 0.0, 0.25]
    G = cond.gamma_nm_exact(m, lat.e_min, lat.e_max, 4096, 0, 1)
    assert np.max(np.abs(cond.gamma_nm_exact(m, lat.e_min, lat.e_max, 64, 1, 0) - G[:64, :64].T)) < 1e-15
    sxy = cond.sigma_bastin(G, E, lat.e_min, lat.e_max, 0.03, opn, 8192)
    syx = cond.sigma_bastin(G.T.copy(), E, lat.e_min, lat.e_max, 0.03, opn, 8192)
    exact = np.array([cond.sigma_kubo_eigen(m, e, 0, 1) for e in E])
    assert np.max(np.abs(sxy - exact) / np.abs(exact)) < 5e-3, (sxy, exact)
    assert np.max(np.abs(syx + exact) / np.abs(exact)) < 5e-3, (syx, exact)
    assert np.max(np.abs(sxy + syx)) < 1e-3


# --- Finite temperature: the Fermi function f of eq. cond 1st order and of Lambda_n, Lambda_nm ---

def test_fermi_function_and_cell_weights():
    """fermi: f(mu) = 1/2, f(mu + x) + f(mu - x) = 1, no overflow far from mu, the step at
    kT = 0.  occupation_weights: adaptive quadrature of f(cos theta) over each cell (kT > 0;
    within the sub-cell midpoint rule's error, < 2e-5 of a cell on these 0.12 eV cells),
    the covered lengths of [theta_mu, pi] at kT = 0, and kT -> 0 tending
    to those within a sub-cell."""
    from scipy import integrate
    x = np.array([0.0, 0.013, 0.2, 3.0])
    f_p, f_m = cond.fermi(0.3 + x, 0.3, 0.05), cond.fermi(0.3 - x, 0.3, 0.05)
    assert f_p[0] == 0.5 and np.max(np.abs(f_p + f_m - 1.0)) < 1e-15
    assert np.all(np.diff(f_p) < 0) and f_p[-1] < 1e-25
    with np.errstate(over="raise"):
        assert cond.fermi(np.array([-1e4, 1e4]), 0.0, 1e-3).tolist() == [1.0, 0.0]
    assert cond.fermi(np.array([-0.1, 0.0, 0.1]), 0.0, 0.0).tolist() == [1.0, 0.5, 0.0]
    Q, h = 256, np.pi / 256
    for mu, kT in ((0.3, 0.1), (-4.0, 0.5), (9.5, 0.2)):
        w = cond.occupation_weights(Q, mu, kT, -10.0, 10.0)
        ref = [integrate.quad(lambda th: cond.fermi(10.0 * np.cos(th), mu, kT), q * h, (q + 1) * h,
                              epsabs=1e-15, epsrel=1e-12)[0] for q in range(Q)]
        assert np.max(np.abs(w - ref)) < 2e-5 * h, (mu, kT)
    for mu in (-10.5, -3.3, 0.0, 7.1, 10.5):
        w0 = cond.occupation_weights(Q, mu, 0.0, -10.0, 10.0)
        # Covered length of each cell inside {theta : 10 cos(theta) < mu}, by brute force.
        fine = (np.arange(Q * 2000) + 0.5) * (h / 2000)
        ref = (10.0 * np.cos(fine) < mu).reshape(Q, 2000).sum(axis=1) * (h / 2000)
        assert np.max(np.abs(w0 - ref)) <= h / 2000, mu
        w1 = cond.occupation_weights(Q, mu, 1e-9, -10.0, 10.0)
        assert np.max(np.abs(w1 - w0)) <= h / cond.FERMI_SUB, mu


def test_bastin_finite_T_is_the_fermi_smearing_of_T0():
    """Integrating the f-weighted energy integral by parts gives
    sigma(mu, T) = int dE sigma(E, 0) (-df/dE), and this holds cell by cell for the
    theta quadrature (up to its sub-cell rule): the T > 0 path against Simpson's rule
    over the separate T = 0 path (disordered 4 x 4 QAHE model, M = 256).  Below a
    cell's width (kT = 20 meV) the sub-cell rule limits the agreement to 5e-4."""
    from scipy import integrate
    lat = _qahe(4, W=1.0, seed=9)
    m = lattice.build(lat)
    opn = m.n_active / (16 * m.cell_area)
    G = cond.gamma_nm_exact(m, lat.e_min, lat.e_max, 256, 0, 1)
    for kT, mu, tol in ((0.1, 0.3, 1e-6), (0.3, 2.0, 1e-4), (0.02, -1.1, 5e-4)):
        Eg = np.linspace(mu - 25 * kT, mu + 25 * kT, 20001)
        s0 = cond.sigma_bastin(G, Eg, lat.e_min, lat.e_max, 0.1, opn, 512)
        x = (Eg - mu) / kT
        smeared = integrate.simpson(s0 / (kT * (2.0 + np.exp(x) + np.exp(-x))), x=Eg)
        sT = cond.sigma_bastin(G, [mu], lat.e_min, lat.e_max, 0.1, opn, 512, kT_ev=kT)[0]
        assert abs(sT - smeared) < tol * abs(smeared), (kT, mu, sT, smeared)


def test_bastin_finite_T_converges_to_eigenstate_bastin():
    """The eigenstate Kubo-Bastin sum at finite eta tends to the eta -> 0 Kubo sum
    (1e-7, at T = 0 and kT = 0.1 eV); the Gamma/Lambda route (exact Gamma^xy, M = 4096,
    eta = 30 meV) matches it at kT = 0.05 and 0.2 eV to 1e-4 on the disordered 4 x 4
    QAHE model, where the finite-T values differ from T = 0 by up to 2.3x."""
    lat = _qahe(4, W=1.0, seed=9)
    m = lattice.build(lat)
    opn = m.n_active / (16 * m.cell_area)
    E = [-0.4, 0.0, 0.25]
    for kT in (0.0, 0.1):
        for e in E:
            a, b = cond.sigma_bastin_eigen(m, e, 1e-9, 0, 1, kT), cond.sigma_kubo_eigen(m, e, 0, 1, kT)
            assert abs(a - b) < 1e-7 * abs(b), (kT, e, a, b)
    G = cond.gamma_nm_exact(m, lat.e_min, lat.e_max, 4096, 0, 1)
    for kT in (0.05, 0.2):
        s = cond.sigma_bastin(G, E, lat.e_min, lat.e_max, 0.03, opn, 8192, kT_ev=kT)
        ex = np.array([cond.sigma_bastin_eigen(m, e, 0.03, 0, 1, kT) for e in E])
        assert np.max(np.abs(s - ex) / np.abs(ex)) < 1e-4, (kT, s, ex)


# --- Optical conductivity sigma_ab(omega) (eq. cond 1st order, rank-1 and rank-2 Gamma) ---

def test_gamma1_exact_matches_trace_and_stochastic_basis():
    """gamma_n_exact = Tr[h~^{ab} T_n(H~)]/(N(1+d_n0)) with dense T_n; the stochastic
    gamma_n with the scaled basis vectors (so that <r|r> = N) gives the same trace;
    h~^{ab} is Hermitian and Gamma_n^{ab} real; the n = 1 term of clean graphene
    is the bond sum (1/N) sum_ij d^a_ij d^b_ij |H_ij|^2 / de-."""
    lat = _qahe(3, W=1.5, seed=3).replace(vacancy_p=0.1, disorder_seed=5)
    m = lattice.build(lat)
    Ht = kpm.rescale(m.H, lat.e_min, lat.e_max)
    N = m.n_active
    vecs = np.sqrt(N) * np.eye(N, dtype=complex)
    for ab in ((0, 0), (0, 1), (1, 1)):
        h2 = cond.velocity2(m, *ab).toarray()
        assert np.max(np.abs(h2 - h2.conj().T)) < 1e-14
        G = cond.gamma_n_exact(m, lat.e_min, lat.e_max, 7, *ab)
        Gs = cond.gamma_n(Ht, cond.velocity2(m, *ab), vecs, 7)
        for n in range(7):
            ref = np.trace(h2 @ _cheb_dense(Ht.toarray(), n)) / N / (2 if n == 0 else 1)
            assert abs(G[n] - ref) < 1e-12 and abs(Gs[n] - ref) < 1e-12
    g = wl.Lattice(kind=wl.HONEYCOMB, L1=6, L2=6, t=T_HOP)
    mg = lattice.build(g)
    de_m = 0.5 * (g.e_max - g.e_min)
    G1 = cond.gamma_n_exact(mg, g.e_min, g.e_max, 3, 0, 0)
    dx = np.abs(mg.hx.toarray() / np.where(mg.H.toarray() != 0, mg.H.toarray(), 1))
    ref = np.sum(dx ** 2 * np.abs(mg.H.toarray()) ** 2) / mg.n_active / de_m
    assert abs(G1[1].real - ref) < 1e-12 * ref and abs(G1[0]) < 1e-15


def test_graphene_universal_optical_conductivity():
    """Clean spinless graphene at mu = 0: Re sigma_xx(omega) -> pi/4 e^2/h (the
    universal interband value e^2/(4 hbar) for spin and valley degeneracy 4,
    halved without spin).  k-space sum on a 600^2 torus, eta = 50 meV: within
    1 % at 0.5 eV, and the quadratic extrapolation from 0.5 and 1 eV to omega -> 0
    within 0.5 %; sigma_xy = 0 (time reversal; checked at mu = 50 meV)."""
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=600, L2=600, t=T_HOP, e_min=-9.0, e_max=9.0)
    s = cond.sigma_optical_kgrid(lat, [0.5, 1.0], 0.0, 0.05, 0, 0).real / (np.pi / 4)
    assert abs(s[0] - 1.0) < 0.01, s
    s0 = s[0] - (s[1] - s[0]) / 3.0          # a + b w^2 through w = 0.5, 1
    assert abs(s0 - 1.0) < 0.005, s0
    # sigma_xy at mu = 50 meV (off the degenerate Dirac level, which a 60^2 grid contains).
    assert np.max(np.abs(cond.sigma_optical_kgrid(wl.Lattice(kind=wl.HONEYCOMB, L1=60, L2=60, t=T_HOP),
                                                  [0.5, 1.0], 0.05, 0.05, 0, 1))) < 1e-12


def test_optical_real_space_equals_k_space():
    """Eigenstate sigma_ab(omega) of the real-space torus = the Bloch-state sum (graphene
    xx, QAHE xx and xy): independent matrices, 1e-12."""
    for lat in (wl.Lattice(kind=wl.HONEYCOMB, L1=6, L2=6, t=T_HOP, e_min=-9, e_max=9), _qahe(4)):
        m = lattice.build(lat)
        for ab in ((0, 0), (0, 1)):
            a = cond.sigma_optical_eigen(m, [0.5, 1.0, 2.5], 0.2, 0.1, *ab)
            b = cond.sigma_optical_kgrid(lat, [0.5, 1.0, 2.5], 0.2, 0.1, *ab)
            assert np.max(np.abs(a - b)) < 1e-12 * max(1.0, np.max(np.abs(a)))


def test_optical_spectral_converges_to_eigenstate_definition():
    """The Gamma/Lambda route (exact rank-1 and rank-2 Gamma, M = 2048) against the
    eigenstate formula on the disordered 4 x 4 QAHE model at hbar omega = 0.3,
    1, 2.5 eV, mu = 0.1 eV, eta = 0.1 eV: sigma_xy within 1 %, sigma_xx (M = 512)
    within 1.5 %."""
    lat = _qahe(4, W=1.0, seed=9)
    m = lattice.build(lat)
    opn = m.n_active / (16 * m.cell_area)
    W = [0.3, 1.0, 2.5]
    for ab, M, tol in (((0, 1), 2048, 0.01), ((0, 0), 512, 0.015)):
        ex = cond.sigma_optical_eigen(m, W, 0.1, 0.1, *ab)
        s = cond.sigma_optical(cond.gamma_nm_exact(m, lat.e_min, lat.e_max, M, *ab),
                               cond.gamma_n_exact(m, lat.e_min, lat.e_max, M, *ab), W, 0.1, lat.e_min, lat.e_max,
                               0.1, opn, 2 * M)
        assert np.max(np.abs(s - ex) / np.abs(ex)) < tol, (ab, s, ex)


def test_optical_finite_T_converges_to_eigenstate_definition():
    """The optical route with the Fermi function (kT = 0.1 and 0.4 eV, mu = 0.1 eV)
    against the eigenstate formula with the same occupations: sigma_xx (M = 512) within
    2e-3, sigma_xy (M = 1024) within 1e-4; at kT = 0.4 eV both differ from T = 0 by 7-30 %."""
    lat = _qahe(4, W=1.0, seed=9)
    m = lattice.build(lat)
    opn = m.n_active / (16 * m.cell_area)
    W = [0.3, 1.0, 2.5]
    for ab, M, tol in (((0, 0), 512, 2e-3), ((0, 1), 1024, 1e-4)):
        G2 = cond.gamma_nm_exact(m, lat.e_min, lat.e_max, M, *ab)
        G1 = cond.gamma_n_exact(m, lat.e_min, lat.e_max, M, *ab)
        for kT in (0.1, 0.4):
            ex = cond.sigma_optical_eigen(m, W, 0.1, 0.1, *ab, kT_ev=kT)
            s = cond.sigma_optical(G2, G1, W, 0.1, lat.e_min, lat.e_max, 0.1, opn, 2 * M, kT_ev=kT)
            assert np.max(np.abs(s - ex) / np.abs(ex)) < tol, (ab, kT, s, ex)
        ex0 = cond.sigma_optical_eigen(m, W, 0.1, 0.1, *ab)
        assert np.min(np.abs(ex - ex0) / np.abs(ex0)) > 0.05


# --- Single-shot Fermi-surface DC conductivity --------------------------------

def test_singleshot_equals_gamma_contraction_for_the_same_vectors():
    """With the same random vectors and M, the single-shot sums equal the rank-2
    Gamma route with the weights c_n c_m (an algebraic identity: <a|b> =
    -N de-^2 sum_nm c_n c_m Gamma_nm(1+d_n0)(1+d_m0)/de-^2 ...), here checked
    numerically on a disordered QAHE model with a vacancy, xx and xy."""
    lat = _qahe(3, W=1.5, seed=3).replace(vacancy_p=0.1, disorder_seed=5)
    m = lattice.build(lat)
    M, R = 24, 2
    vecs = kpm.random_phase_vectors(m, R, 11, 0)
    E = np.array([-2.0, 0.0, 0.7])
    Ht = kpm.rescale(m.H, lat.e_min, lat.e_max)
    C = cond.singleshot_coefficients(M, E, lat.e_min, lat.e_max, 0.2)     # includes 1/(de-(1+d_n0))
    omega = 9 * m.cell_area
    for ab in ((0, 0), (0, 1)):
        ss = cond.sigma_singleshot(m, lat.e_min, lat.e_max, E, 0.2, M, vecs, *ab)
        G = cond.gamma_nm(Ht, cond.velocity(m, ab[0]), cond.velocity(m, ab[1]), vecs, M)   # /(R N (1+d)(1+d))
        w = C * np.where(np.arange(M) == 0, 2.0, 1.0)[None, :]                              # c_n / de-
        via_g = -2 * np.pi ** 2 / omega * m.n_active * np.real(np.einsum("kn,nm,km->k", w, G, w))
        assert np.max(np.abs(ss - via_g)) < 1e-10 * np.max(np.abs(ss)), (ab, ss, via_g)


def test_singleshot_converges_to_lorentzian_kubo_greenwood():
    """Exact trace (scaled basis vectors) at M = 2048, eta = 0.2 eV on the disordered
    4 x 4 QAHE model: the single-shot series equals the eigenstate formula with
    Lorentzian deltas to 1e-6 relative (the CPGF series of a Lorentzian converges
    exponentially for eta > 0)."""
    lat = _qahe(4, W=1.0, seed=9)
    m = lattice.build(lat)
    vecs = np.sqrt(m.n_active) * np.eye(m.n_active, dtype=complex)
    E = np.array([-1.5, 0.1, 0.9])
    ss = cond.sigma_singleshot(m, lat.e_min, lat.e_max, E, 0.2, 2048, vecs, 0, 0)
    ex = cond.sigma_kubo_greenwood_eigen(m, E, 0.2)
    assert np.max(np.abs(ss - ex) / np.abs(ex)) < 1e-6, (ss, ex)


def test_kubo_greenwood_real_space_equals_k_space_and_graphene_minimum():
    """Real-space eigenstate Kubo-Greenwood = Bloch-state sum (6 x 6 graphene); clean
    spinless graphene at the Dirac point gives the universal minimum 2/pi e^2/h
    (4 e^2/(pi h) with spin and valley), independent of eta: 600^2 grid, eta = 0.05
    and 0.1 eV, within 0.3 %."""
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=6, L2=6, t=T_HOP, e_min=-9, e_max=9)
    a = cond.sigma_kubo_greenwood_eigen(lattice.build(lat), [0.3, 1.0], 0.2)
    b = cond.sigma_kubo_greenwood_kgrid(lat, [0.3, 1.0], 0.2)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))
    big = wl.Lattice(kind=wl.HONEYCOMB, L1=600, L2=600, t=T_HOP, e_min=-9, e_max=9)
    for eta in (0.05, 0.1):
        s0 = cond.sigma_kubo_greenwood_kgrid(big, [0.0], eta)[0]
        assert abs(s0 - 2 / np.pi) < 0.003 * (2 / np.pi), (eta, s0)
