"""Pins for the oracle's moments, Jackson kernel and DOS reconstruction.

Each check ties the oracle to something outside its own code: the k-space
spectrum of clean graphene, closed-walk counts, eigen-decompositions of tiny
Hamiltonians (per random vector), exact-trace identities, and sum rules of the
Chebyshev-Gauss quadrature.
"""
import os

import numpy as np
import pytest

import workload as wl
from oracle import kpm, lattice

GOLDEN_WALKS = os.path.join(os.path.dirname(__file__), "golden", "honeycomb_walks.txt")


def _walks():
    out = {}
    with open(GOLDEN_WALKS) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, a = line.split()
                out[int(k)] = int(a)
    return out


def _exact_trace_moments(lat, M):
    m = lattice.build(lat)
    par = wl.DosParams(num_moments=M, start=wl.START_SITES, sites=list(m.orb_index))
    mu_r, mu, _ = kpm.dos_moments(lat, par, model=m)
    return mu, m


def test_exact_trace_matches_kspace_graphene():
    L1, L2, t, M = 10, 12, -2.7, 48
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=L1, L2=L2, t=t, e_min=-8.5, e_max=8.5)
    mu, _ = _exact_trace_moments(lat, M)
    k1 = 2 * np.pi * np.arange(L1) / L1
    k2 = 2 * np.pi * np.arange(L2) / L2
    K1, K2 = np.meshgrid(k1, k2)
    e = (np.abs(t) * np.abs(1 + np.exp(1j * (K1 - K2)) + np.exp(-1j * K2))).ravel() / 8.5
    ref = np.array([0.5 * np.mean(np.cos(n * np.arccos(e)) + np.cos(n * np.arccos(-e))) for n in range(M)])
    assert np.max(np.abs(mu - ref)) < 1e-12


def test_walk_count_moments():
    """mu_2, mu_4, mu_6 of clean graphene from closed-walk counts (t = -2.7, bound 8.5)."""
    a = _walks()
    x2 = (2.7 / 8.5) ** 2
    m2 = [a[k] * x2 ** k for k in range(4)]       # <x^(2k)> for k = 0..3
    ref = {2: 2 * m2[1] - 1,
           4: 8 * m2[2] - 8 * m2[1] + 1,
           6: 32 * m2[3] - 48 * m2[2] + 18 * m2[1] - 1}
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=8, L2=8, t=-2.7)
    mu, _ = _exact_trace_moments(lat, 8)
    for n, v in ref.items():
        assert abs(mu[n] - v) < 1e-12
    assert abs(ref[2] - (-0.394602076)) < 1e-9
    assert np.all(np.abs(mu[1::2]) < 1e-13)


def _eig_moments(model, Ht_dense, vec, M, norm):
    lam, U = np.linalg.eigh(Ht_dense)
    w = np.abs(U.conj().T @ vec) ** 2
    n = np.arange(M)[:, None]
    return (np.cos(n * np.arccos(np.clip(lam, -1, 1))[None, :]) @ w) / norm


CASES = [
    wl.Lattice(kind=wl.HONEYCOMB, L1=6, L2=5, t=-2.7, anderson_w=1.0, vacancy_p=0.05, disorder_seed=7,
               e_min=-9.0, e_max=8.0),
    wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=6, L2=4, t=-2.7, rashba=0.2, flux=1 / 6, anderson_w=0.5,
               disorder_seed=3),
    wl.Lattice(kind=wl.SQUARE, L1=7, L2=6, t=-2.7, anderson_w=3.0, vacancy_p=0.02, disorder_seed=9,
               e_min=-12.5, e_max=12.5),
    wl.Lattice(kind=wl.HONEYCOMB, L1=6, L2=6, t=-2.7, flux=2 / 6, disorder_seed=1),
]


@pytest.mark.parametrize("lat", CASES)
def test_per_vector_moments_match_eigendecomposition(lat):
    M, R = 64, 3
    par = wl.DosParams(num_moments=M, num_random=R, vector_seed=5194)
    mu_r, mu, model = kpm.dos_moments(lat, par)
    Ht = kpm.rescale(model.H, lat.e_min, lat.e_max).toarray()
    vecs = kpm.random_phase_vectors(model, R, 5194)
    for r in range(R):
        ref = _eig_moments(model, Ht, vecs[r], M, model.n_active)
        assert np.max(np.abs(mu_r[r] - ref)) < 1e-12
    assert np.allclose(mu_r[:, 0], 1.0, atol=1e-14, rtol=0)
    assert np.all(np.abs(mu_r) <= 1 + 1e-12)


def test_ldos_matches_eigendecomposition():
    lat = CASES[0]
    M = 40
    model = lattice.build(lat)
    sites = [int(model.orb_index[0]), int(model.orb_index[7]), int(model.orb_index[-1])]
    par = wl.DosParams(num_moments=M, start=wl.START_SITES, sites=sites)
    mu_r, _, _ = kpm.dos_moments(lat, par, model=model)
    Ht = kpm.rescale(model.H, lat.e_min, lat.e_max).toarray()
    for r, o in enumerate(sites):
        v = np.zeros(model.n_active, dtype=complex)
        v[list(model.orb_index).index(o)] = 1
        assert np.max(np.abs(mu_r[r] - _eig_moments(model, Ht, v, M, 1.0))) < 1e-12
    with pytest.raises(ValueError):
        vac = int(np.nonzero(~model.site_active)[0][0])
        kpm.dos_moments(lat, par.replace(sites=[vac]), model=model)


def test_exact_trace_identities():
    lat = CASES[0]
    mu, model = _exact_trace_moments(lat, 6)
    Ht = kpm.rescale(model.H, lat.e_min, lat.e_max).toarray()
    N = model.n_active
    assert abs(mu[0] - 1) < 1e-14
    assert abs(mu[1] - np.trace(Ht).real / N) < 1e-14
    assert abs(mu[2] - (2 * np.sum(np.abs(Ht) ** 2) / N - 1)) < 1e-13


def test_stochastic_trace_within_error():
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=16, L2=16, t=-2.7, anderson_w=1.0, disorder_seed=1910)
    M, R = 32, 24
    mu_exact, model = _exact_trace_moments(lat, M)
    par = wl.DosParams(num_moments=M, num_random=R, vector_seed=5194)
    mu_r, mu, _ = kpm.dos_moments(lat, par, model=model)
    sem = mu_r.std(axis=0, ddof=1) / np.sqrt(R)
    assert np.all(np.abs(mu[1:] - mu_exact[1:]) <= 5 * sem[1:] + 1e-12)


def test_random_phase_variance_bound():
    """The statistical error behind the learned path's acceptance test: for
    random-phase vectors one vector's estimate of mu_n = Tr T_n(H~)/N has
    variance sum_{i != j} |T_n,ij|^2 / N^2 (the phases of different orbitals
    are independent and uniform), at most Tr T_n(H~)^2 / N^2 = (1 + mu_2n) /
    (2 N) <= 1/N.  Exact variances from dense T_n on a disordered lattice with
    vacancies against the bound, and the sample variance of 1600 vectors'
    moments against the exact variance (the spread of a sample variance of
    1600 draws is about 3.5 %)."""
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=6, L2=5, t=-2.7, anderson_w=1.5, vacancy_p=0.05, disorder_seed=3)
    M, R = 12, 1600
    par = wl.DosParams(num_moments=M, num_random=R, vector_seed=11)
    mu_r, _, model = kpm.dos_moments(lat, par)
    N = model.n_active
    Ht = kpm.rescale(model.H, lat.e_min, lat.e_max).toarray()
    T = [np.eye(N), Ht.copy()]
    for _ in range(2, 2 * M):
        T.append(2 * Ht @ T[-1] - T[-2])
    mu_exact = np.array([np.trace(t).real / N for t in T])
    for n in range(1, M):
        off = np.sum(np.abs(T[n]) ** 2) - np.sum(np.abs(np.diag(T[n])) ** 2)
        var = off / N ** 2
        assert abs(np.sum(np.abs(T[n]) ** 2) / N ** 2 - (1 + mu_exact[2 * n]) / (2 * N)) < 1e-12
        assert var <= (1 + mu_exact[2 * n]) / (2 * N) + 1e-15 <= 1.0 / N + 1e-15
        assert abs(np.var(mu_r[:, n], ddof=1) / var - 1) < 0.2, (n, np.var(mu_r[:, n], ddof=1), var)
    # A planted mistake, the diagonal counted in the variance, fails the sample
    # comparison at n = 2 (where the diagonal holds 40 % of ||T_2||_F^2).
    wrong = np.sum(np.abs(T[2]) ** 2) / N ** 2
    assert abs(np.var(mu_r[:, 2], ddof=1) / wrong - 1) >= 0.2


def test_jackson_kernel_properties():
    for M in [2, 16, 256, 2048]:
        g = kpm.jackson(M)
        assert abs(g[0] - 1) < 1e-14
        assert np.all(g > 0) and np.all(g <= 1 + 1e-15)
        assert np.all(np.diff(g) < 0)
        # Extending the formula to n = M gives exactly zero.
        q = np.pi / (M + 1)
        gM = (np.cos(q * M) + np.sin(q * M) / np.tan(q)) / (M + 1)
        assert abs(gM) < 1e-15 * M


def test_dos_sum_rules_chebyshev_gauss():
    """With Chebyshev-Gauss nodes, (1/K) sum_k pi sqrt(1-e_k^2) rho~(e_k) = g0 mu0 and
    (1/K) sum_k e_k pi sqrt(1-e_k^2) rho~(e_k) = g1 mu1 exactly for M < 2K."""
    lat = CASES[0]
    M, K = 128, 512
    par = wl.DosParams(num_moments=M, num_random=2, vector_seed=1)
    _, mu, _ = kpm.dos_moments(lat, par)
    de_p = 0.5 * (lat.e_max + lat.e_min)
    de_m = 0.5 * (lat.e_max - lat.e_min)
    eps = np.cos(np.pi * (np.arange(K) + 0.5) / K)
    rho = kpm.dos(mu, de_p + de_m * eps, lat.e_min, lat.e_max) * de_m
    w = np.pi * np.sqrt(1 - eps ** 2) / K
    g = kpm.jackson(M)
    assert abs(np.sum(w * rho) - g[0] * mu[0]) < 1e-12
    assert abs(np.sum(w * eps * rho) - g[1] * mu[1]) < 1e-12


def test_dos_positive_for_single_vector_moments():
    lat = CASES[1]
    par = wl.DosParams(num_moments=200, num_random=1, vector_seed=3)
    mu_r, _, _ = kpm.dos_moments(lat, par)
    E = wl.energy_grid(lat.e_min, lat.e_max, 1024)
    rho = kpm.dos(mu_r[0], E, lat.e_min, lat.e_max)
    assert rho.min() > -1e-12


def test_delta_peak_is_resolved():
    """Moments of a single level at a: the Jackson DOS peaks at a with width ~ pi/M."""
    M, a = 256, 0.3
    mu = np.cos(np.arange(M) * np.arccos(a))
    eps = np.linspace(-0.99, 0.99, 20001)
    rho = kpm.dos(mu, eps, -1.0, 1.0)
    k = np.argmax(rho)
    assert abs(eps[k] - a) < 2e-3
    de = eps[1] - eps[0]
    assert abs(np.sum(rho) * de - 1.0) < 1e-3
    sd = np.sqrt(np.sum(rho * (eps - a) ** 2) * de)
    ref = np.pi / M * np.sqrt(1 - a * a)
    assert 0.8 * ref < sd < 1.25 * ref


def test_kspace_moments_pinned_to_exact_trace_and_walks():
    """The k-space closed form equals the exact trace of the explicit Hamiltonian
    (LDOS over all basis vectors) on a small torus, the walk-count moments, and
    is independent of the torus size for n < 2 min(L1, L2)."""
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=10, L2=12, t=-2.7, e_min=-8.5, e_max=8.5)
    mu, _ = _exact_trace_moments(lat, 40)
    ks = kpm.honeycomb_kspace_moments(10, 12, -2.7, -8.5, 8.5, 40)
    assert np.max(np.abs(mu - ks)) < 1e-12
    a = _walks()
    x2 = (2.7 / 8.5) ** 2
    assert abs(ks[2] - (2 * a[1] * x2 - 1)) < 1e-12
    big = kpm.honeycomb_kspace_moments(40, 37, -2.7, -8.5, 8.5, 60)
    small = kpm.honeycomb_kspace_moments(16, 15, -2.7, -8.5, 8.5, 60)
    assert np.max(np.abs(big[:30] - small[:30])) < 1e-12      # n < 2 * 15
    assert np.max(np.abs(big[30:] - small[30:])) > 1e-6       # the small torus winds beyond
    # Asymmetric bounds shift the rescaled spectrum: mu_1 = -d_plus / d_minus.
    sh = kpm.honeycomb_kspace_moments(8, 8, -2.7, -8.0, 9.0, 4)
    assert abs(sh[1] - (-0.5 / 8.5)) < 1e-12


def test_lorentz_kernel_properties_and_width():
    """Lorentz kernel: g_0 = 1, strictly decreasing, positive; a delta peak at the
    band centre becomes a near-Lorentzian of half width ~ lam/M."""
    M, lam = 1000, 4.0
    g = kpm.lorentz(M, lam)
    assert g[0] == 1.0 and np.all(np.diff(g) < 0) and np.all(g > 0)
    assert abs(g[-1] - np.sinh(lam / M) / np.sinh(lam)) < 1e-15
    mu = kpm.chebyshev_t(M, np.array([0.0]))[:, 0]           # mu_n = T_n(0): a level at eps = 0
    E = np.linspace(-0.05, 0.05, 20001)
    rho = kpm.dos(mu, E, -1.0, 1.0, kernel=g)
    half = E[rho >= rho.max() / 2]
    hwhm = (half[-1] - half[0]) / 2
    assert abs(hwhm / (lam / M) - 1) < 0.1


def test_cpgf_single_level_is_lorentzian():
    """The CPGF series of one level (mu_n = T_n(a)) sums to the broadened delta
    eta / (pi ((eps - a)^2 + eta^2)); truncation error ~ |exp(-i arccos z)|^M."""
    a, eta, M = 0.3, 0.01, 3000
    mu = kpm.chebyshev_t(M, np.array([a]))[:, 0]
    E = np.linspace(-1.5, 1.5, 601)                            # also outside the band
    rho = kpm.cpgf_dos(mu, E, -1.0, 1.0, eta)
    ref = eta / (np.pi * ((E - a) ** 2 + eta ** 2))
    assert np.max(np.abs(rho - ref) / ref) < 1e-9


def test_cpgf_green_matches_resolvent_trace():
    """(1/N) Tr 1/(E - H + i eta) of a disordered, vacancy-diluted honeycomb torus
    from dense eigenvalues, against the CPGF sum over its exact-trace moments."""
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=6, L2=5, t=-2.7, anderson_w=1.5, vacancy_p=0.05, disorder_seed=3,
                     e_min=-9.0, e_max=9.0)
    m = lattice.build(lat)
    lam = np.linalg.eigvalsh(m.H.toarray())
    M, eta = 4000, 0.1
    x = (lam - 0.0) / 9.0
    mu = np.cos(np.arange(M)[:, None] * np.arccos(x)[None, :]).mean(axis=1)
    E = np.linspace(-10.0, 10.0, 81)
    G = kpm.cpgf_green(mu, E, -9.0, 9.0, eta)
    ref = np.mean(1.0 / (E[:, None] - lam[None, :] + 1j * eta), axis=1)
    assert np.max(np.abs(G - ref) / np.abs(ref)) < 1e-10
    assert np.allclose(kpm.cpgf_dos(mu, E, -9.0, 9.0, eta), -ref.imag / np.pi, rtol=1e-10, atol=0)
