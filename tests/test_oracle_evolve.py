"""Pins for the oracle's wave-packet time evolution (Chebyshev-Bessel propagator)."""
import numpy as np
import pytest
from scipy import linalg, special

import workload as wl
from oracle import evolve, kpm, lattice

T_HOP = -2.7


def _spinful(L1=3, L2=3, **kw):
    base = dict(kind=wl.HONEYCOMB_SPIN, L1=L1, L2=L2, t=T_HOP, rashba=0.4, exchange=0.3, anderson_w=1.5,
                vacancy_p=0.1, disorder_seed=7, e_min=-10.0, e_max=10.0)
    base.update(kw)
    return wl.Lattice(**base)


def _random_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("lat", [
    _spinful(),
    _spinful(L1=4, L2=3, flux=0.25, vacancy_p=0.0),
    wl.Lattice(kind=wl.SQUARE, L1=5, L2=4, t=T_HOP, anderson_w=2.0, vacancy_p=0.1, disorder_seed=3,
               e_min=-12.0, e_max=12.0),
], ids=["rashba-exchange-vacancies", "rashba-flux", "square"])
def test_bessel_series_equals_matrix_exponential(lat):
    """The series with (-i)^n J_n and the phase exp(-i de+ dt/hbar) equals scipy's dense
    exp(-i H dt/hbar) psi (1e-12) at dt = 0.5, 2 fs; the coefficients as printed,
    (-1)^n J_n, do not conserve the norm (off by > 1 %)."""
    m = lattice.build(lat)
    H = m.H.toarray()
    psi = _random_state(m.n_active, 11)
    for dt in (0.5, 2.0):
        Ht, coef, phase = evolve.step_operator(lat, m, dt, 80)
        got = evolve.propagate(Ht, psi, coef, phase)
        ref = linalg.expm(-1j * H * dt / evolve.HBAR_EV_FS) @ psi
        assert np.max(np.abs(got - ref)) < 1e-12, dt
        n = np.arange(80)
        x = (lat.e_max - lat.e_min) / 2.0 * dt / evolve.HBAR_EV_FS
        printed = np.where(n == 0, 1.0, 2.0) * (-1.0) ** n * special.jv(n, x)
        bad = evolve.propagate(Ht, psi, printed, phase)
        assert abs(np.linalg.norm(bad) - 1.0) > 1e-2


def test_hbar_constant():
    """hbar in eV fs against scipy's CODATA constants."""
    from scipy import constants
    assert abs(evolve.HBAR_EV_FS - constants.hbar / constants.e * 1e15) < 1e-15


def test_group_property_time_reversal_and_norm():
    """U(dt) U(dt) = U(2 dt), U(-dt) U(dt) = 1 (1e-12) and the norm after 30 steps
    (1e-12) on the disordered spinful model with vacancies."""
    lat = _spinful(L1=4, L2=4)
    m = lattice.build(lat)
    psi = _random_state(m.n_active, 5)
    Ht, c1, p1 = evolve.step_operator(lat, m, 1.0, 60)
    _, c2, p2 = evolve.step_operator(lat, m, 2.0, 90)
    _, cm, pm = evolve.step_operator(lat, m, -1.0, 60)
    one = evolve.propagate(Ht, psi, c1, p1)
    two = evolve.propagate(Ht, one, c1, p1)
    assert np.max(np.abs(two - evolve.propagate(Ht, psi, c2, p2))) < 1e-12
    assert np.max(np.abs(evolve.propagate(Ht, one, cm, pm) - psi)) < 1e-12
    _, obs = evolve.evolve(lat, m, psi, 1.0, 60, 31)
    assert np.max(np.abs(obs[:, 0] - 1.0)) < 1e-12


def test_packet_drifts_at_its_mean_velocity_on_a_clean_square_lattice():
    """Clean square lattice 280 x 150, packet with k = (pi/(2a), 0), sigma = 4 nm, kept
    more than 4.5 sigma from the periodic seams: the velocity operator commutes with H,
    so <x>(t) = <x>(0) + t <v_x> (Ehrenfest; 1e-10 nm over 8 fs), with
    <v_x> = -(i/hbar) <psi|[x, H]|psi> from the model's own velocity operator.  That
    velocity is the band's 2|t| a sin(k a)/hbar averaged over the packet's momentum
    spread, |psi(k)|^2 ~ exp(-k^2 sigma^2): 2|t| a/hbar exp(-a^2/(4 sigma^2)) (1e-6).
    <y> stays (1e-7 nm)."""
    lat = wl.Lattice(kind=wl.SQUARE, L1=280, L2=150, t=T_HOP, e_min=-11.0, e_max=11.0)
    m = lattice.build(lat)
    a, sigma = wl.A_SQUARE, 4.0
    psi0 = evolve.gaussian_wavepacket(lat, m, [[np.pi / (2 * a), 0.0]], [[1.0]], sigma, [90, 75])
    v_x = float(np.real(-1j * np.vdot(psi0, m.hx @ psi0))) / evolve.HBAR_EV_FS
    v_ref = 2 * abs(T_HOP) * a / evolve.HBAR_EV_FS * np.exp(-a * a / (4 * sigma * sigma))
    assert abs(v_x - v_ref) < 1e-6 * v_ref, (v_x, v_ref)
    _, obs = evolve.evolve(lat, m, psi0, 1.0, 50, 9)
    t = np.arange(9) * 1.0
    assert np.max(np.abs(obs[:, 1] - obs[0, 1] - v_x * t)) < 1e-10
    assert np.max(np.abs(obs[:, 2] - obs[0, 2])) < 1e-7


def test_spin_precesses_at_twice_the_exchange_over_hbar():
    """With the exchange term alone (no Rashba) H = H_orb (x) 1 + Delta s_z for any
    spin-independent H_orb (Anderson disorder, vacancies): a packet polarised along x
    has <s> = (cos 2 Delta t/hbar, sin 2 Delta t/hbar, 0) at every t (1e-11)."""
    delta = 0.35
    lat = _spinful(L1=8, L2=8, rashba=0.0, exchange=delta, vacancy_p=0.05)
    m = lattice.build(lat)
    sp = np.array([1, 1, 1, 1]) / 2.0          # A up, A down, B up, B down
    psi0 = evolve.gaussian_wavepacket(lat, m, [[1.3, -0.4], [0.2, 2.0]], [sp, sp], 0.6, [4, 4])
    _, obs = evolve.evolve(lat, m, psi0, 0.7, 50, 12)
    w = 2 * delta / evolve.HBAR_EV_FS
    t = np.arange(12) * 0.7
    assert np.max(np.abs(obs[:, 5] - np.cos(w * t))) < 1e-11
    assert np.max(np.abs(obs[:, 6] - np.sin(w * t))) < 1e-11
    assert np.max(np.abs(obs[:, 7])) < 1e-11


def test_gaussian_packet_moments():
    """Clean honeycomb 120 x 120: norm 1, centre at c1 a1 + c2 a2 (1e-6 nm) and variance
    sigma^2/2 along x and y (|psi|^2 has half the envelope's variance; the sites of both
    sublattices sample the same Gaussian; 1e-6 relative at sigma = 3 nm) for a single
    plane wave; a spinor (1, 1)/sqrt 2 per site gives <s_x> = 1 on the spinful lattice,
    and vacancies carry no weight."""
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=120, L2=120, t=T_HOP, e_min=-9.0, e_max=9.0)
    m = lattice.build(lat)
    psi = evolve.gaussian_wavepacket(lat, m, [[0.7, 0.3]], [[1.0, 1.0]], 3.0, [60, 60])
    obs = evolve.observables(lat, m, psi)
    a1, a2, _, _ = lattice._geometry(lat.kind)
    rc = 60 * a1 + 60 * a2
    assert abs(obs[0] - 1.0) < 1e-12 and np.max(np.abs(obs[1:3] - rc)) < 1e-6
    assert abs(obs[3] - obs[1] ** 2 - 4.5) < 4.5e-6
    assert abs(obs[4] - obs[2] ** 2 - 4.5) < 4.5e-6
    lat2 = _spinful(L1=30, L2=30, vacancy_p=0.02)
    m2 = lattice.build(lat2)
    psi2 = evolve.gaussian_wavepacket(lat2, m2, [[0.0, 0.0]], [[1, 1, 1, 1]], 2.0, [15, 15])
    assert psi2.size == m2.n_active and abs(np.linalg.norm(psi2) - 1.0) < 1e-12
    assert abs(evolve.observables(lat2, m2, psi2)[5] - 1.0) < 1e-12
