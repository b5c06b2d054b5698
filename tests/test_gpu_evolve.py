"""GPU parity of the wave-packet time evolution (kpm_wavepacket_gaussian,
kpm_time_evolve) against the oracle's Chebyshev-Bessel propagator."""
import numpy as np
import pytest

import workload as wl
from oracle import evolve as oev
from oracle import lattice as olat

pytestmark = pytest.mark.gpu

T_HOP = -2.7
LATS = [
    wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=8, L2=6, t=T_HOP, rashba=0.4, exchange=0.3, anderson_w=1.5, vacancy_p=0.08,
               disorder_seed=7, e_min=-10.0, e_max=10.0),
    wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=8, L2=6, t=T_HOP, rashba=0.3, flux=0.25, anderson_w=0.5, disorder_seed=2,
               e_min=-10.0, e_max=10.0),
    wl.Lattice(kind=wl.HONEYCOMB, L1=12, L2=10, t=T_HOP, anderson_w=1.0, vacancy_p=0.05, disorder_seed=4,
               e_min=-9.0, e_max=9.0),
    wl.Lattice(kind=wl.SQUARE, L1=9, L2=7, t=T_HOP, anderson_w=2.0, vacancy_p=0.05, disorder_seed=3,
               e_min=-12.0, e_max=12.0),
]
IDS = ["spin-rashba-exchange-vac", "spin-rashba-flux", "honeycomb-vac", "square-vac"]


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_05194_amd import kpm
    return kpm


def _per_cell(lat):
    return {wl.HONEYCOMB: 2, wl.HONEYCOMB_SPIN: 4, wl.SQUARE: 1}[lat.kind]


def _packets(lat, m, R):
    """R oracle packets (different momenta, spinors, centres) in the active-orbital space."""
    rng = np.random.default_rng(3)
    out = []
    for r in range(R):
        kv = rng.uniform(-3, 3, size=(2, 2))
        sp = rng.standard_normal((2, _per_cell(lat))) + 1j * rng.standard_normal((2, _per_cell(lat)))
        out.append((kv, sp, 0.5 + 0.2 * r, [lat.L1 / 2 + r, lat.L2 / 2 - r]))
    return out


def _full(m, lat, psi):
    f = np.zeros(lat.L1 * lat.L2 * _per_cell(lat), dtype=np.complex128)
    f[m.orb_index] = psi
    return f


@pytest.mark.parametrize("lat", LATS, ids=IDS)
def test_wavepacket_builder_matches_oracle(K, lat):
    """The Gaussian packet from the GPU against the oracle's (1e-12), zero on vacancies,
    host and device outputs identical."""
    m = olat.build(lat)
    for kv, sp, w, c in _packets(lat, m, 2):
        ref = _full(m, lat, oev.gaussian_wavepacket(lat, m, kv, sp, w, c))
        got = K.wavepacket_gaussian(lat, kv, sp, w, c)
        assert np.max(np.abs(got - ref)) < 1e-12
        d = K.wavepacket_gaussian(lat, kv, sp, w, c, out_device="cuda").cpu().numpy()
        assert np.array_equal(d[:, 0] + 1j * d[:, 1], got)


@pytest.mark.parametrize("lat", LATS, ids=IDS)
def test_time_evolution_matches_oracle(K, lat):
    """R = 3 packets (FP32 packs two per 16 bytes: one padded slot), M = 150 terms
    per step (history flushes of 64, 64 and 22 vectors), 4 time points of 1 fs:
    states and observables against the oracle, FP64 1e-10, FP32 2e-5."""
    m = olat.build(lat)
    R, M, npt, dt = 3, 150, 4, 1.0
    pk = [oev.gaussian_wavepacket(lat, m, *p) for p in _packets(lat, m, R)]
    refs = [oev.evolve(lat, m, p, dt, M, npt) for p in pk]
    psi0 = np.stack([_full(m, lat, p) for p in pk])
    for prec, tol in ((wl.FP64, 1e-10), (wl.FP32, 2e-5)):
        psi_t, obs = K.time_evolve(lat, psi0, dt, M, npt, precision=prec)
        for r in range(R):
            assert np.max(np.abs(psi_t[r] - _full(m, lat, refs[r][0]))) < tol, (prec, r)
            scale = np.maximum(1.0, np.abs(refs[r][1]))
            assert np.max(np.abs(obs[:, r, :] - refs[r][1]) / scale) < tol, (prec, r, obs[:, r, :], refs[r][1])


def test_device_pointers_and_arguments(K):
    """Device inputs give the host path's values bit for bit; amplitude on vacant
    orbitals is ignored; M < 2, dt = 0 and a spinless lattice's spin components (zero)
    are handled."""
    import torch
    lat = LATS[0]
    m = olat.build(lat)
    p = oev.gaussian_wavepacket(lat, m, *_packets(lat, m, 1)[0])
    psi0 = _full(m, lat, p)
    h_psi, h_obs = K.time_evolve(lat, psi0, 0.8, 60, 3, precision=wl.FP64)
    t0 = torch.tensor(np.stack([psi0.real, psi0.imag], -1), device="cuda")
    d_psi, d_obs = K.time_evolve(lat, t0, 0.8, 60, 3, precision=wl.FP64)
    d_psi = d_psi.cpu().numpy()[0]
    assert np.array_equal(d_psi[:, 0] + 1j * d_psi[:, 1], h_psi)
    assert np.array_equal(d_obs.cpu().numpy()[:, 0, :], h_obs[:, 0, :])
    # Amplitude on vacant orbitals is ignored: bit-identical results.
    vac = np.setdiff1d(np.arange(psi0.size), m.orb_index)
    assert vac.size > 0
    bad = psi0.copy()
    bad[vac] = 0.3 - 0.7j
    b_psi, b_obs = K.time_evolve(lat, bad, 0.8, 60, 3, precision=wl.FP64)
    assert np.array_equal(b_psi, h_psi) and np.array_equal(b_obs, h_obs)
    with pytest.raises(K.KPMError):
        K.time_evolve(lat, psi0, 0.8, 1, 3)
    with pytest.raises(K.KPMError):
        K.time_evolve(lat, psi0, 0.0, 60, 3)
    lat2 = LATS[2]
    m2 = olat.build(lat2)
    p2 = _full(m2, lat2, oev.gaussian_wavepacket(lat2, m2, *_packets(lat2, m2, 1)[0]))
    _, o2 = K.time_evolve(lat2, p2, 0.8, 60, 3, precision=wl.FP64)
    assert np.all(o2[:, 0, 5:] == 0.0)


def test_exchange_precession_and_norm_at_size(K):
    """Spinful honeycomb 512 x 512 (1,048,576 orbitals) with Anderson disorder, vacancies
    and the exchange term alone: a packet polarised along x precesses as
    (cos 2 Delta t/hbar, sin 2 Delta t/hbar, 0) (exact for any spin-independent
    orbital part) and keeps its norm; FP32, 2 fs steps, M = 60, 16 time points."""
    delta = 0.05
    lat = wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=512, L2=512, t=T_HOP, exchange=delta, anderson_w=1.0,
                     vacancy_p=0.01, disorder_seed=11, e_min=-9.5, e_max=9.5)
    sp = np.array([1, 1, 1, 1]) / 2.0
    psi0 = K.wavepacket_gaussian(lat, [[2.0, 0.5]], [sp], 12.0, [256, 256], out_device="cuda")
    _, obs = K.time_evolve(lat, psi0.unsqueeze(0), 2.0, 60, 16, precision=wl.FP32)
    st = K.evolve_last_stats()
    # 60 terms: flushes of 32 and 28 history vectors; FP32 packs of 2 complex (R = 1 padded to 2).
    vec = lat.L1 * lat.L2 * 4 * 2 * 8
    site = lat.L1 * lat.L2 * 2 * (4 + 1)
    assert st["history"] == 32 and st["time_steps"] == 15 and st["loop_ms"] > 0
    assert st["bytes"] == pytest.approx(15 * (59 * (3 * vec + site) + (60 + 2 * 2 - 1) * vec), rel=1e-12)
    obs = obs.cpu().numpy()[:, 0, :]
    t = np.arange(16) * 2.0
    w = 2 * delta / oev.HBAR_EV_FS
    print("S_x:", np.round(obs[:, 5], 5), "norm drift:", np.max(np.abs(obs[:, 0] - 1)))
    assert np.max(np.abs(obs[:, 0] - 1.0)) < 1e-4
    assert np.max(np.abs(obs[:, 5] - np.cos(w * t))) < 1e-4
    assert np.max(np.abs(obs[:, 6] - np.sin(w * t))) < 1e-4
    assert np.max(np.abs(obs[:, 7])) < 1e-4


def test_backward_steps_return_the_initial_state(K):
    """Ten steps of +1.5 fs then ten of -1.5 fs bring the packets back (FP64 1e-11) on
    the disordered spinful lattice with vacancies; observables at the end equal those
    at t = 0."""
    lat = LATS[0]
    m = olat.build(lat)
    pk = np.stack([_full(m, lat, oev.gaussian_wavepacket(lat, m, *p)) for p in _packets(lat, m, 2)])
    fwd, o1 = K.time_evolve(lat, pk, 1.5, 60, 11, precision=wl.FP64)
    back, o2 = K.time_evolve(lat, fwd, -1.5, 60, 11, precision=wl.FP64)
    assert np.max(np.abs(back - pk)) < 1e-11
    assert np.max(np.abs(o2[-1] - o1[0])) < 1e-10
