"""GPU parity: DOS/LDOS moments from libkpm vs the FP64 oracle, element by element.

Tolerances:
* FP64 path: max |dmu_n| <= 1e-6 (absolute, |mu_n| <= 1); measured ~1e-13.
* FP32 path: the recursion stores FP32 vectors, so each step adds a relative
  rounding error ~ (Z + 2) * 2^-24 ~ 3e-7 to the vector; errors are
  accumulated over ceil(M/2) steps and enter the doubling formula twice, so
  |dmu_n| <= 4 * (M/2) * 3e-7 is the bound used here (5e-5 at M = 64).
"""
import numpy as np
import pytest

import workload as wl
from oracle import kpm as okpm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_05194_amd import kpm
    return kpm


def fp32_tol(M):
    return 4 * (M / 2) * 3e-7


def oracle_moments(lat, par, lat_index=0):
    mu_r, mu, _ = okpm.dos_moments(lat, par, lat_index=lat_index)
    return mu_r, mu


def test_graphene_64_fp64_parity(K):
    """64x64 honeycomb + Anderson W=1, FP64, M=256, R=4 (element-wise vs oracle)."""
    lat, par = wl.graphene_small()
    mu_g, mean_g = K.moments_dos([lat], par)
    mu_o, mean_o = oracle_moments(lat, par)
    err = np.max(np.abs(mu_g[0] - mu_o))
    print("max |dmu| fp64 graphene 64x64:", err)
    assert err <= 1e-6
    assert err <= 1e-11
    assert np.max(np.abs(mean_g[0] - mean_o)) <= 1e-11


RAGGED = [
    wl.Lattice(kind=wl.HONEYCOMB, L1=37, L2=23, t=-2.7, anderson_w=1.0, vacancy_p=0.03, disorder_seed=17,
               e_min=-9.0, e_max=8.7),
    wl.Lattice(kind=wl.HONEYCOMB, L1=19, L2=29, t=-2.7, flux=3 / 19, anderson_w=0.5, disorder_seed=2),
    wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=13, L2=11, t=-2.7, rashba=0.2, flux=2 / 13, anderson_w=0.8,
               vacancy_p=0.02, disorder_seed=5),
    wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=16, L2=9, t=-2.7, rashba=0.35, disorder_seed=6),
    # The paper's QAHE model (eq. HQAHE): Rashba 0.3 t, exchange 0.4 t, Anderson disorder, vacancies.
    wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=12, L2=10, t=-2.7, rashba=0.81, exchange=1.08, anderson_w=1.25,
               vacancy_p=0.02, disorder_seed=12, e_min=-10.0, e_max=10.0),
    wl.Lattice(kind=wl.SQUARE, L1=29, L2=17, t=-2.7, anderson_w=2.0, vacancy_p=0.05, disorder_seed=9,
               e_min=-12.0, e_max=12.0),
]


@pytest.mark.parametrize("lat", RAGGED, ids=lambda l: f"{wl.KIND_NAMES[l.kind]}{l.L1}x{l.L2}")
@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("R", [1, 3, 8])
def test_ragged_lattices(K, lat, prec, R):
    M = 64
    par = wl.DosParams(num_moments=M, num_random=R, vector_seed=5194, precision=prec)
    mu_g, _ = K.moments_dos([lat], par)
    mu_o, _ = oracle_moments(lat, par)
    err = np.max(np.abs(mu_g[0] - mu_o))
    tol = 1e-10 if prec == wl.FP64 else fp32_tol(M)
    print(f"{lat.kind} {lat.L1}x{lat.L2} prec={prec} R={R}: max|dmu|={err:.3e} tol={tol:.1e}")
    assert err <= tol


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32], ids=["fp64", "fp32"])
def test_ldos_sites(K, prec):
    lat = RAGGED[2]
    from oracle import lattice as olat
    model = olat.build(lat)
    sites = [int(model.orb_index[i]) for i in (0, 1, 5, 100, model.n_active - 1)]
    par = wl.DosParams(num_moments=48, start=wl.START_SITES, sites=sites, precision=prec)
    mu_g, _ = K.moments_dos([lat], par)
    mu_o, _, _ = okpm.dos_moments(lat, par, model=model)
    err = np.max(np.abs(mu_g[0] - mu_o))
    assert err <= (1e-10 if prec == wl.FP64 else fp32_tol(48))


def test_ldos_vacant_site_rejected(K):
    lat = RAGGED[0]
    from oracle import lattice as olat
    model = olat.build(lat)
    vac_site = int(np.nonzero(~model.site_active)[0][0])
    par = wl.DosParams(num_moments=8, start=wl.START_SITES, sites=[vac_site])
    with pytest.raises(K.KPMError) as e:
        K.moments_dos([lat], par)
    assert e.value.code == K.KPM_E_INVALID


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32], ids=["fp64", "fp32"])
def test_uneven_batch(K, prec):
    lats = [wl.Lattice(kind=wl.HONEYCOMB, L1=L, L2=L2, t=-2.7, vacancy_p=0.01 * (i + 1),
                       disorder_seed=100 + i)
            for i, (L, L2) in enumerate([(8, 8), (33, 17), (2, 5), (64, 40), (21, 22)])]
    M, R = 80, 4
    par = wl.DosParams(num_moments=M, num_random=R, vector_seed=77, precision=prec)
    mu_g, mean_g = K.moments_dos(lats, par)
    for i, lat in enumerate(lats):
        mu_o, mean_o = oracle_moments(lat, par, lat_index=i)
        err = np.max(np.abs(mu_g[i] - mu_o))
        assert err <= (1e-10 if prec == wl.FP64 else fp32_tol(M)), (i, err)


def test_plan_graph_replay_deterministic(K):
    import torch
    lats = [wl.Lattice(kind=wl.HONEYCOMB, L1=L, L2=L, t=-2.7, vacancy_p=0.005, disorder_seed=i)
            for i, L in enumerate([48, 96, 31])]
    par = wl.DosParams(num_moments=128, num_random=4, vector_seed=5, precision=wl.FP32)
    ref, _ = K.moments_dos(lats, par)
    plan = K.Plan(lats, par, use_graph=True)
    eager = K.Plan(lats, par, use_graph=False)
    outs = []
    for it in range(3):
        mu = torch.zeros((3, 4, 128), dtype=torch.float64, device="cuda")
        plan.run(mu)
        torch.cuda.synchronize()
        outs.append(mu.cpu().numpy())
        # Unrelated eager work between replays.
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
    mu_e = np.zeros((3, 4, 128))
    eager.run(mu_e)
    for o in outs:
        assert np.array_equal(o, outs[0])
    assert np.array_equal(outs[0], mu_e)
    assert np.array_equal(outs[0], ref)
    info = plan.info()
    assert info["n_steps"] == 64 and info["last_loop_ms"] > 0
    plan.close()
    eager.close()


@pytest.mark.parametrize("tune", [dict(block=64, rows=1, grid=8), dict(block=128, rows=3, grid=16),
                                  dict(block=512, rows=8, grid=0), dict(block=512, rows=64, grid=24)])
def test_launch_shapes_agree(K, tune):
    lat = RAGGED[0]
    par = wl.DosParams(num_moments=40, num_random=5, vector_seed=3, precision=wl.FP64)
    mu_o, _ = oracle_moments(lat, par)
    plan = K.Plan([lat], par, **tune)
    mu = np.zeros((1, 5, 40))
    plan.run(mu)
    assert np.max(np.abs(mu[0] - mu_o)) <= 1e-10
    plan.close()


def test_large_r_groups(K):
    """R large enough to need several r-groups per tile (LDOS exact trace of a tiny lattice)."""
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=10, L2=12, t=-2.7, anderson_w=1.0, disorder_seed=4)
    from oracle import lattice as olat
    model = olat.build(lat)
    sites = list(range(model.n_active))          # 240 basis vectors
    par = wl.DosParams(num_moments=32, start=wl.START_SITES, sites=sites, precision=wl.FP64)
    plan = K.Plan([lat], par, block=64)
    mu = np.zeros((1, len(sites), 32))
    mean = np.zeros((1, 32))
    plan.run(mu, mean)
    mu_o, mean_o, _ = okpm.dos_moments(lat, par, model=model)
    assert np.max(np.abs(mu[0] - mu_o)) <= 1e-10
    assert np.max(np.abs(mean[0] - mean_o)) <= 1e-12
    plan.close()


def test_spectrum_escape_detected(K):
    """Bounds inside the band: a quarter of the half-width past the Gershgorin
    radius (8.6 eV here) passes validation and the escape shows in the moments
    (the band edge is near 8.1 eV); farther inside, validation rejects them."""
    lat, par = wl.graphene_small()
    with pytest.raises(K.KPMError) as e:
        K.moments_dos([lat.replace(e_min=-7.6, e_max=7.6)], par.replace(num_moments=128))
    assert e.value.code == K.KPM_E_SPECTRUM
    with pytest.raises(K.KPMError) as e:
        K.moments_dos([lat.replace(e_min=-6.0, e_max=6.0)], par.replace(num_moments=128))
    assert e.value.code == K.KPM_E_INVALID and "Gershgorin" in str(e.value)


def test_device_outputs_and_stream(K):
    import torch
    lat, par = wl.graphene_small()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        mu, mean = K.moments_dos([lat], par, out_device="cuda")
    s.synchronize()
    mu_h, mean_h = K.moments_dos([lat], par)
    assert np.array_equal(mu.cpu().numpy(), mu_h)
    assert np.array_equal(mean.cpu().numpy(), mean_h)


def test_jackson_reconstruction(K):
    import torch
    lat, par = wl.graphene_small()
    mu_o, mean_o = oracle_moments(lat, par)
    E = wl.energy_grid(-9.0, 9.0, 1024)
    ref = okpm.dos(mean_o, E, lat.e_min, lat.e_max)
    rho = K.reconstruct_jackson(mean_o, E, lat.e_min, lat.e_max)
    assert np.max(np.abs(rho - ref)) <= 1e-12 * np.max(np.abs(ref))
    rho_d = K.reconstruct_jackson(torch.tensor(mean_o, device="cuda"), torch.tensor(E, device="cuda"),
                                  lat.e_min, lat.e_max)
    assert np.array_equal(rho_d.cpu().numpy(), rho)
    # Prefix reconstruction with fewer moments (post-processing a subset).
    rho64 = K.reconstruct_jackson(mean_o[:64], E, lat.e_min, lat.e_max)
    ref64 = okpm.dos(mean_o[:64], E, lat.e_min, lat.e_max)
    assert np.max(np.abs(rho64 - ref64)) <= 1e-12 * np.max(np.abs(ref64))


@pytest.mark.parametrize("lat", RAGGED + [wl.Lattice(kind=wl.HONEYCOMB, L1=2, L2=3, t=-2.7, anderson_w=0.3,
                                                      disorder_seed=1)],
                         ids=lambda l: f"{wl.KIND_NAMES[l.kind]}{l.L1}x{l.L2}")
@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32], ids=["fp64", "fp32"])
def test_ring_and_direct_kernels_bitwise_equal(K, lat, prec):
    """The LDS-ring and direct-load step kernels share the per-site arithmetic and
    the reduction order; they agree to rounding (the compiler may contract the
    two kernels' sums into FMAs differently), for several tile shapes."""
    par = wl.DosParams(num_moments=40, num_random=5, vector_seed=8, precision=prec)
    outs = []
    for kernel in (1, 2):
        # (block 384 keeps the ring of the spinful FP64 case within 64 KiB of LDS)
        for tune in (dict(block=64, rows=3), dict(block=256, rows=0), dict(block=384, rows=7, grid=16)):
            plan = K.Plan([lat], par, kernel=kernel, **tune)
            assert plan.info()["kernel"] == kernel
            mu = np.zeros((1, 5, 40))
            plan.run(mu)
            plan.close()
            outs.append(mu)
    tol_pair = 1e-12 if prec == wl.FP64 else 2e-6
    for o in outs[1:]:
        assert np.max(np.abs(o - outs[0])) <= tol_pair
    mu_o, _ = oracle_moments(lat, par)
    tol = 1e-10 if prec == wl.FP64 else fp32_tol(40)
    assert np.max(np.abs(outs[4][0] - mu_o)) <= tol


def test_autotune_cache(K, tmp_path, monkeypatch):
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=96, L2=80, t=-2.7, anderson_w=1.0, disorder_seed=3)
    par = wl.DosParams(num_moments=64, num_random=4, vector_seed=1, precision=wl.FP32)
    cache = str(tmp_path / "tune.txt")
    best = K.autotune([lat], par, probe_steps=4, cache_path=cache)
    assert best["kernel"] in (1, 2, 3, 4, 5, 6) and best["block"] in (256, 448, 512) and best["GBs"] > 0
    line = open(cache).read().strip().split()
    assert [int(v) for v in line[4:9]] == [best["kernel"], best["block"], best["rows"], best["grid"], best["chunks"]]
    monkeypatch.setenv("KPM_TUNE_CACHE", cache)
    plan = K.Plan([lat], par)
    info = plan.info()
    assert (info["kernel"], info["block"], info["rows"], info["grid"]) == \
        (best["kernel"], best["block"], best["rows"], best["grid"])
    assert best["chunks"] == 0 or info["tile_chunks"] == best["chunks"]
    mu = np.zeros((1, 4, 64))
    plan.run(mu)
    plan.close()
    mu_o, _ = oracle_moments(lat, par)
    assert np.max(np.abs(mu[0] - mu_o)) <= fp32_tol(64)


SWEEP_LATS = [
    wl.Lattice(kind=wl.HONEYCOMB, L1=37, L2=23, t=-2.7, anderson_w=1.0, vacancy_p=0.03, disorder_seed=17,
               e_min=-9.0, e_max=8.7),
    wl.Lattice(kind=wl.HONEYCOMB, L1=64, L2=70, t=-2.7, anderson_w=0.7, disorder_seed=3),
    wl.Lattice(kind=wl.HONEYCOMB, L1=2, L2=2, t=-2.7, anderson_w=0.3, disorder_seed=1),
    wl.Lattice(kind=wl.HONEYCOMB, L1=3, L2=5, t=-2.7, disorder_seed=1),
    wl.Lattice(kind=wl.SQUARE, L1=29, L2=17, t=-2.7, anderson_w=2.0, vacancy_p=0.05, disorder_seed=9,
               e_min=-12.0, e_max=12.0),
    wl.Lattice(kind=wl.SQUARE, L1=5, L2=3, t=-2.7, disorder_seed=2, e_min=-11.0, e_max=11.0),
    # Peierls phases (flux per cell 3/19 and 1/4): tile columns wrap across the gauge's seam.
    wl.Lattice(kind=wl.HONEYCOMB, L1=19, L2=29, t=-2.7, flux=3 / 19, anderson_w=0.5, disorder_seed=2),
    wl.Lattice(kind=wl.HONEYCOMB, L1=4, L2=5, t=-2.7, flux=0.25, anderson_w=0.6, vacancy_p=0.05, disorder_seed=8),
]


@pytest.mark.parametrize("lat", SWEEP_LATS, ids=lambda l: f"{wl.KIND_NAMES[l.kind]}{l.L1}x{l.L2}")
@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kernel", [3, 4, 5, 6], ids=["ks2", "ks3", "ks4", "ks5"])
def test_sweep_kernel_matches_single_step_and_oracle(K, lat, prec, kernel):
    """The multi-step sweep kernels (variants 3..6: 2..5 steps per launch)
    against the single-step ring kernel and the oracle: step counts that end
    on a full and on every kind of short last sweep (M = 2 is one step), tile
    shapes down to one row and one r-chunk, halo columns that wrap onto the
    tile itself on tiny lattices, Peierls phases."""
    for M, R in ((2, 3), (8, 5), (14, 2), (41, 2)):
        par = wl.DosParams(num_moments=M, num_random=R, vector_seed=8, precision=prec)
        ref = K.Plan([lat], par, kernel=2)
        mu_r = np.zeros((1, R, M))
        ref.run(mu_r)
        ref.close()
        mu_o, _ = oracle_moments(lat, par)
        tol = 1e-10 if prec == wl.FP64 else fp32_tol(max(M, 8))
        for tune in (dict(block=64, rows=1), dict(block=128, rows=3, grid=16), dict(block=512, rows=0)):
            plan = K.Plan([lat], par, kernel=kernel, **tune)
            # Wide tiles (few r-chunks) may not fit the deeper sweeps' rings in LDS.
            used = plan.info()["kernel"]
            assert used == kernel or (tune["block"] == 512 and 3 <= used < kernel), (used, tune)
            mu = np.zeros((1, R, M))
            plan.run(mu)
            plan.close()
            assert np.max(np.abs(mu - mu_r)) <= (1e-12 if prec == wl.FP64 else 2e-6), (M, tune)
            assert np.max(np.abs(mu[0] - mu_o)) <= tol, (M, tune)


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kernel", [3, 4, 5, 6], ids=["ks2", "ks3", "ks4", "ks5"])
def test_sweep_uneven_batch_and_ldos(K, prec, kernel):
    """Uneven lattices of both spinless kinds in one sweep plan, several
    r-groups per tile (R = 40), and LDOS start vectors."""
    lats = [wl.Lattice(kind=wl.HONEYCOMB, L1=L, L2=L2, t=-2.7, vacancy_p=0.01 * (i + 1), anderson_w=0.5,
                       disorder_seed=100 + i)
            for i, (L, L2) in enumerate([(8, 8), (33, 17), (2, 5), (64, 40), (91, 22)])]
    M, R = 30, 40
    par = wl.DosParams(num_moments=M, num_random=R, vector_seed=77, precision=prec)
    plan = K.Plan(lats, par, kernel=kernel, block=256)
    assert plan.info()["kernel"] == kernel
    mu = np.zeros((len(lats), R, M))
    plan.run(mu)
    plan.close()
    for i, lat in enumerate(lats):
        mu_o, _ = oracle_moments(lat, par, lat_index=i)
        assert np.max(np.abs(mu[i] - mu_o)) <= (1e-10 if prec == wl.FP64 else fp32_tol(M)), i
    lat = SWEEP_LATS[4]
    from oracle import lattice as olat
    model = olat.build(lat)
    sites = [int(model.orb_index[i]) for i in (0, 3, 77, model.n_active - 1)]
    par = wl.DosParams(num_moments=24, start=wl.START_SITES, sites=sites, precision=prec)
    plan = K.Plan([lat], par, kernel=kernel)
    mu = np.zeros((1, len(sites), 24))
    plan.run(mu)
    plan.close()
    mu_o, _, _ = okpm.dos_moments(lat, par, model=model)
    assert np.max(np.abs(mu[0] - mu_o)) <= (1e-10 if prec == wl.FP64 else fp32_tol(24))


@pytest.mark.parametrize("kernel", [3, 4, 5, 6], ids=["ks2", "ks3", "ks4", "ks5"])
def test_sweep_kernel_falls_back_where_ineligible(K, kernel):
    """Spinful lattices (with or without Peierls phases) take the single-step ring kernel."""
    par = wl.DosParams(num_moments=16, num_random=2, vector_seed=3, precision=wl.FP32)
    for lat in (RAGGED[2], RAGGED[3]):
        plan = K.Plan([lat], par, kernel=kernel)
        assert plan.info()["kernel"] == 2
        mu = np.zeros((1, 2, 16))
        plan.run(mu)
        plan.close()
        mu_o, _ = oracle_moments(lat, par)
        assert np.max(np.abs(mu[0] - mu_o)) <= fp32_tol(16)


def test_lorentz_and_cpgf_reconstruction(K):
    """Lorentz-kernel KPM and CPGF (resolvent and DOS) from the GPU against the
    oracle on the same moments, inside and outside the spectrum bounds, host and
    device pointers; and a 20000-term CPGF series of one level against the exact
    Lorentzian (truncation ~ exp(-M eta / sqrt(1 - eps^2)) ~ e^-40)."""
    import torch
    lat, par = wl.graphene_small()
    _, mean_o = oracle_moments(lat, par)
    E = np.concatenate([wl.energy_grid(-9.0, 9.0, 1024), [-12.0, -8.7, 8.9, 12.0]])
    for lam in (1.0, 4.0):
        ref = okpm.dos(mean_o, E, lat.e_min, lat.e_max, kernel=okpm.lorentz(mean_o.size, lam))
        rho = K.reconstruct_lorentz(mean_o, E, lat.e_min, lat.e_max, lam)
        assert np.max(np.abs(rho - ref)) <= 1e-12 * np.max(np.abs(ref))
    for eta in (0.02, 0.3):
        g_ref = okpm.cpgf_green(mean_o, E, lat.e_min, lat.e_max, eta)
        rho, g = K.reconstruct_cpgf(mean_o, E, lat.e_min, lat.e_max, eta, green=True)
        assert np.max(np.abs(g - g_ref)) <= 1e-11 * np.max(np.abs(g_ref))
        assert np.max(np.abs(rho + g_ref.imag / np.pi)) <= 1e-11 * np.max(np.abs(g_ref))
        rho_d, g_d = K.reconstruct_cpgf(torch.tensor(mean_o, device="cuda"), torch.tensor(E, device="cuda"),
                                        lat.e_min, lat.e_max, eta, green=True)
        assert np.array_equal(rho_d.cpu().numpy(), rho) and np.array_equal(g_d.cpu().numpy(), g)
    a, eta, M = -0.4, 0.002, 20000
    mu1 = okpm.chebyshev_t(M, np.array([a]))[:, 0]
    e = np.linspace(-1.2, 1.2, 241)
    rho1 = K.reconstruct_cpgf(mu1, e, -1.0, 1.0, eta)
    lor = eta / (np.pi * ((e - a) ** 2 + eta ** 2))
    assert np.max(np.abs(rho1 - lor) / lor) <= 1e-9
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(K.KPMError):
            K.reconstruct_cpgf(mean_o, E, lat.e_min, lat.e_max, bad)
        with pytest.raises(K.KPMError):
            K.reconstruct_lorentz(mean_o, E, lat.e_min, lat.e_max, bad)


@pytest.mark.parametrize("pattern,per_elem", [(0, 2), (1, 1), (2, 3), (3, 2)], ids=["copy", "read", "rmw", "copy4"])
def test_bandwidth_probe_patterns(K, pattern, per_elem):
    """The HBM probe's patterns (measurement support for the roofline) on an
    array whose element count leaves a tail past the unrolled loop: bytes per
    launch as stated, a positive time."""
    nbytes = (1 << 20) + 3 * 16
    r = K.bandwidth_probe(pattern, nbytes, iters=2, grid=64, block=256, nontemporal=pattern == 3)
    assert r["bytes"] == per_elem * nbytes
    assert r["ms"] > 0 and np.isfinite(r["GBs"])
