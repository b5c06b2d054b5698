"""GPU parity for the rank-2 Gamma tensor and sigma_xx against the FP64 oracle.

Tolerances:
* FP64 blocks + FP64 GEMM: element-wise |dGamma| <= 1e-10 max|Gamma| (measured ~1e-14).
* FP32 blocks: every stored vector carries FP32 rounding (~3e-7 per step,
  accumulated over M steps); split-BF16 products add ~3 * 2^-17 relative per
  term.  Gate: ||dGamma||_F / ||Gamma||_F <= 1e-4 (and the split-BF16 GEMM alone,
  against the FP64 GEMM on the same FP32 blocks, <= 2e-5).
"""
import numpy as np
import pytest

import workload as wl
from _bounds import fp32_chain_bound, split_bf16_bound
from oracle import cond as ocond
from oracle import lattice as olat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_05194_amd import kpm
    return kpm


LATS = [
    wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=7, L2=5, t=-2.7, rashba=0.3, flux=2 / 7, anderson_w=0.6,
               vacancy_p=0.03, disorder_seed=21),
    wl.Lattice(kind=wl.HONEYCOMB, L1=11, L2=6, t=-2.7, anderson_w=1.0, vacancy_p=0.05, disorder_seed=4,
               e_min=-8.9, e_max=8.6),
    wl.Lattice(kind=wl.SQUARE, L1=9, L2=13, t=-2.7, anderson_w=2.0, disorder_seed=8, e_min=-12.0, e_max=12.0),
    # QAHE model (eq. HQAHE) with exchange, disorder and vacancies.
    wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=8, L2=6, t=-2.7, rashba=0.81, exchange=1.08, anderson_w=1.25,
               vacancy_p=0.03, disorder_seed=31, e_min=-10.0, e_max=10.0),
]


def rel_fro(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("lat", LATS, ids=lambda l: f"{wl.KIND_NAMES[l.kind]}{l.L1}x{l.L2}")
@pytest.mark.parametrize("ab", [(0, 0), (0, 1), (1, 1)])
def test_gamma_fp64_parity(K, lat, ab):
    M, R = 24, 3
    par = wl.CondParams(num_moments=M, num_random=R, vector_seed=99, alpha=ab[0], beta=ab[1],
                        gamma_mode=wl.GAMMA_FP64)
    G = K.moments_cond(lat, par, precision=wl.FP64)
    Go, _ = ocond.cond_gamma(lat, par)
    err = np.max(np.abs(G - Go)) / np.max(np.abs(Go))
    print(f"Gamma fp64 {lat.kind} {ab}: rel max err {err:.2e}")
    assert err <= 1e-10


@pytest.mark.parametrize("M", [40, 130])
def test_gamma_split_bf16(K, M):
    lat = LATS[0]
    R = 2
    par = wl.CondParams(num_moments=M, num_random=R, vector_seed=7, alpha=0, beta=0,
                        gamma_mode=wl.GAMMA_SPLIT_BF16)
    G_bf16 = K.moments_cond(lat, par, precision=wl.FP32)
    G_f32b = K.moments_cond(lat, par.replace(gamma_mode=wl.GAMMA_FP64), precision=wl.FP32)
    Go, _ = ocond.cond_gamma(lat, par)
    e_gemm = rel_fro(G_bf16, G_f32b)
    e_tot = rel_fro(G_bf16, Go)
    e_f32 = rel_fro(G_f32b, Go)
    print(f"M={M}: split-bf16 vs fp64 GEMM on same blocks {e_gemm:.2e}; fp32 blocks vs oracle {e_f32:.2e}; "
          f"total {e_tot:.2e}")
    assert e_gemm <= 2e-5
    assert e_tot <= 1e-4


def _tile_report(err_ratio, n_idx, m_idx):
    """Worst |dGamma| / B per (128-row n tile, 256-row m tile) of the split-BF16 GEMM."""
    out = {}
    for a, n in enumerate(n_idx):
        for b, m in enumerate(m_idx):
            key = (int(n) // 128, int(m) // 256)
            out[key] = max(out.get(key, 0.0), float(err_ratio[a, b]))
    return out


def test_gamma_split_bf16_elementwise_all_tiles(K):
    """M = 300 (rows padded to 512): the GEMM runs 3 n tiles x 2 m tiles.  Every
    element of split-BF16 Gamma against the FP64 GEMM on the same FP32 blocks
    (the GEMM's own error) under the element bound above, and against the FP64
    oracle (the GEMM plus the FP32 chains) under that bound plus the FP32
    recursion term."""
    lat = LATS[0]
    M, R = 300, 2
    par = wl.CondParams(num_moments=M, num_random=R, vector_seed=7, alpha=0, beta=1,
                        gamma_mode=wl.GAMMA_SPLIT_BF16)
    print(f"split-bf16 elementwise: {lat.L1}x{lat.L2} spinful, M={M}, R={R}", flush=True)
    G_bf16 = K.moments_cond(lat, par, precision=wl.FP32)
    G_f64g = K.moments_cond(lat, par.replace(gamma_mode=wl.GAMMA_FP64), precision=wl.FP32)
    (Go, B), model = ocond.cond_gamma(lat, par, with_bound=True)
    assert np.all(B > 0)
    # Whole K in one chunk is the worst case: K = R x (orbitals padded to a 256 block).
    k_chunk = R * 256 * int(np.ceil(model.H.shape[0] / 256))
    bound = split_bf16_bound(k_chunk)
    d_gemm = np.maximum(np.abs((G_bf16 - G_f64g).real), np.abs((G_bf16 - G_f64g).imag)) / B
    idx = np.arange(M)
    tiles = _tile_report(d_gemm, idx, idx)
    print(f"split-bf16 vs fp64 GEMM: max |dG|/B = {d_gemm.max():.2e} (bound {bound:.2e}); per (n tile, m tile): "
          + ", ".join(f"{k}: {v:.1e}" for k, v in sorted(tiles.items())))
    assert len(tiles) == 6 and all(k[1] in (0, 1) for k in tiles)
    assert np.all(d_gemm <= bound)
    chain = fp32_chain_bound(idx[:, None], idx[None, :])
    d_tot = np.maximum(np.abs((G_bf16 - Go).real), np.abs((G_bf16 - Go).imag)) / B
    d_f32 = np.maximum(np.abs((G_f64g - Go).real), np.abs((G_f64g - Go).imag)) / B
    print(f"fp32 blocks + fp64 GEMM vs oracle: max |dG|/B = {d_f32.max():.2e}; split-bf16 vs oracle: "
          f"{d_tot.max():.2e}; worst ratio to the bound {np.max(d_tot / (bound + chain)):.2f}")
    assert np.all(d_f32 <= chain)
    assert np.all(d_tot <= bound + chain)


def test_batching_matches(K):
    lat = LATS[1]
    par = wl.CondParams(num_moments=20, num_random=5, vector_seed=3, alpha=1, beta=1,
                        gamma_mode=wl.GAMMA_FP64)
    G_all = K.moments_cond(lat, par, precision=wl.FP64)
    G_one = K.moments_cond(lat, par, precision=wl.FP64, max_batch=1)
    G_two = K.moments_cond(lat, par, precision=wl.FP64, max_batch=2)
    scale = np.max(np.abs(G_all))
    assert np.max(np.abs(G_one - G_all)) <= 1e-13 * scale
    assert np.max(np.abs(G_two - G_all)) <= 1e-13 * scale


def test_sigma_reconstruction(K):
    import torch
    lat = LATS[1]
    par = wl.CondParams(num_moments=32, num_random=2, vector_seed=5, gamma_mode=wl.GAMMA_FP64)
    Go, model = ocond.cond_gamma(lat, par)
    E = np.linspace(-8.0, 8.0, 101)
    dens = model.n_active / (lat.L1 * lat.L2 * model.cell_area)
    ref = ocond.sigma_from_gamma(Go, E, lat.e_min, lat.e_max, model.n_active, lat.L1 * lat.L2 * model.cell_area)
    sig = K.reconstruct_sigma(Go, E, lat.e_min, lat.e_max, dens)
    assert np.max(np.abs(sig - ref)) <= 1e-10 * np.max(np.abs(ref))
    gt = torch.tensor(np.stack([Go.real, Go.imag], -1), device="cuda")
    sd = K.reconstruct_sigma(gt, torch.tensor(E, device="cuda"), lat.e_min, lat.e_max, dens)
    assert np.array_equal(sd.cpu().numpy(), sig)


def test_gamma_device_output(K):
    lat = LATS[2]
    par = wl.CondParams(num_moments=16, num_random=1, vector_seed=1, gamma_mode=wl.GAMMA_FP64)
    G = K.moments_cond(lat, par, precision=wl.FP64)
    Gd = K.moments_cond(lat, par, precision=wl.FP64, out_device="cuda")
    gd = Gd.cpu().numpy()
    assert np.array_equal(gd[..., 0] + 1j * gd[..., 1], G)


def test_cond_invalid_mode(K):
    lat = LATS[0]
    par = wl.CondParams(num_moments=8, num_random=1, gamma_mode=wl.GAMMA_SPLIT_BF16)
    with pytest.raises(K.KPMError) as e:
        K.moments_cond(lat, par, precision=wl.FP64)
    assert e.value.code == K.KPM_E_INVALID


def _qahe(L, W=0.0, seed=0):
    return wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=L, L2=L, t=-2.7, rashba=0.81, exchange=1.08, anderson_w=W,
                      disorder_seed=seed, e_min=-10.0, e_max=10.0)


def test_sigma_bastin_matches_oracle(K):
    """kpm_reconstruct_sigma_bastin against the oracle's sigma_bastin (same
    quadrature): the exact Gamma^xy of a disordered 4 x 4 QAHE model (M = 256) at
    T = 0 and kT = 5, 50, 300 meV, and a random complex Gamma with M = 100 (padding
    to the 64-wide tiles), host and device pointers, chemical potentials inside and
    outside the spectrum."""
    import torch
    lat = _qahe(4, W=1.0, seed=9)
    m = olat.build(lat)
    opn = m.n_active / (16 * m.cell_area)
    E = np.array([-11.0, -9.99, -3.0, -0.4, 0.0, 0.25, 2.0, 9.99, 11.0])
    G = ocond.gamma_nm_exact(m, lat.e_min, lat.e_max, 256, 0, 1)
    for eta, q in ((0.1, 1024), (0.03, 700)):
        ref = ocond.sigma_bastin(G, E, lat.e_min, lat.e_max, eta, opn, q)
        got = K.reconstruct_sigma_bastin(G, E, lat.e_min, lat.e_max, eta, opn, n_theta=q)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"bastin eta {eta}: rel err {err:.2e}")
        assert err <= 1e-10
    for kT in (0.005, 0.05, 0.3):
        ref = ocond.sigma_bastin(G, E, lat.e_min, lat.e_max, 0.05, opn, 1024, kT_ev=kT)
        got = K.reconstruct_sigma_bastin(G, E, lat.e_min, lat.e_max, 0.05, opn, n_theta=1024, kT=kT)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"bastin kT {kT}: rel err {err:.2e}")
        assert err <= 1e-10
    rng = np.random.default_rng(4)
    Gr = (rng.standard_normal((100, 100)) + 1j * rng.standard_normal((100, 100))) * 1e-3
    ref = ocond.sigma_bastin(Gr, E, -7.0, 9.0, 0.05, 30.0, 400)
    got = K.reconstruct_sigma_bastin(Gr, E, -7.0, 9.0, 0.05, 30.0)   # default n_theta = 4 M
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))
    gt = torch.tensor(np.stack([Gr.real, Gr.imag], -1), device="cuda")
    gd = K.reconstruct_sigma_bastin(gt, torch.tensor(E, device="cuda"), -7.0, 9.0, 0.05, 30.0)
    assert np.array_equal(gd.cpu().numpy(), got)
    with pytest.raises(K.KPMError):
        K.reconstruct_sigma_bastin(Gr, E, -7.0, 9.0, 0.0, 30.0)
    with pytest.raises(K.KPMError):
        K.reconstruct_sigma_bastin(Gr, E, -7.0, 9.0, 0.05, 30.0, kT=-0.01)


def test_gamma_xy_with_exchange_split_bf16(K):
    """Gamma^xy of the QAHE model through the production path (FP32 chains,
    split-BF16 MFMA GEMM) against the FP64 oracle (same random vectors)."""
    lat = LATS[-1]
    par = wl.CondParams(num_moments=64, num_random=2, vector_seed=13, alpha=0, beta=1,
                        gamma_mode=wl.GAMMA_SPLIT_BF16)
    G = K.moments_cond(lat, par)
    Go, _ = ocond.cond_gamma(lat, par)
    err = rel_fro(G, Go)
    print(f"Gamma^xy QAHE split-bf16: rel fro err {err:.2e}")
    assert err <= 1e-4


def test_qahe_hall_plateau_end_to_end(K):
    """The paper's QAHE result (Sec. 4, Fig. qahe): sigma_xy = 2 e^2/h inside the
    gap of the clean model (lambda_R = 0.3 t, Delta_ex = 0.4 t; the oracle pins
    the Chern number 2 and the 2 e^2/h Kubo sum).  Production path: FP32 chains,
    split-BF16 Gamma^xy, 512 x 512 cells (1,048,576 orbitals), M = 1024, R = 1,
    CPGF eta = 50 meV.  Measured 1.988-2.002 at |E| <= 0.5 eV (gap |E| < 0.62);
    gate 1.5 %.  At room temperature (kT = 25.9 meV, far below the half-gap) the
    plateau holds at |mu| <= 0.3 eV to the same gate."""
    import torch
    L = 512
    lat = _qahe(L)
    par = wl.CondParams(num_moments=1024, num_random=1, vector_seed=3, alpha=0, beta=1,
                        gamma_mode=wl.GAMMA_SPLIT_BF16)
    G = K.moments_cond(lat, par, out_device="cuda")
    cell = wl.A_HONEYCOMB ** 2 * np.sqrt(3) / 2
    opn = 4 / cell
    E = torch.tensor([-0.5, -0.3, 0.0, 0.3, 0.5], dtype=torch.float64, device="cuda")
    s = K.reconstruct_sigma_bastin(G, E, lat.e_min, lat.e_max, 0.05, opn).cpu().numpy()
    print("QAHE sigma_xy:", np.round(s, 4))
    assert np.max(np.abs(s - 2.0)) < 0.03, s
    sT = K.reconstruct_sigma_bastin(G, E[1:4], lat.e_min, lat.e_max, 0.05, opn, kT=0.0259).cpu().numpy()
    print("QAHE sigma_xy at kT = 25.9 meV:", np.round(sT, 4))
    assert np.max(np.abs(sT - 2.0)) < 0.03, sT


@pytest.mark.parametrize("lat", [LATS[0], LATS[1], LATS[3]], ids=["spin-flux", "honeycomb", "qahe"])
@pytest.mark.parametrize("ab", [(0, 0), (0, 1), (1, 1)])
def test_gamma1_parity(K, lat, ab):
    """Rank-1 Gamma_n^{ab} (second-order velocity stencil + recursion + FP64 dots)
    against the oracle with the same random vectors: FP64 1e-10, FP32 2e-5."""
    M, R = 40, 3
    par = wl.CondParams(num_moments=M, num_random=R, vector_seed=17, alpha=ab[0], beta=ab[1])
    ref, _ = ocond.cond_gamma1(lat, par)
    scale = np.max(np.abs(ref))
    g64 = K.moments_gamma1(lat, par, precision=wl.FP64)
    assert np.max(np.abs(g64 - ref)) <= 1e-10 * scale
    g32 = K.moments_gamma1(lat, par, precision=wl.FP32)
    assert np.max(np.abs(g32 - ref)) <= 2e-5 * scale
    gd = K.moments_gamma1(lat, par, precision=wl.FP64, out_device="cuda").cpu().numpy()
    assert np.array_equal(gd[:, 0] + 1j * gd[:, 1], g64)


def test_sigma_optical_matches_oracle(K):
    """kpm_reconstruct_sigma_optical against the oracle's sigma_optical (same
    quadrature) on the exact Gammas of the disordered 4 x 4 QAHE model (M = 200,
    padding to 256), xx and xy, several frequencies, T = 0 and kT = 0.2 eV; host
    and device pointers."""
    import torch
    lat = _qahe(4, W=1.0, seed=9)
    m = olat.build(lat)
    opn = m.n_active / (16 * m.cell_area)
    W = np.array([0.05, 0.3, 1.0, 2.5, 7.0])
    for ab in ((0, 0), (0, 1)):
        G2 = ocond.gamma_nm_exact(m, lat.e_min, lat.e_max, 200, *ab)
        G1 = ocond.gamma_n_exact(m, lat.e_min, lat.e_max, 200, *ab)
        ref = ocond.sigma_optical(G2, G1, W, 0.1, lat.e_min, lat.e_max, 0.1, opn, 900)
        got = K.reconstruct_sigma_optical(G2, G1, W, 0.1, lat.e_min, lat.e_max, 0.1, opn, n_theta=900)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"optical {ab}: rel err {err:.2e}")
        assert err <= 1e-10
        ref = ocond.sigma_optical(G2, G1, W, 0.1, lat.e_min, lat.e_max, 0.1, opn, 900, kT_ev=0.2)
        gT = K.reconstruct_sigma_optical(G2, G1, W, 0.1, lat.e_min, lat.e_max, 0.1, opn, n_theta=900, kT=0.2)
        err = np.max(np.abs(gT - ref)) / np.max(np.abs(ref))
        print(f"optical {ab} kT 0.2: rel err {err:.2e}")
        assert err <= 1e-10
    g2t = torch.tensor(np.stack([G2.real, G2.imag], -1), device="cuda")
    g1t = torch.tensor(np.stack([G1.real, G1.imag], -1), device="cuda")
    d = K.reconstruct_sigma_optical(g2t, g1t, torch.tensor(W, device="cuda"), 0.1, lat.e_min, lat.e_max, 0.1, opn,
                                    n_theta=900).cpu().numpy()
    assert np.array_equal(d[:, 0] + 1j * d[:, 1], got)
    with pytest.raises(K.KPMError):
        K.reconstruct_sigma_optical(G2, G1, np.array([0.5, 0.0]), 0.1, lat.e_min, lat.e_max, 0.1, opn)


def test_graphene_optical_conductivity_end_to_end(K):
    """Clean spinless graphene 1024 x 1024 at mu = 0: Re sigma_xx(omega) from the
    GPU chains (FP32, split-BF16 Gamma, M = 1024, R = 4), the GPU rank-1 Gamma and
    the GPU optical reconstruction (eta = 0.1 eV), against the oracle's converged
    k-space values of the same model (600^2 Bloch grid, same eta; about 1.02,
    1.04, 1.07 times the universal pi/4 e^2/h at 1, 1.5, 2 eV), computed here.
    The remaining difference is the stochastic trace (+-1 % between seeds; FP64
    chains give the same values as FP32): gate 2.5 %."""
    import torch
    L = 1024
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=L, L2=L, t=-2.7, e_min=-9.0, e_max=9.0)
    par = wl.CondParams(num_moments=1024, num_random=4, vector_seed=4, alpha=0, beta=0,
                        gamma_mode=wl.GAMMA_SPLIT_BF16)
    G2 = K.moments_cond(lat, par, out_device="cuda")
    G1 = K.moments_gamma1(lat, par, out_device="cuda")
    opn = 2 / (wl.A_HONEYCOMB ** 2 * np.sqrt(3) / 2)
    W = torch.tensor([1.0, 1.5, 2.0], dtype=torch.float64, device="cuda")
    s = K.reconstruct_sigma_optical(G2, G1, W, 0.0, lat.e_min, lat.e_max, 0.1, opn).cpu().numpy()
    ratio = s[:, 0] / (np.pi / 4)
    ref = ocond.sigma_optical_kgrid(lat.replace(L1=600, L2=600), [1.0, 1.5, 2.0], 0.0, 0.1, 0, 0).real / (np.pi / 4)
    print("graphene Re sigma_xx / (pi/4):", np.round(ratio, 4), "Im:", np.round(s[:, 1], 4), "k-space:",
          np.round(ref, 4))
    assert np.max(np.abs(ratio - ref)) < 0.025, (ratio, ref)


@pytest.mark.parametrize("lat", [LATS[0], LATS[1], LATS[3]], ids=["spin-flux", "honeycomb", "qahe"])
@pytest.mark.parametrize("ab", [(0, 0), (0, 1)])
def test_singleshot_parity(K, lat, ab):
    """kpm_sigma_singleshot against the oracle's single-shot sums with the same
    random vectors (M = 40, R = 2, 5 energies): FP64 1e-10 relative to the largest
    value, FP32 2e-5; device pointers give the same values."""
    import torch
    M, R = 40, 2
    par = wl.CondParams(num_moments=M, num_random=R, vector_seed=23, alpha=ab[0], beta=ab[1])
    m = olat.build(lat)
    from oracle import kpm as okpm
    vecs = okpm.random_phase_vectors(m, R, par.vector_seed, 0)
    E = np.array([lat.e_min * 0.6, -0.8, 0.0, 0.45, lat.e_max * 0.5])
    ref = ocond.sigma_singleshot(m, lat.e_min, lat.e_max, E, 0.15, M, vecs, *ab)
    scale = np.max(np.abs(ref))
    s64 = K.sigma_singleshot(lat, par, E, 0.15, precision=wl.FP64)
    assert np.max(np.abs(s64 - ref)) <= 1e-10 * scale, (s64, ref)
    s32 = K.sigma_singleshot(lat, par, E, 0.15, precision=wl.FP32)
    assert np.max(np.abs(s32 - ref)) <= 2e-5 * scale, (s32, ref)
    sd = K.sigma_singleshot(lat, par, torch.tensor(E, device="cuda"), 0.15, precision=wl.FP64).cpu().numpy()
    assert np.array_equal(sd, s64)


def test_singleshot_history_flushes_and_energy_groups(K):
    """M = 150 (two full 64-vector history flushes and a partial one) and 21 energies
    (two flush passes of up to 16) against the oracle's single-shot sums: FP64 1e-10,
    FP32 2e-5 relative to the largest value."""
    lat = LATS[3]
    M, R = 150, 2
    par = wl.CondParams(num_moments=M, num_random=R, vector_seed=29, alpha=0, beta=1)
    m = olat.build(lat)
    from oracle import kpm as okpm
    vecs = okpm.random_phase_vectors(m, R, par.vector_seed, 0)
    E = np.linspace(lat.e_min * 0.7, lat.e_max * 0.7, 21)
    ref = ocond.sigma_singleshot(m, lat.e_min, lat.e_max, E, 0.12, M, vecs, 0, 1)
    scale = np.max(np.abs(ref))
    s64 = K.sigma_singleshot(lat, par, E, 0.12, precision=wl.FP64)
    assert np.max(np.abs(s64 - ref)) <= 1e-10 * scale, (s64, ref)
    s32 = K.sigma_singleshot(lat, par, E, 0.12, precision=wl.FP32)
    assert np.max(np.abs(s32 - ref)) <= 2e-5 * scale, (s32, ref)


def test_graphene_minimum_conductivity_singleshot(K):
    """Clean spinless graphene 1024 x 1024, single-shot on the GPU (FP32, M = 1024,
    R = 4, eta = 0.1 eV): sigma_xx(0) = 2/pi e^2/h (the universal minimum, pinned in
    the oracle), and the oracle's k-space Kubo-Greenwood values at 0.2 and 0.5 eV
    (600^2 Bloch grid, same eta; about 1.20 and 2.59 e^2/h), computed here; gate 4 %
    (stochastic trace)."""
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=1024, L2=1024, t=-2.7, e_min=-9.0, e_max=9.0)
    par = wl.CondParams(num_moments=1024, num_random=4, vector_seed=6, alpha=0, beta=0)
    s = K.sigma_singleshot(lat, par, np.array([0.0, 0.2, 0.5]), 0.1)
    kg = ocond.sigma_kubo_greenwood_kgrid(lat.replace(L1=600, L2=600), [0.2, 0.5], 0.1, 0, 0)
    ref = np.array([2 / np.pi, kg[0], kg[1]])
    print("graphene single-shot sigma_xx:", np.round(s, 4), "ref", np.round(ref, 4))
    assert np.max(np.abs(s - ref) / ref) < 0.04, s
