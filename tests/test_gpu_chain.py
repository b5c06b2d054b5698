"""Multi-step sweeps of the Gamma chains (chain_sweep_kernel, kpm_chain.hip)
against single steps and the oracle (eq. Gammanm, eq. generalized velocity).

kpm_moments_cond runs its two chains as KS-step sweeps by default (KS = 4 on
the spinful lattice, 3 there in FP64; KS = 2 on the spinless ones).  KPM_CHAIN_STEPS = 1 selects one step per launch,
2..4 the steps per sweep; KPM_CHAIN_ROWS the rows per tile.  In FP64 the
sweeps reproduce single steps to rounding (1e-12 of max |Gamma|) and the
oracle to 1e-10; the split-BF16 path stays within the element bound of the
GEMM plus the FP32 chain term against the oracle.

Cases: spinful Rashba + exchange + Peierls flux + Anderson + vacancies,
spinless honeycomb with flux and vacancies, the square lattice; lattices
wider than one tile (several column tiles, a ragged last one) and taller
than one row band (several row tiles, a ragged last one); chain lengths
that leave a short last sweep (M - 1 and M not multiples of KS) and chains
shorter than one sweep (M = 2, 3).
"""
import numpy as np
import pytest

import workload as wl
from _bounds import fp32_chain_bound, split_bf16_bound
from oracle import cond as ocond

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_05194_amd import kpm
    return kpm


SPIN = wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=14, L2=11, t=-2.7, rashba=0.4, exchange=0.3, flux=1 / 14,
                  anderson_w=0.8, vacancy_p=0.03, disorder_seed=21, e_min=-9.5, e_max=9.5)
SPIN_WIDE = wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=70, L2=7, t=-2.7, rashba=0.3, flux=1 / 70, anderson_w=0.5,
                       disorder_seed=4, e_min=-9.5, e_max=9.5)
HC = wl.Lattice(kind=wl.HONEYCOMB, L1=12, L2=40, t=-2.7, flux=1 / 12, anderson_w=1.0, vacancy_p=0.04,
                disorder_seed=9)
SQ = wl.Lattice(kind=wl.SQUARE, L1=9, L2=13, t=-2.7, anderson_w=2.0, disorder_seed=8, e_min=-12.0, e_max=12.0)


def _gamma(K, monkeypatch, lat, par, prec, steps, rows=None):
    monkeypatch.setenv("KPM_CHAIN_STEPS", str(steps))
    if rows is None:
        monkeypatch.delenv("KPM_CHAIN_ROWS", raising=False)
    else:
        monkeypatch.setenv("KPM_CHAIN_ROWS", str(rows))
    return K.moments_cond(lat, par, precision=prec)


@pytest.mark.parametrize("lat,rows", [(SPIN, None), (SPIN, 4), (SPIN_WIDE, None), (HC, 16), (SQ, 5)],
                         ids=["spin", "spin-rows4", "spin-wide", "honeycomb-rows16", "square-rows5"])
@pytest.mark.parametrize("M", [2, 3, 23])
def test_chain_sweeps_fp64_match_single_steps_and_oracle(K, monkeypatch, lat, rows, M):
    par = wl.CondParams(num_moments=M, num_random=2, vector_seed=31, alpha=0, beta=1, gamma_mode=wl.GAMMA_FP64)
    print(f"chain sweep fp64: {wl.KIND_NAMES[lat.kind]} {lat.L1}x{lat.L2}, M={M}, rows={rows}", flush=True)
    G1 = _gamma(K, monkeypatch, lat, par, wl.FP64, 1)
    scale = np.max(np.abs(G1))
    for ks in (2, 3, 4):
        Gk = _gamma(K, monkeypatch, lat, par, wl.FP64, ks, rows)
        err = np.max(np.abs(Gk - G1)) / scale
        print(f"  KS={ks}: max |G - G_single| / max |G| = {err:.2e}", flush=True)
        assert err <= 1e-12, (ks, err)
    Go, _ = ocond.cond_gamma(lat, par)
    err = np.max(np.abs(Gk - Go)) / np.max(np.abs(Go))
    print(f"  vs oracle: {err:.2e}", flush=True)
    assert err <= 1e-10


@pytest.mark.parametrize("ab", [(0, 0), (1, 1), (1, 0)])
def test_chain_sweeps_velocity_directions(K, monkeypatch, ab):
    """Both chains' velocity directions (L_0 = -h~^a r by the single-step launch,
    R_m = h~^b T_m r fused into the sweep) on the spinful lattice, FP64."""
    par = wl.CondParams(num_moments=17, num_random=2, vector_seed=5, alpha=ab[0], beta=ab[1],
                        gamma_mode=wl.GAMMA_FP64)
    G1 = _gamma(K, monkeypatch, SPIN, par, wl.FP64, 1)
    G4 = _gamma(K, monkeypatch, SPIN, par, wl.FP64, 4, 3)
    err = np.max(np.abs(G4 - G1)) / np.max(np.abs(G1))
    print(f"chain sweep {ab}: {err:.2e}", flush=True)
    assert err <= 1e-12


def test_chain_sweeps_split_bf16_elementwise(K, monkeypatch):
    """Split-BF16 Gamma from FP32 sweeps, element by element against the oracle
    under the GEMM bound plus the FP32 chain term (relative to B_nm, the
    magnitude sum of each element's products), and against the single-step
    FP32 chains under twice the chain term (both sides round)."""
    lat = SPIN
    M, R = 40, 2
    par = wl.CondParams(num_moments=M, num_random=R, vector_seed=7, alpha=0, beta=1,
                        gamma_mode=wl.GAMMA_SPLIT_BF16)
    (Go, B), model = ocond.cond_gamma(lat, par, with_bound=True)
    k_chunk = R * 256 * int(np.ceil(model.H.shape[0] / 256))
    bound = split_bf16_bound(k_chunk)
    idx = np.arange(M)
    chain = fp32_chain_bound(idx[:, None], idx[None, :])
    G1 = _gamma(K, monkeypatch, lat, par, wl.FP32, 1)
    for ks in (2, 3, 4):
        Gk = _gamma(K, monkeypatch, lat, par, wl.FP32, ks, 4)
        d_or = np.maximum(np.abs((Gk - Go).real), np.abs((Gk - Go).imag)) / B
        d_ss = np.maximum(np.abs((Gk - G1).real), np.abs((Gk - G1).imag)) / B
        print(f"split-bf16 KS={ks}: vs oracle worst ratio {np.max(d_or / (bound + chain)):.2f}; vs single steps "
              f"max |dG|/B {d_ss.max():.2e}", flush=True)
        assert np.all(d_or <= bound + chain)
        assert np.all(d_ss <= 2 * (bound + chain))


def test_chain_stats_bytes_drop(K, monkeypatch):
    """The sweeps move fewer chain bytes than single steps (two vectors in and
    out per KS steps plus one block row per step, against three vectors and a
    block row per step)."""
    lat = SPIN
    par = wl.CondParams(num_moments=33, num_random=2, vector_seed=3, alpha=0, beta=1, gamma_mode=wl.GAMMA_FP64)
    _gamma(K, monkeypatch, lat, par, wl.FP32, 1)
    b1 = K.cond_last_stats()["chain_bytes"]
    _gamma(K, monkeypatch, lat, par, wl.FP32, 2)
    b2 = K.cond_last_stats()["chain_bytes"]
    _gamma(K, monkeypatch, lat, par, wl.FP32, 4)
    b4 = K.cond_last_stats()["chain_bytes"]
    print(f"chain bytes: single steps {b1:.3e}, KS=2 sweeps {b2:.3e}, KS=4 sweeps {b4:.3e}", flush=True)
    assert b4 < b2 < 0.8 * b1 and b4 < 0.6 * b1
