"""The allocation-free DOS entry point (kpm_moments_dos_noalloc) against
kpm_moments_dos and the oracle.

Two calls in a row share the library's static scratch array, the second with a
smaller workload, so stale contents of the first call must not leak into the
second.  Both are compared with kpm_moments_dos on the same inputs (same
launch shape and reduction order: bit for bit) and with the FP64 oracle
(FP64: |d mu| <= 1e-6, the binding moment tolerance; FP32: the FP32
recursion bound used elsewhere, 4 (n/2) 3e-7).
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


def _case_large():
    lat, par = wl.graphene_small()   # honeycomb 64x64 + Anderson, FP64, M=256, R=4
    return lat, par


def _case_small():
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=30, L2=22, t=-2.7, anderson_w=0.8, vacancy_p=0.04, disorder_seed=77)
    par = wl.DosParams(num_moments=128, num_random=3, vector_seed=12, precision=wl.FP32)
    return lat, par


def _check(K, lat, par, out_device):
    print(f"noalloc: {wl.KIND_NAMES[lat.kind]} {lat.L1}x{lat.L2}, M={par.num_moments}, R={par.num_random}, "
          f"{'fp64' if par.precision == wl.FP64 else 'fp32'}, out_device={out_device}", flush=True)
    mu_n, mean_n = K.moments_dos_noalloc([lat], par, out_device=out_device)
    mu_r, mean_r = K.moments_dos([lat], par, out_device=out_device)
    if out_device is not None:
        import torch
        torch.cuda.synchronize()
        mu_n, mean_n, mu_r, mean_r = (x.cpu().numpy() for x in (mu_n, mean_n, mu_r, mean_r))
    assert np.array_equal(mu_n, mu_r) and np.array_equal(mean_n, mean_r)
    mu_o, _, _ = okpm.dos_moments(lat, par)
    err = float(np.max(np.abs(mu_n[0] - mu_o)))
    M = par.num_moments
    tol = 1e-6 if par.precision == wl.FP64 else 4 * (M / 2) * 3e-7
    print(f"noalloc: max |mu - mu_oracle| = {err:.3e} (tolerance {tol:.1e})", flush=True)
    assert err <= tol


def test_noalloc_two_calls_second_smaller(K):
    lat, par = _case_large()
    _check(K, lat, par, None)
    lat2, par2 = _case_small()
    _check(K, lat2, par2, None)


def test_noalloc_device_outputs_and_ldos(K):
    lat, par = _case_small()
    _check(K, lat, par, "cuda:0")
    sites = [0, 5, 2 * lat.L1 + 1]
    lat_clean = lat.replace(vacancy_p=0.0)
    par_l = par.replace(start=wl.START_SITES, sites=sites, precision=wl.FP64)
    _check(K, lat_clean, par_l, None)


def test_noalloc_rejects_oversize(K):
    lat, par = wl.graphene_small()
    big = lat.replace(L1=1024, L2=1024)   # 2M orbitals x 4 vectors x 16 B = 128 MiB per vector
    with pytest.raises(K.KPMError) as e:
        K.moments_dos_noalloc([big], par)
    assert e.value.code == K.KPM_E_INVALID and "scratch array" in str(e.value)
    # The library still works afterwards.
    _check(K, *_case_small(), None)
