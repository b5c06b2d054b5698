"""C-ABI checks that need no GPU: exported symbols, struct layouts, argument validation.

Validation errors are returned before any device call, so they run on a CPU host.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kpm.h")
LIB = os.path.join(ROOT, "paper_1910_05194_amd", "libkpm.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libkpm.so not built")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|int32_t|int64_t|const char\*)\s+(kpm_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (kpm_\w+)", out))
    assert set(names) <= exported
    # Nothing exported that the header does not declare.
    assert exported <= set(names), exported - set(names)


STRUCTS = {
    "kpm_lattice_t": "c_lattice",
    "kpm_dos_params_t": "c_dos_params",
    "kpm_tune_t": "c_tune",
    "kpm_plan_info_t": "c_plan_info",
    "kpm_cond_params_t": "c_cond_params",
    "kpm_cond_stats_t": "c_cond_stats",
    "kpm_evolve_params_t": "c_evolve_params",
    "kpm_evolve_stats_t": "c_evolve_stats",
}


def test_struct_layouts_match_binding(tmp_path):
    from paper_1910_05194_amd import kpm
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "kpm.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(kpm, pyname)
        src.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            src.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    src.append("  return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(c), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for ln in lines:
        if ln:
            parts = ln.split()
            got[(parts[0], parts[1])] = int(parts[2])
    for cname, pyname in STRUCTS.items():
        cls = getattr(kpm, pyname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)


def test_argument_validation_without_device():
    import workload as wl
    from paper_1910_05194_amd import kpm
    lat, par = wl.graphene_small()
    bad = [
        ([lat.replace(L1=1)], par, "L1, L2"),
        ([lat.replace(e_min=9.0)], par, "e_min < e_max"),
        ([lat.replace(flux=0.1)], par, "flux*L1"),
        ([lat.replace(kind=wl.SQUARE, flux=1 / 64)], par, "square"),
        ([lat.replace(rashba=0.1)], par, "Rashba"),
        ([lat.replace(e_min=-6.0, e_max=6.0)], par, "Gershgorin"),
        ([lat.replace(e_min=-3.0, e_max=12.0)], par, "Gershgorin"),
        ([lat.replace(vacancy_p=1.0)], par, "vacancy_p"),
        ([lat, lat.replace(kind=wl.SQUARE, e_min=-11.5, e_max=11.5)], par, "same kind"),
        ([lat], par.replace(num_moments=1), "num_moments"),
        ([lat], par.replace(num_random=0), "num_random"),
        ([lat], par.replace(precision=7), "precision"),
        ([lat], par.replace(start=wl.START_SITES, sites=[lat.n_orbitals]), "out of range"),
    ]
    for lats, p, msg in bad:
        for fn in (kpm.moments_dos, kpm.moments_dos_noalloc):
            with pytest.raises(kpm.KPMError) as e:
                fn(lats, p)
            assert e.value.code == kpm.KPM_E_INVALID
            assert msg in str(e.value), (fn.__name__, msg, str(e.value))
    # Bounds within a quarter of their half-width of the Gershgorin radius
    # (8.6 eV) pass validation (without a device the call then fails otherwise).
    try:
        kpm.moments_dos([lat.replace(e_min=-7.6, e_max=7.6)], par.replace(num_moments=8))
    except kpm.KPMError as e:
        assert e.code != kpm.KPM_E_INVALID, str(e)
    # The allocation-free form rejects a workspace beyond its static array
    # before touching a device: 2M orbitals x 4 complex128 vectors x 2 buffers.
    with pytest.raises(kpm.KPMError) as e:
        kpm.moments_dos_noalloc([lat.replace(L1=1024, L2=1024)], par)
    assert e.value.code == kpm.KPM_E_INVALID and "scratch array" in str(e.value), str(e.value)
    assert str(kpm.NOALLOC_SCRATCH_BYTES) in str(e.value)
    for blk in (100, 1024):
        with pytest.raises(kpm.KPMError) as e:
            kpm.Plan([lat], par, block=blk)
        assert e.value.code == kpm.KPM_E_INVALID
    for ch in (-1, 129):   # more chunks than a 256-thread honeycomb tile has lanes per sublattice
        with pytest.raises(kpm.KPMError) as e:
            kpm.Plan([lat], par, block=256, chunks=ch)
        assert e.value.code == kpm.KPM_E_INVALID and "chunks" in str(e.value)
    lat3, par3 = wl.rashba_flux(L=8, M=8, R=1)
    for p, msg in [(par3.replace(alpha=2), "alpha"), (par3.replace(gamma_mode=9), "gamma_mode")]:
        with pytest.raises(kpm.KPMError) as e:
            kpm.moments_cond(lat3, p)
        assert msg in str(e.value)
    with pytest.raises(kpm.KPMError):
        kpm.moments_cond(lat3, par3, precision=wl.FP64)   # split-BF16 needs FP32 blocks
    import numpy as np
    with pytest.raises(kpm.KPMError):
        kpm.reconstruct_jackson(np.zeros(0), np.zeros(4), -1.0, 1.0)
    with pytest.raises(kpm.KPMError):
        kpm.reconstruct_jackson(np.ones(4), np.zeros(4), 1.0, -1.0)
    for bad in (0.0, -0.1):
        with pytest.raises(kpm.KPMError):
            kpm.reconstruct_cpgf(np.ones(4), np.zeros(4), -1.0, 1.0, bad)
        with pytest.raises(kpm.KPMError):
            kpm.reconstruct_lorentz(np.ones(4), np.zeros(4), -1.0, 1.0, bad)
    with pytest.raises(kpm.KPMError):
        kpm.bandwidth_probe(7, 1 << 20)
    for kw in (dict(n0=7, count=4), dict(n0=-1, count=2), dict(kernel=1, lam=-1.0), dict(kernel=2)):
        with pytest.raises(kpm.KPMError) as e:
            kpm.kernel_factors(8, **kw)
        assert e.value.code == kpm.KPM_E_INVALID
    with pytest.raises(kpm.KPMError):
        kpm.MLP(0, 16, 16)
    # The acceptance measures reject NULL handles and arrays before touching a device.
    assert kpm.LIB.kpm_mlp_noise_z(None, None, None, None, None, 1, 1, 0, None, None) == kpm.KPM_E_INVALID
    assert kpm.LIB.kpm_mlp_rel_error(None, None, None, None, 1, 1, 0, None, None) == kpm.KPM_E_INVALID
    psi = np.zeros((1, lat.n_orbitals), dtype=np.complex128)
    for args, msg in (((1.0, 1, 3), "num_moments"), ((0.0, 40, 3), "dt"), ((1.0, 40, 0), "num_points")):
        with pytest.raises(kpm.KPMError) as e:
            kpm.time_evolve(lat, psi, *args)
        assert e.value.code == kpm.KPM_E_INVALID and msg in str(e.value), str(e.value)
    with pytest.raises(kpm.KPMError) as e:
        kpm.wavepacket_gaussian(lat, [[0.0, 0.0]], [[1.0, 1.0]], -1.0, [0, 0])
    assert "width" in str(e.value)
    G = np.zeros((8, 8), dtype=np.complex128)
    with pytest.raises(kpm.KPMError) as e:
        kpm.reconstruct_sigma_bastin(G, np.zeros(2), -1.0, 1.0, 0.1, 1.0, kT=-0.01)
    assert "kT" in str(e.value)
    with pytest.raises(kpm.KPMError) as e:
        kpm.reconstruct_sigma_optical(G, np.zeros(8), np.array([0.5]), 0.0, -1.0, 1.0, 0.1, 1.0, kT=-0.01)
    assert "kT" in str(e.value)
    assert kpm.last_error() != ""


def test_fault_injection_hook_without_device():
    """kpm_debug_inject_failure: argument checks, arming and disarming; a call that
    fails validation returns before any checked HIP operation, so nothing fires."""
    from paper_1910_05194_amd import kpm
    assert kpm.debug_live_allocations() >= 0
    for nth, kind in ((-1, 0), (1, 2), (1, -1)):
        with pytest.raises(kpm.KPMError) as e:
            kpm.debug_inject_failure(nth, kind)
        assert e.value.code == kpm.KPM_E_INVALID
    assert kpm.debug_inject_failure(0, 0) == 0
    assert kpm.debug_inject_failure(3, 1) == 0
    with pytest.raises(kpm.KPMError) as e:
        kpm.kernel_factors(8, n0=7, count=4)
    assert e.value.code == kpm.KPM_E_INVALID
    assert kpm.debug_inject_failure(0, 0) == 0


def test_traffic_record_matches_kernel_sources():
    """The HBM-traffic record that bench.py reports beside the step kernel's
    roofline was taken on the committed kernel sources (a record counts only
    for the sources whose SHA-256 it names), for the benchmarked workload and
    both launch shapes the autotuner chooses between, with a calibration
    factor from the plain copy."""
    import importlib.util
    import json
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    with open(os.path.join(root, "profiles", "step_kernel_traffic.json")) as fh:
        rec = json.load(fh)
    sha = bench.step_kernel_source_hash()
    launches = {tuple(r["launch"]) for r in rec["records"] if r["source_sha256"] == sha and r["workload"] == [4096, 32]}
    assert {(5, 512, 256, 1024, 8), (5, 512, 128, 2048, 8)} <= launches
    for r in rec["records"]:
        assert 1.0 <= r["hbm_bytes_per_launch"] / r["algorithmic_bytes_per_launch"] < 1.2
        assert abs(r["calibration"]["fetch_factor"] - 2.0) < 0.01 and abs(r["calibration"]["write_factor"] - 1.0) < 0.01
