"""Thin ctypes binding of libkpm (include/kpm.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  If libkpm.so is missing the import of this module raises; there is
no CPU fallback.  Device outputs are torch tensors (torch supplies device
memory and streams); host outputs are numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkpm.so")

KPM_OK = 0
KPM_E_INVALID = -1
KPM_E_NOMEM = -2
KPM_E_DEVICE = -3
KPM_E_SPECTRUM = -4
KPM_E_UNSUPPORTED = -5

HONEYCOMB, HONEYCOMB_SPIN, SQUARE = 0, 1, 2
FP32, FP64 = 0, 1
START_RANDOM_PHASE, START_SITES = 0, 1
GAMMA_FP64, GAMMA_FP32, GAMMA_SPLIT_BF16 = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 64 << 20   # KPM_NOALLOC_SCRATCH_BYTES


class KPMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libkpm error {code}: {msg}")
        self.code = code


class c_lattice(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("L1", ctypes.c_int32), ("L2", ctypes.c_int32),
                ("t", ctypes.c_double), ("rashba", ctypes.c_double), ("flux", ctypes.c_double),
                ("anderson_w", ctypes.c_double), ("vacancy_p", ctypes.c_double),
                ("disorder_seed", ctypes.c_uint64), ("e_min", ctypes.c_double), ("e_max", ctypes.c_double),
                ("exchange", ctypes.c_double)]


class c_dos_params(ctypes.Structure):
    _fields_ = [("num_moments", ctypes.c_int32), ("num_random", ctypes.c_int32),
                ("vector_seed", ctypes.c_uint64), ("precision", ctypes.c_int32), ("start", ctypes.c_int32),
                ("sites", ctypes.POINTER(ctypes.c_int64)), ("num_sites", ctypes.c_int32)]


class c_cond_params(ctypes.Structure):
    _fields_ = [("num_moments", ctypes.c_int32), ("num_random", ctypes.c_int32),
                ("vector_seed", ctypes.c_uint64), ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("gamma_mode", ctypes.c_int32), ("precision", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class c_evolve_params(ctypes.Structure):
    _fields_ = [("num_moments", ctypes.c_int32), ("num_points", ctypes.c_int32), ("num_packets", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("dt_fs", ctypes.c_double)]


class c_evolve_stats(ctypes.Structure):
    _fields_ = [("history", ctypes.c_int32), ("time_steps", ctypes.c_int32), ("loop_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class c_cond_stats(ctypes.Structure):
    _fields_ = [("n_batches", ctypes.c_int32), ("vectors_per_batch", ctypes.c_int32), ("chain_ms", ctypes.c_double),
                ("gemm_ms", ctypes.c_double), ("total_ms", ctypes.c_double), ("chain_bytes", ctypes.c_double),
                ("gemm_useful_flops", ctypes.c_double), ("gemm_mfma_flops", ctypes.c_double),
                ("gemm_operand_bytes", ctypes.c_double)]


class c_tune(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("rows", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("kernel", ctypes.c_int32), ("chunks", ctypes.c_int32)]


class c_plan_info(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("n_tiles", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("block", ctypes.c_int32), ("rows", ctypes.c_int32), ("tile_cells_x", ctypes.c_int32),
                ("r_padded", ctypes.c_int32), ("kernel", ctypes.c_int32), ("n_orbitals", ctypes.c_int64), ("bytes_per_step", ctypes.c_double),
                ("last_loop_ms", ctypes.c_double), ("last_run_ms", ctypes.c_double),
                ("n_active_total", ctypes.c_int64), ("tile_chunks", ctypes.c_int32)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1910_05194_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "kpm_version": (ctypes.c_int, []),
        "kpm_last_error": (ctypes.c_char_p, []),
        "kpm_moments_dos": (ctypes.c_int, [ctypes.POINTER(c_lattice), ctypes.c_int32, ctypes.POINTER(c_dos_params),
                                           _P, _P, ctypes.c_int32, _P]),
        "kpm_moments_dos_noalloc": (ctypes.c_int, [ctypes.POINTER(c_lattice), ctypes.c_int32,
                                                   ctypes.POINTER(c_dos_params), _P, _P, ctypes.c_int32, _P]),
        "kpm_plan_create": (ctypes.c_int, [ctypes.POINTER(c_lattice), ctypes.c_int32, ctypes.POINTER(c_dos_params),
                                           ctypes.POINTER(c_tune), ctypes.POINTER(_P)]),
        "kpm_plan_run": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P]),
        "kpm_plan_info": (ctypes.c_int, [_P, ctypes.POINTER(c_plan_info)]),
        "kpm_plan_destroy": (ctypes.c_int, [_P]),
        "kpm_reconstruct_jackson": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_double,
                                                   ctypes.c_double, _P, ctypes.c_int32, _P]),
        "kpm_reconstruct_lorentz": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_double,
                                                   ctypes.c_double, ctypes.c_double, _P, ctypes.c_int32, _P]),
        "kpm_reconstruct_cpgf": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_double, _P, _P, ctypes.c_int32, _P]),
        "kpm_moments_cond": (ctypes.c_int, [ctypes.POINTER(c_lattice), ctypes.POINTER(c_cond_params), _P,
                                            ctypes.c_int32, _P]),
        "kpm_reconstruct_sigma": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_double, _P, ctypes.c_int32, _P]),
        "kpm_reconstruct_sigma_bastin": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_double,
                                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                        ctypes.c_double, ctypes.c_int32, _P, ctypes.c_int32, _P]),
        "kpm_reconstruct_sigma_optical": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_int32,
                                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                         ctypes.c_int32, _P, ctypes.c_int32, _P]),
        "kpm_mlp_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                          ctypes.POINTER(_P)]),
        "kpm_mlp_destroy": (ctypes.c_int, [_P]),
        "kpm_mlp_num_params": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
        "kpm_mlp_get_params": (ctypes.c_int, [_P, _P]),
        "kpm_mlp_set_params": (ctypes.c_int, [_P, _P]),
        "kpm_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P]),
        "kpm_mlp_train_step": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_float, _P, _P]),
        "kpm_mlp_gradients": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, _P, _D, _P]),
        "kpm_mlp_fit_scaling": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P]),
        "kpm_mlp_rel_error": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P]),
        "kpm_mlp_noise_z": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                                           _P]),
        "kpm_mlp_eval_loss": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
        "kpm_kernel_factors": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                              ctypes.c_int32, _P, ctypes.c_int32, _P]),
        "kpm_cond_last_stats": (ctypes.c_int, [ctypes.POINTER(c_cond_stats)]),
        "kpm_moments_gamma1": (ctypes.c_int, [ctypes.POINTER(c_lattice), ctypes.POINTER(c_cond_params), _P,
                                              ctypes.c_int32, _P]),
        "kpm_sigma_singleshot": (ctypes.c_int, [ctypes.POINTER(c_lattice), ctypes.POINTER(c_cond_params), _P,
                                                ctypes.c_int32, ctypes.c_double, _P, ctypes.c_int32, _P]),
        "kpm_wavepacket_gaussian": (ctypes.c_int, [ctypes.POINTER(c_lattice), ctypes.c_int32, _P, _P, ctypes.c_double,
                                                   _P, _P, ctypes.c_int32, _P]),
        "kpm_time_evolve": (ctypes.c_int, [ctypes.POINTER(c_lattice), ctypes.POINTER(c_evolve_params), _P, _P,
                                           ctypes.c_int32, _P]),
        "kpm_evolve_last_stats": (ctypes.c_int, [ctypes.POINTER(c_evolve_stats)]),
        "kpm_autotune": (ctypes.c_int, [ctypes.POINTER(c_lattice), ctypes.c_int32, ctypes.POINTER(c_dos_params),
                                        ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(c_tune), _D, _P]),
        "kpm_bandwidth_probe": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.c_int32, _P, _D, _D]),
        "kpm_debug_inject_failure": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32]),
        "kpm_debug_live_allocations": (ctypes.c_int64, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def _check(code: int):
    if code != KPM_OK:
        raise KPMError(code, LIB.kpm_last_error().decode(errors="replace"))


def debug_inject_failure(nth: int, kind: int = 0) -> int:
    """Arm the library's fault countdown (kpm_debug_inject_failure): the nth checked
    HIP operation from now on fails (kind 0: out of memory, 1: launch failure);
    nth = 0 disarms.  Returns how many failures fired since the previous call."""
    r = int(LIB.kpm_debug_inject_failure(int(nth), int(kind)))
    if r < 0:
        _check(r)
    return r


def debug_live_allocations() -> int:
    """Device buffers the library holds right now (kpm_debug_live_allocations)."""
    return int(LIB.kpm_debug_live_allocations())


def last_error() -> str:
    return LIB.kpm_last_error().decode(errors="replace")


def c_lattices(lattices) -> ctypes.Array:
    arr = (c_lattice * len(lattices))()
    for i, L in enumerate(lattices):
        arr[i] = c_lattice(int(L.kind), int(L.L1), int(L.L2), float(L.t), float(getattr(L, "rashba", 0.0)),
                           float(getattr(L, "flux", 0.0)), float(getattr(L, "anderson_w", 0.0)),
                           float(getattr(L, "vacancy_p", 0.0)), int(getattr(L, "disorder_seed", 0)) & (2**64 - 1),
                           float(L.e_min), float(L.e_max), float(getattr(L, "exchange", 0.0)))
    return arr


def c_params(par):
    sites = getattr(par, "sites", None)
    start = int(getattr(par, "start", START_RANDOM_PHASE))
    keep = None
    p = c_dos_params()
    p.num_moments = int(par.num_moments)
    p.num_random = int(par.num_random)
    p.vector_seed = int(par.vector_seed) & (2**64 - 1)
    p.precision = int(par.precision)
    p.start = start
    if start == START_SITES and sites is not None:
        keep = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
        p.sites = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        p.num_sites = int(keep.size)
    return p, keep


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


def _num_vectors(par) -> int:
    if int(getattr(par, "start", START_RANDOM_PHASE)) == START_SITES:
        return len(par.sites)
    return int(par.num_random)


def moments_dos(lattices: Sequence, par, out_device=None, stream=None):
    """kpm_moments_dos.  Returns (mu_per_vector [n_lat, R, M], mu_mean [n_lat, M]).

    out_device=None -> numpy arrays (host outputs); otherwise a torch device
    (e.g. "cuda:0") on which torch float64 tensors are allocated and filled.
    """
    return _moments_dos(LIB.kpm_moments_dos, lattices, par, out_device, stream)


def moments_dos_noalloc(lattices: Sequence, par, out_device=None, stream=None):
    """kpm_moments_dos_noalloc: kpm_moments_dos with its workspace in the
    library's static device array (no device allocation inside the call).
    Arguments and results as moments_dos; the caller's output tensors are
    allocated here, outside the library call."""
    return _moments_dos(LIB.kpm_moments_dos_noalloc, lattices, par, out_device, stream)


def _moments_dos(fn, lattices: Sequence, par, out_device, stream):
    lats = c_lattices(lattices)
    p, keep = c_params(par)
    R = _num_vectors(par)
    shape_pv = (len(lattices), R, int(par.num_moments))
    shape_mean = (len(lattices), int(par.num_moments))
    if out_device is None:
        mu = np.zeros(shape_pv)
        mean = np.zeros(shape_mean)
        code = fn(lats, len(lattices), ctypes.byref(p), mu.ctypes.data, mean.ctypes.data, 0, _stream_handle(stream))
    else:
        import torch
        mu = torch.zeros(shape_pv, dtype=torch.float64, device=out_device)
        mean = torch.zeros(shape_mean, dtype=torch.float64, device=out_device)
        if stream is None:
            stream = torch.cuda.current_stream(mu.device)
        code = fn(lats, len(lattices), ctypes.byref(p), mu.data_ptr(), mean.data_ptr(), 1, _stream_handle(stream))
    del keep
    _check(code)
    return mu, mean


class Plan:
    """kpm_plan_*: a reusable, graph-captured DOS/LDOS moment pipeline."""

    def __init__(self, lattices: Sequence, par, block: int = 0, rows: int = 0, grid: int = 0,
                 use_graph: bool = True, kernel: int = 0, chunks: int = 0):
        self.n_lat = len(lattices)
        self.R = _num_vectors(par)
        self.M = int(par.num_moments)
        lats = c_lattices(lattices)
        p, keep = c_params(par)
        tune = c_tune(int(block), int(rows), int(grid), 1 if use_graph else 0, int(kernel), int(chunks))
        h = _P()
        _check(LIB.kpm_plan_create(lats, self.n_lat, ctypes.byref(p), ctypes.byref(tune), ctypes.byref(h)))
        del keep
        self._h = h

    def run(self, mu_per_vector=None, mu_mean=None, stream=None, check: bool = True):
        """Run the plan.  Outputs are torch device tensors (float64) or numpy arrays."""
        import torch
        on_dev = None
        ptrs = []
        for t in (mu_per_vector, mu_mean):
            if t is None:
                ptrs.append(None)
            elif isinstance(t, np.ndarray):
                assert t.dtype == np.float64 and t.flags.c_contiguous
                ptrs.append(t.ctypes.data)
                on_dev = 0 if on_dev is None else on_dev
                assert on_dev == 0, "outputs must all be host or all be device"
            else:
                assert t.dtype == torch.float64 and t.is_contiguous()
                ptrs.append(t.data_ptr())
                on_dev = 1 if on_dev is None else on_dev
                assert on_dev == 1, "outputs must all be host or all be device"
                if stream is None:
                    stream = torch.cuda.current_stream(t.device)
        code = LIB.kpm_plan_run(self._h, ptrs[0], ptrs[1], on_dev or 0, _stream_handle(stream))
        if check:
            _check(code)
        return code

    def info(self) -> dict:
        i = c_plan_info()
        _check(LIB.kpm_plan_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in c_plan_info._fields_}

    def close(self):
        if getattr(self, "_h", None):
            LIB.kpm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reconstruct_jackson(mu, energies, e_min: float, e_max: float, stream=None):
    """kpm_reconstruct_jackson on host numpy arrays or device torch tensors."""
    if isinstance(mu, np.ndarray):
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        en = np.ascontiguousarray(energies, dtype=np.float64)
        rho = np.zeros(en.shape)
        _check(LIB.kpm_reconstruct_jackson(mu.ctypes.data, mu.size, en.ctypes.data, en.size, float(e_min),
                                           float(e_max), rho.ctypes.data, 0, _stream_handle(stream)))
        return rho
    import torch
    mu = mu.contiguous().to(torch.float64)
    en = energies.contiguous().to(torch.float64)
    rho = torch.zeros_like(en)
    if stream is None:
        stream = torch.cuda.current_stream(mu.device)
    _check(LIB.kpm_reconstruct_jackson(mu.data_ptr(), mu.numel(), en.data_ptr(), en.numel(), float(e_min),
                                       float(e_max), rho.data_ptr(), 1, _stream_handle(stream)))
    return rho


def kernel_factors(M: int, n0: int = 0, count: Optional[int] = None, kernel: int = 0, lam: float = 0.0,
                   out_device=None, stream=None):
    """kpm_kernel_factors: damping factors g_n0 .. g_(n0+count-1) of an M-moment expansion
    (kernel 0 = Jackson, 1 = Lorentz with lam); numpy array, or a float64 tensor on out_device."""
    count = M - n0 if count is None else count
    if out_device is None:
        g = np.zeros(count)
        _check(LIB.kpm_kernel_factors(int(kernel), int(M), float(lam), int(n0), int(count), g.ctypes.data, 0,
                                      _stream_handle(stream)))
        return g
    import torch
    g = torch.zeros(count, dtype=torch.float64, device=out_device)
    if stream is None:
        stream = torch.cuda.current_stream(g.device)
    _check(LIB.kpm_kernel_factors(int(kernel), int(M), float(lam), int(n0), int(count), g.data_ptr(), 1,
                                  _stream_handle(stream)))
    return g


def reconstruct_lorentz(mu, energies, e_min: float, e_max: float, lam: float, stream=None):
    """kpm_reconstruct_lorentz on host numpy arrays or device torch tensors."""
    if isinstance(mu, np.ndarray):
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        en = np.ascontiguousarray(energies, dtype=np.float64)
        rho = np.zeros(en.shape)
        _check(LIB.kpm_reconstruct_lorentz(mu.ctypes.data, mu.size, en.ctypes.data, en.size, float(e_min),
                                           float(e_max), float(lam), rho.ctypes.data, 0, _stream_handle(stream)))
        return rho
    import torch
    mu = mu.contiguous().to(torch.float64)
    en = energies.contiguous().to(torch.float64)
    rho = torch.zeros_like(en)
    if stream is None:
        stream = torch.cuda.current_stream(mu.device)
    _check(LIB.kpm_reconstruct_lorentz(mu.data_ptr(), mu.numel(), en.data_ptr(), en.numel(), float(e_min),
                                       float(e_max), float(lam), rho.data_ptr(), 1, _stream_handle(stream)))
    return rho


def reconstruct_cpgf(mu, energies, e_min: float, e_max: float, eta: float, green: bool = False, stream=None):
    """kpm_reconstruct_cpgf: rho [K] (and the complex traced resolvent [K] if green)
    on host numpy arrays or device torch tensors."""
    if isinstance(mu, np.ndarray):
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        en = np.ascontiguousarray(energies, dtype=np.float64)
        rho = np.zeros(en.shape)
        g = np.zeros(en.shape + (2,)) if green else None
        _check(LIB.kpm_reconstruct_cpgf(mu.ctypes.data, mu.size, en.ctypes.data, en.size, float(e_min),
                                        float(e_max), float(eta), rho.ctypes.data, g.ctypes.data if green else None,
                                        0, _stream_handle(stream)))
        return (rho, g[..., 0] + 1j * g[..., 1]) if green else rho
    import torch
    mu = mu.contiguous().to(torch.float64)
    en = energies.contiguous().to(torch.float64)
    rho = torch.zeros_like(en)
    g = torch.zeros(en.shape + (2,), dtype=torch.float64, device=en.device) if green else None
    if stream is None:
        stream = torch.cuda.current_stream(mu.device)
    _check(LIB.kpm_reconstruct_cpgf(mu.data_ptr(), mu.numel(), en.data_ptr(), en.numel(), float(e_min),
                                    float(e_max), float(eta), rho.data_ptr(), g.data_ptr() if green else None, 1,
                                    _stream_handle(stream)))
    return (rho, torch.view_as_complex(g)) if green else rho


def bandwidth_probe(pattern: int, bytes_per_array: int, iters: int = 10, grid: int = 4096, block: int = 256,
                    nontemporal: bool = False, stream=None) -> dict:
    """kpm_bandwidth_probe: returns {"ms": ..., "bytes": ..., "GBs": ...} per launch."""
    ms = ctypes.c_double()
    nb = ctypes.c_double()
    _check(LIB.kpm_bandwidth_probe(int(pattern), int(bytes_per_array), int(iters), int(grid), int(block),
                                   1 if nontemporal else 0, _stream_handle(stream), ctypes.byref(ms),
                                   ctypes.byref(nb)))
    return {"ms": ms.value, "bytes": nb.value, "GBs": nb.value / (ms.value * 1e-3) / 1e9}


def moments_cond(lattice, par, precision: int = FP32, max_batch: int = 0, out_device=None, stream=None):
    """kpm_moments_cond: Gamma_nm as a complex array [M, M] (numpy) or a float64 [M, M, 2] torch tensor."""
    lat = c_lattices([lattice])
    p = c_cond_params(int(par.num_moments), int(par.num_random), int(par.vector_seed) & (2**64 - 1),
                      int(par.alpha), int(par.beta), int(par.gamma_mode), int(precision), int(max_batch))
    M = int(par.num_moments)
    if out_device is None:
        g = np.zeros((M, M, 2))
        _check(LIB.kpm_moments_cond(lat, ctypes.byref(p), g.ctypes.data, 0, _stream_handle(stream)))
        return g[..., 0] + 1j * g[..., 1]
    import torch
    g = torch.zeros((M, M, 2), dtype=torch.float64, device=out_device)
    if stream is None:
        stream = torch.cuda.current_stream(g.device)
    _check(LIB.kpm_moments_cond(lat, ctypes.byref(p), g.data_ptr(), 1, _stream_handle(stream)))
    return g


def moments_gamma1(lattice, par, precision: int = FP32, out_device=None, stream=None):
    """kpm_moments_gamma1: Gamma_n^{ab} as a complex array [M] (numpy) or a float64 [M, 2] torch tensor."""
    lat = c_lattices([lattice])
    p = c_cond_params(int(par.num_moments), int(par.num_random), int(par.vector_seed) & (2**64 - 1),
                      int(par.alpha), int(par.beta), int(par.gamma_mode), int(precision), 0)
    M = int(par.num_moments)
    if out_device is None:
        g = np.zeros((M, 2))
        _check(LIB.kpm_moments_gamma1(lat, ctypes.byref(p), g.ctypes.data, 0, _stream_handle(stream)))
        return g[:, 0] + 1j * g[:, 1]
    import torch
    g = torch.zeros((M, 2), dtype=torch.float64, device=out_device)
    if stream is None:
        stream = torch.cuda.current_stream(g.device)
    _check(LIB.kpm_moments_gamma1(lat, ctypes.byref(p), g.data_ptr(), 1, _stream_handle(stream)))
    return g


def sigma_singleshot(lattice, par, energies, eta: float, precision: int = FP32, stream=None):
    """kpm_sigma_singleshot: sigma_ab(E) in e^2/h (T = 0, CPGF broadening eta in eV) for
    energies as a numpy array (host result) or a float64 torch tensor (device result)."""
    lat = c_lattices([lattice])
    p = c_cond_params(int(par.num_moments), int(par.num_random), int(par.vector_seed) & (2**64 - 1),
                      int(par.alpha), int(par.beta), int(par.gamma_mode), int(precision), 0)
    if isinstance(energies, np.ndarray) or not hasattr(energies, "data_ptr"):
        en = np.ascontiguousarray(np.atleast_1d(energies), dtype=np.float64)
        out = np.zeros(en.shape)
        _check(LIB.kpm_sigma_singleshot(lat, ctypes.byref(p), en.ctypes.data, en.size, float(eta), out.ctypes.data, 0,
                                        _stream_handle(stream)))
        return out
    import torch
    en = energies.contiguous().to(torch.float64)
    out = torch.zeros_like(en)
    if stream is None:
        stream = torch.cuda.current_stream(en.device)
    _check(LIB.kpm_sigma_singleshot(lat, ctypes.byref(p), en.data_ptr(), en.numel(), float(eta), out.data_ptr(), 1,
                                    _stream_handle(stream)))
    return out


def wavepacket_gaussian(lattice, k_vectors, spinors, width_nm: float, center_cells, out_device=None, stream=None):
    """kpm_wavepacket_gaussian: the normalised Gaussian packet as complex numpy [n_orbitals]
    (host) or float64 torch [n_orbitals, 2] on ``out_device``.  k_vectors [n_k, 2] (1/nm),
    spinors [n_k, orbitals per cell] complex, center_cells (c1, c2)."""
    lat = c_lattices([lattice])
    kv = np.ascontiguousarray(np.atleast_2d(k_vectors), dtype=np.float64)
    sp = np.atleast_2d(np.asarray(spinors, dtype=np.complex128))
    spr = np.ascontiguousarray(np.stack([sp.real, sp.imag], axis=-1))
    cc = np.ascontiguousarray(center_cells, dtype=np.float64)
    n = int(lattice.L1) * int(lattice.L2) * {0: 2, 1: 4, 2: 1}.get(int(lattice.kind), 2)
    if out_device is None:
        out = np.zeros((n, 2))
        _check(LIB.kpm_wavepacket_gaussian(lat, kv.shape[0], kv.ctypes.data, spr.ctypes.data, float(width_nm),
                                           cc.ctypes.data, out.ctypes.data, 0, _stream_handle(stream)))
        return out[:, 0] + 1j * out[:, 1]
    import torch
    out = torch.zeros((n, 2), dtype=torch.float64, device=out_device)
    if stream is None:
        stream = torch.cuda.current_stream(out.device)
    _check(LIB.kpm_wavepacket_gaussian(lat, kv.shape[0], kv.ctypes.data, spr.ctypes.data, float(width_nm),
                                       cc.ctypes.data, out.data_ptr(), 1, _stream_handle(stream)))
    return out


def time_evolve(lattice, psi0, dt_fs: float, num_moments: int, num_points: int, precision: int = FP32, stream=None):
    """kpm_time_evolve: (psi at t = (num_points - 1) dt, observables [num_points, R, 8]).
    psi0: complex numpy [R, n_orbitals] or [n_orbitals] (host results), or float64 torch
    [R, n_orbitals, 2] on the device (device results, psi0 left unchanged)."""
    lat = c_lattices([lattice])
    if isinstance(psi0, np.ndarray):
        p0 = np.atleast_2d(np.asarray(psi0, dtype=np.complex128))
        R = p0.shape[0]
        buf = np.ascontiguousarray(np.stack([p0.real, p0.imag], axis=-1))
        obs = np.zeros((int(num_points), R, 8))
        par = c_evolve_params(int(num_moments), int(num_points), R, int(precision), float(dt_fs))
        _check(LIB.kpm_time_evolve(lat, ctypes.byref(par), buf.ctypes.data, obs.ctypes.data, 0,
                                   _stream_handle(stream)))
        out = buf[..., 0] + 1j * buf[..., 1]
        return (out[0] if np.ndim(psi0) == 1 else out), obs
    import torch
    buf = psi0.detach().to(torch.float64).contiguous().clone()
    if buf.dim() == 2:
        buf = buf.unsqueeze(0)
    R = buf.shape[0]
    obs = torch.zeros((int(num_points), R, 8), dtype=torch.float64, device=buf.device)
    if stream is None:
        stream = torch.cuda.current_stream(buf.device)
    par = c_evolve_params(int(num_moments), int(num_points), R, int(precision), float(dt_fs))
    _check(LIB.kpm_time_evolve(lat, ctypes.byref(par), buf.data_ptr(), obs.data_ptr(), 1, _stream_handle(stream)))
    return buf, obs


def evolve_last_stats() -> dict:
    """kpm_evolve_last_stats of the calling thread."""
    st = c_evolve_stats()
    _check(LIB.kpm_evolve_last_stats(ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in c_evolve_stats._fields_}


def cond_last_stats() -> dict:
    """kpm_cond_last_stats of the calling thread."""
    st = c_cond_stats()
    _check(LIB.kpm_cond_last_stats(ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in c_cond_stats._fields_}


def reconstruct_sigma(gamma, energies, e_min: float, e_max: float, orbitals_per_nm2: float, stream=None):
    """kpm_reconstruct_sigma: sigma_xx(E) in e^2/h from Gamma ([M, M] complex numpy or [M, M, 2] torch)."""
    if isinstance(gamma, np.ndarray):
        g = np.ascontiguousarray(np.stack([gamma.real, gamma.imag], axis=-1)) if np.iscomplexobj(gamma) else \
            np.ascontiguousarray(gamma, dtype=np.float64)
        en = np.ascontiguousarray(energies, dtype=np.float64)
        out = np.zeros(en.shape)
        _check(LIB.kpm_reconstruct_sigma(g.ctypes.data, g.shape[0], en.ctypes.data, en.size, float(e_min),
                                         float(e_max), float(orbitals_per_nm2), out.ctypes.data, 0,
                                         _stream_handle(stream)))
        return out
    import torch
    g = gamma.contiguous()
    en = energies.contiguous().to(torch.float64)
    out = torch.zeros_like(en)
    if stream is None:
        stream = torch.cuda.current_stream(g.device)
    _check(LIB.kpm_reconstruct_sigma(g.data_ptr(), g.shape[0], en.data_ptr(), en.numel(), float(e_min),
                                     float(e_max), float(orbitals_per_nm2), out.data_ptr(), 1,
                                     _stream_handle(stream)))
    return out


def reconstruct_sigma_bastin(gamma, energies, e_min: float, e_max: float, eta: float, orbitals_per_nm2: float,
                             n_theta: int = 0, stream=None, kT: float = 0.0):
    """kpm_reconstruct_sigma_bastin: Kubo-Bastin sigma_ab(mu) in e^2/h from Gamma^{ab}
    ([M, M] complex numpy or [M, M, 2] float64 torch on the device) at chemical potentials
    ``energies`` and temperature kT; eta and kT in eV."""
    if isinstance(gamma, np.ndarray):
        g = np.ascontiguousarray(np.stack([gamma.real, gamma.imag], axis=-1)) if np.iscomplexobj(gamma) else \
            np.ascontiguousarray(gamma, dtype=np.float64)
        en = np.ascontiguousarray(np.atleast_1d(energies), dtype=np.float64)
        out = np.zeros(en.shape)
        _check(LIB.kpm_reconstruct_sigma_bastin(g.ctypes.data, g.shape[0], en.ctypes.data, en.size, float(e_min),
                                                float(e_max), float(eta), float(kT), float(orbitals_per_nm2),
                                                int(n_theta), out.ctypes.data, 0, _stream_handle(stream)))
        return out
    import torch
    g = gamma.contiguous()
    en = energies.contiguous().to(torch.float64)
    out = torch.zeros_like(en)
    if stream is None:
        stream = torch.cuda.current_stream(g.device)
    _check(LIB.kpm_reconstruct_sigma_bastin(g.data_ptr(), g.shape[0], en.data_ptr(), en.numel(), float(e_min),
                                            float(e_max), float(eta), float(kT), float(orbitals_per_nm2),
                                            int(n_theta), out.data_ptr(), 1, _stream_handle(stream)))
    return out


def reconstruct_sigma_optical(gamma_nm, gamma_n, omegas, mu: float, e_min: float, e_max: float, eta: float,
                              orbitals_per_nm2: float, n_theta: int = 0, stream=None, kT: float = 0.0):
    """kpm_reconstruct_sigma_optical: complex sigma_ab(omega) in e^2/h (chemical potential mu and
    temperature kT in eV) from the rank-2 and rank-1 Gamma (numpy complex [M, M] and [M], or float64
    torch [M, M, 2] and [M, 2])."""
    if isinstance(gamma_nm, np.ndarray):
        g2 = np.ascontiguousarray(np.stack([gamma_nm.real, gamma_nm.imag], axis=-1), dtype=np.float64)
        g1 = np.ascontiguousarray(np.stack([np.real(gamma_n), np.imag(gamma_n)], axis=-1), dtype=np.float64)
        om = np.ascontiguousarray(np.atleast_1d(omegas), dtype=np.float64)
        out = np.zeros((om.size, 2))
        _check(LIB.kpm_reconstruct_sigma_optical(g2.ctypes.data, g1.ctypes.data, g2.shape[0], om.ctypes.data, om.size,
                                                 float(mu), float(e_min), float(e_max), float(eta), float(kT),
                                                 float(orbitals_per_nm2), int(n_theta), out.ctypes.data, 0,
                                                 _stream_handle(stream)))
        return out[:, 0] + 1j * out[:, 1]
    import torch
    g2 = gamma_nm.contiguous()
    g1 = gamma_n.contiguous()
    om = omegas.contiguous().to(torch.float64)
    out = torch.zeros((om.numel(), 2), dtype=torch.float64, device=g2.device)
    if stream is None:
        stream = torch.cuda.current_stream(g2.device)
    _check(LIB.kpm_reconstruct_sigma_optical(g2.data_ptr(), g1.data_ptr(), g2.shape[0], om.data_ptr(), om.numel(),
                                             float(mu), float(e_min), float(e_max), float(eta), float(kT),
                                             float(orbitals_per_nm2), int(n_theta), out.data_ptr(), 1,
                                             _stream_handle(stream)))
    return out


class MLP:
    """kpm_mlp_*: the moment-extrapolation network (device-resident FP32 parameters)."""

    def __init__(self, n_in: int = 256, n_hidden: int = 1024, n_out: int = 1792, seed: int = 7):
        self.n_in, self.n_hidden, self.n_out = n_in, n_hidden, n_out
        h = _P()
        _check(LIB.kpm_mlp_create(n_in, n_hidden, n_out, int(seed) & (2**64 - 1), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        _check(LIB.kpm_mlp_num_params(h, ctypes.byref(n)))
        self.n_params = n.value

    def shapes(self):
        i, h, o = self.n_in, self.n_hidden, self.n_out
        return [(i, h), (h,), (h, h), (h,), (h, o), (o,)]

    def get_params(self):
        flat = np.zeros(self.n_params, dtype=np.float32)
        _check(LIB.kpm_mlp_get_params(self._h, flat.ctypes.data))
        return self._unpack(flat)

    def set_params(self, params):
        flat = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.float32).ravel() for p in params]))
        assert flat.size == self.n_params
        _check(LIB.kpm_mlp_set_params(self._h, flat.ctypes.data))

    def _unpack(self, flat):
        out, o = [], 0
        for shp in self.shapes():
            n = int(np.prod(shp))
            out.append(flat[o:o + n].reshape(shp))
            o += n
        return out

    def forward(self, x, bf16: bool = False, stream=None):
        import torch
        x = x.contiguous()
        assert x.dtype == torch.float32 and x.shape[1] == self.n_in
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=x.device)
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        _check(LIB.kpm_mlp_forward(self._h, x.data_ptr(), x.shape[0], y.data_ptr(), 1 if bf16 else 0,
                                   _stream_handle(stream)))
        return y

    def train_step(self, x, target, weights, lr: float, loss_out=None, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        _check(LIB.kpm_mlp_train_step(self._h, x.data_ptr(), target.data_ptr(), weights.data_ptr(), x.shape[0],
                                      float(lr), None if loss_out is None else loss_out.data_ptr(),
                                      _stream_handle(stream)))

    def gradients(self, x, target, weights, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        flat = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_double()
        _check(LIB.kpm_mlp_gradients(self._h, x.data_ptr(), target.data_ptr(), weights.data_ptr(), x.shape[0],
                                     flat.ctypes.data, ctypes.byref(loss), _stream_handle(stream)))
        return self._unpack(flat), loss.value

    def fit_scaling(self, x, target, stream=None):
        """Standardise inputs and outputs column by column (statistics of x, target on the device)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        x = x.contiguous()
        target = target.contiguous()
        _check(LIB.kpm_mlp_fit_scaling(self._h, x.data_ptr(), target.data_ptr(), x.shape[0],
                                       _stream_handle(stream)))

    def rel_error(self, x, ref, weights, bf16: bool = True, stream=None):
        """kpm_mlp_rel_error: ||w (y - ref)|| / ||w ref|| per row on the first ref.shape[1] outputs.
        x [B, n_in] float32, ref [B, n_cmp] float64, weights [n_cmp] float32 (device tensors)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        x, ref, weights = x.contiguous(), ref.contiguous(), weights.contiguous()
        assert x.dtype == torch.float32 and ref.dtype == torch.float64 and weights.dtype == torch.float32
        err = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
        _check(LIB.kpm_mlp_rel_error(self._h, x.data_ptr(), ref.data_ptr(), weights.data_ptr(), x.shape[0],
                                     ref.shape[1], 1 if bf16 else 0, err.data_ptr(), _stream_handle(stream)))
        return err

    def noise_z(self, x, ref, noise, weights, bf16: bool = True, stream=None):
        """kpm_mlp_noise_z: ||w (y - ref)|| / (noise ||w||) per row on the first ref.shape[1] outputs.
        x [B, n_in] float32, ref [B, n_cmp] float64, noise [B] float64, weights [n_cmp] float32 (device)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        x, ref, noise, weights = x.contiguous(), ref.contiguous(), noise.contiguous(), weights.contiguous()
        assert x.dtype == torch.float32 and ref.dtype == torch.float64 and weights.dtype == torch.float32
        assert noise.dtype == torch.float64 and noise.shape == (x.shape[0],)
        z = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
        _check(LIB.kpm_mlp_noise_z(self._h, x.data_ptr(), ref.data_ptr(), noise.data_ptr(), weights.data_ptr(),
                                   x.shape[0], ref.shape[1], 1 if bf16 else 0, z.data_ptr(), _stream_handle(stream)))
        return z

    def eval_loss(self, x, target, weights, bf16: bool = False, stream=None):
        """kpm_mlp_eval_loss: the weighted training loss of the network's output (no update), a device double."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        x, target, weights = x.contiguous(), target.contiguous(), weights.contiguous()
        loss = torch.zeros(1, dtype=torch.float64, device=x.device)
        _check(LIB.kpm_mlp_eval_loss(self._h, x.data_ptr(), target.data_ptr(), weights.data_ptr(), x.shape[0],
                                     1 if bf16 else 0, loss.data_ptr(), _stream_handle(stream)))
        return loss

    def close(self):
        if getattr(self, "_h", None):
            LIB.kpm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(lattices: Sequence, par, probe_steps: int = 16, cache_path: Optional[str] = None, stream=None) -> dict:
    """kpm_autotune: the fastest launch shape for this workload (optionally appended to a cache file)."""
    lats = c_lattices(lattices)
    p, keep = c_params(par)
    best = c_tune()
    gbs = ctypes.c_double()
    _check(LIB.kpm_autotune(lats, len(lattices), ctypes.byref(p), int(probe_steps),
                            None if cache_path is None else cache_path.encode(), ctypes.byref(best),
                            ctypes.byref(gbs), _stream_handle(stream)))
    del keep
    return {"kernel": best.kernel, "block": best.block, "rows": best.rows, "grid": best.grid, "chunks": best.chunks,
            "GBs": gbs.value}
