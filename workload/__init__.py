"""Seeded, synthetic workload descriptions shared by the oracle and the HIP path.

This module holds *inputs only*: lattice parameters, seeds, sizes and the
workload presets used by the tests and the benchmark.  It contains none of
the spectral method's arithmetic (no Hamiltonian, no recursion, no moments).
Random numbers that the method itself draws (random-phase vectors, Anderson
potentials, vacancy positions) are *not* produced here: each side implements
the counter-based SplitMix64 generator on its own from its published
definition (Steele, Lea & Flood, OOPSLA 2014), keyed as described in
``RNG_STREAMS`` below.

Model conventions (paper Sec. 3(d) lattice listing; Sec. 4 QAHE model and
magnetic-field example):

* Honeycomb: a1 = (a, 0), a2 = (a/2, a*sqrt(3)/2), a = 0.24595 nm; sublattice
  A at (0, -a_cc/2), B at (0, +a_cc/2), a_cc = 0.142 nm.  Nearest-neighbour
  bonds A(n) - B(n + d) with d in {(0,0), (1,-1), (0,-1)}; periodic wrap.
* Square: one orbital per cell, a1 = (a_sq, 0), a2 = (0, a_sq); bonds to the
  four neighbours (+-1, 0), (0, +-1).
* Orbital index o = ((n2*L1 + n1)*n_sub + s)*n_spin + sigma  (n1 fastest).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional

# Lattice kinds (the same integer codes cross the C ABI).
HONEYCOMB = 0
HONEYCOMB_SPIN = 1
SQUARE = 2

KIND_NAMES = {HONEYCOMB: "honeycomb", HONEYCOMB_SPIN: "honeycomb_spin", SQUARE: "square"}

# Sublattices and spins per cell for each kind.
N_SUB = {HONEYCOMB: 2, HONEYCOMB_SPIN: 2, SQUARE: 1}
N_SPIN = {HONEYCOMB: 1, HONEYCOMB_SPIN: 2, SQUARE: 1}

# Geometry (nm).
A_HONEYCOMB = 0.24595
ACC_HONEYCOMB = 0.142
A_SQUARE = 0.24595

# Precision codes.
FP32 = 0
FP64 = 1

# Start-vector kinds.
START_RANDOM_PHASE = 0
START_SITES = 1

# Gamma accumulation modes.
GAMMA_FP64 = 0
GAMMA_FP32 = 1
GAMMA_SPLIT_BF16 = 2

# RNG stream purposes: stream key = f(purpose, seed, a, b), counter = site or
# orbital index.  Both sides implement the same keying.
RNG_PHASE = 1      # a = lattice index in the batch, b = random vector r; counter = orbital
RNG_ANDERSON = 2   # a = b = 0; counter = site (cell*n_sub + s)
RNG_VACANCY = 3    # a = b = 0; counter = site
RNG_SIZES = 4      # input generation only (this module)
RNG_MLP = 5        # weight initialisation / data shuffling

RNG_STREAMS = {
    "phase": RNG_PHASE, "anderson": RNG_ANDERSON, "vacancy": RNG_VACANCY,
    "sizes": RNG_SIZES, "mlp": RNG_MLP,
}


@dataclass
class Lattice:
    """One tight-binding lattice (mirrors a KITE configuration + disorder + modification)."""
    kind: int = HONEYCOMB
    L1: int = 64
    L2: int = 64
    t: float = -2.7            # NN hopping matrix element, eV
    rashba: float = 0.0        # lambda_R, eV (HONEYCOMB_SPIN only)
    flux: float = 0.0          # flux per unit cell in units of h/e; flux*L1 must be an integer
    anderson_w: float = 0.0    # on-site potential uniform in [-W/2, W/2] eV, spin independent
    vacancy_p: float = 0.0     # per-site removal probability
    disorder_seed: int = 0
    e_min: float = -8.5
    e_max: float = 8.5
    exchange: float = 0.0      # Delta_ex s_z, eV (HONEYCOMB_SPIN only)

    @property
    def n_sub(self) -> int:
        return N_SUB[self.kind]

    @property
    def n_spin(self) -> int:
        return N_SPIN[self.kind]

    @property
    def n_orb_cell(self) -> int:
        return self.n_sub * self.n_spin

    @property
    def n_sites(self) -> int:
        return self.L1 * self.L2 * self.n_sub

    @property
    def n_orbitals(self) -> int:
        return self.L1 * self.L2 * self.n_orb_cell

    def replace(self, **kw) -> "Lattice":
        return dataclasses.replace(self, **kw)


@dataclass
class DosParams:
    num_moments: int = 256
    num_random: int = 4
    vector_seed: int = 0
    precision: int = FP64
    start: int = START_RANDOM_PHASE
    sites: Optional[List[int]] = None   # orbital indices for LDOS (num_random := len(sites))

    def replace(self, **kw) -> "DosParams":
        return dataclasses.replace(self, **kw)


@dataclass
class CondParams:
    num_moments: int = 64
    num_random: int = 1
    vector_seed: int = 0
    alpha: int = 0    # 0 = x, 1 = y
    beta: int = 0
    gamma_mode: int = GAMMA_SPLIT_BF16

    def replace(self, **kw) -> "CondParams":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# Input-generation RNG (sizes of the uneven batch only).  SplitMix64 as
# published: x_i = mix(seed + (i+1)*gamma), with the 64-bit finaliser below.
# --------------------------------------------------------------------------
_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def _mix(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def _key(purpose: int, seed: int, a: int = 0, b: int = 0) -> int:
    k = _mix(seed + purpose * _GAMMA)
    k = _mix(k + a * _GAMMA)
    return _mix(k + b * _GAMMA)


def _uniform(key: int, i: int) -> float:
    return (_mix(key + (i + 1) * _GAMMA) >> 11) * (1.0 / (1 << 53))


# --------------------------------------------------------------------------
# Workload presets (sizes, seeds and value distributions of the paper's
# graphene benchmarks and of the five target configurations).
# --------------------------------------------------------------------------
DISORDER_SEED = 1910
VECTOR_SEED = 5194


def graphene_small() -> tuple:
    """64x64 honeycomb, NN t=-2.7 eV, Anderson W=1 eV, bound 8.5 eV, FP64, M=256, R=4."""
    lat = Lattice(kind=HONEYCOMB, L1=64, L2=64, t=-2.7, anderson_w=1.0,
                  disorder_seed=DISORDER_SEED, e_min=-8.5, e_max=8.5)
    par = DosParams(num_moments=256, num_random=4, vector_seed=VECTOR_SEED, precision=FP64)
    return lat, par


def graphene_large(precision: int = FP32, L: int = 4096, M: int = 2048, R: int = 32) -> tuple:
    """4096x4096 honeycomb + Anderson (33.5M orbitals), M=2048, R=32 complex vectors."""
    lat = Lattice(kind=HONEYCOMB, L1=L, L2=L, t=-2.7, anderson_w=1.0,
                  disorder_seed=DISORDER_SEED, e_min=-8.5, e_max=8.5)
    par = DosParams(num_moments=M, num_random=R, vector_seed=VECTOR_SEED, precision=precision)
    return lat, par


def rashba_flux(L: int = 1024, M: int = 512, R: int = 8, gamma_mode: int = GAMMA_SPLIT_BF16) -> tuple:
    """Spinful honeycomb, Rashba 0.2 eV, flux 1/L per cell, clean, bound 8.5 eV; sigma_xx."""
    lat = Lattice(kind=HONEYCOMB_SPIN, L1=L, L2=L, t=-2.7, rashba=0.2, flux=1.0 / L,
                  disorder_seed=DISORDER_SEED, e_min=-8.5, e_max=8.5)
    par = CondParams(num_moments=M, num_random=R, vector_seed=VECTOR_SEED, alpha=0, beta=0,
                     gamma_mode=gamma_mode)
    return lat, par


def qahe(L: int = 512, M: int = 1024, R: int = 1) -> tuple:
    """The paper's QAHE model (eq. HQAHE, Fig. qahe): spinful honeycomb, t = -2.7 eV,
    lambda_R = 0.3 |t|, Delta_ex = 0.4 |t|, clean, bounds +-10 eV; Gamma^xy split-BF16."""
    lat = Lattice(kind=HONEYCOMB_SPIN, L1=L, L2=L, t=-2.7, rashba=0.81, exchange=1.08,
                  disorder_seed=DISORDER_SEED, e_min=-10.0, e_max=10.0)
    par = CondParams(num_moments=M, num_random=R, vector_seed=3, alpha=0, beta=1, gamma_mode=GAMMA_SPLIT_BF16)
    return lat, par


def spin_wavepacket(L: int = 7168) -> dict:
    """The paper's spin-dynamics example (Sec. 4, Fig. spinpress(a)): spinful honeycomb
    L x L cells, t = -2.507 eV, lambda_R = 10 meV, Anderson W = 1.5 eV, bounds +-8.5 eV;
    2 fs time steps with M = 70 terms; a Gaussian packet of width 110 nm at the centre,
    momentum K + q with hbar v_F q = E_F = 0.1 eV (v_F from the hopping), polarised along
    z (first packet) and along x (second)."""
    lat = Lattice(kind=HONEYCOMB_SPIN, L1=L, L2=L, t=-2.507, rashba=0.010, anderson_w=1.5,
                  disorder_seed=DISORDER_SEED, e_min=-8.5, e_max=8.5)
    hbar_vf = 1.5 * 2.507 * ACC_HONEYCOMB                      # eV nm
    k = [4.0 * 3.141592653589793 / (3.0 * A_HONEYCOMB) + 0.1 / hbar_vf, 0.0]
    s = 0.5 ** 0.5
    sz = [s, 0.0, s, 0.0]                                       # A up, A down, B up, B down
    sx = [0.5, 0.5, 0.5, 0.5]
    return {"lattice": lat, "k": [k], "spinors": [[sz], [sx]], "width_nm": 110.0, "center": [L / 2, L / 2],
            "dt_fs": 2.0, "num_moments": 70}


def graphene_clean(L: int = 1024, M: int = 1024, R: int = 4) -> tuple:
    """Clean spinless graphene, t = -2.7 eV, bounds +-9 eV; xx response, split-BF16 Gamma."""
    lat = Lattice(kind=HONEYCOMB, L1=L, L2=L, t=-2.7, disorder_seed=DISORDER_SEED, e_min=-9.0, e_max=9.0)
    par = CondParams(num_moments=M, num_random=R, vector_seed=4, alpha=0, beta=0, gamma_mode=GAMMA_SPLIT_BF16)
    return lat, par


def uneven_batch(n_lat: int = 64, lo: int = 256, hi: int = 2048, M: int = 1024, R: int = 4,
                 vacancy_p: float = 0.005, size_seed: int = 4) -> tuple:
    """n_lat graphene lattices with L_i ~ U{lo..hi} (square L_i x L_i), vacancies only."""
    key = _key(RNG_SIZES, size_seed)
    lats = []
    for i in range(n_lat):
        L = lo + int(_uniform(key, i) * (hi - lo + 1))
        lats.append(Lattice(kind=HONEYCOMB, L1=L, L2=L, t=-2.7, vacancy_p=vacancy_p,
                            disorder_seed=DISORDER_SEED + i, e_min=-8.5, e_max=8.5))
    par = DosParams(num_moments=M, num_random=R, vector_seed=VECTOR_SEED, precision=FP32)
    return lats, par


def mlp_training_lattice(i: int, L: int = 256, seed: int = 20000) -> Lattice:
    """Random honeycomb or square lattice for the moment-extrapolation training set.

    Lattice kind ~ Bernoulli(1/2), W ~ U[0, 3] eV, vacancy fraction ~ U[0, 0.02];
    bound 1.01*(Z|t| + W/2) with t = -2.7 eV.
    """
    key = _key(RNG_SIZES, seed, i)
    kind = HONEYCOMB if _uniform(key, 0) < 0.5 else SQUARE
    W = 3.0 * _uniform(key, 1)
    p = 0.02 * _uniform(key, 2)
    Z = 3 if kind == HONEYCOMB else 4
    b = 1.01 * (Z * 2.7 + W / 2)
    return Lattice(kind=kind, L1=L, L2=L, t=-2.7, anderson_w=W, vacancy_p=p,
                   disorder_seed=seed * 7919 + i, e_min=-b, e_max=b)


def mlp_eval_lattice(i: int, L: int = 2048, seed: int = 30000) -> Lattice:
    """Held-out honeycomb evaluation draw from the training disorder distribution."""
    key = _key(RNG_SIZES, seed, i)
    W = 3.0 * _uniform(key, 1)
    p = 0.02 * _uniform(key, 2)
    b = 1.01 * (3 * 2.7 + W / 2)
    return Lattice(kind=HONEYCOMB, L1=L, L2=L, t=-2.7, anderson_w=W, vacancy_p=p,
                   disorder_seed=seed * 7919 + i, e_min=-b, e_max=b)


def energy_grid(e_min: float, e_max: float, K: int = 1024):
    """Midpoint grid E_k = E_min + (k + 1/2)(E_max - E_min)/K (k = 0..K-1)."""
    import numpy as np
    k = np.arange(K, dtype=np.float64)
    return e_min + (k + 0.5) * (e_max - e_min) / K
