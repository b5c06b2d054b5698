"""Counter-based SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), vectorised over the counter.

Definition used on both sides (each side has its own code):

    mix(z):  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
             z = (z ^ (z >> 27)) * 0x94D049BB133111EB
             return z ^ (z >> 31)                     (all mod 2^64)
    gamma = 0x9E3779B97F4A7C15
    key(purpose, seed, a, b) = mix(mix(mix(seed + purpose*gamma) + a*gamma) + b*gamma)
    x_i = mix(key + (i + 1)*gamma)                    (counter i >= 0)
    u_i = (x_i >> 11) * 2^-53                         in [0, 1)

The paper only asks for white-noise random vectors (Sec. 2(c), STE); the
generator and its keying are this implementation's convention.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
C1 = 0xBF58476D1CE4E5B9
C2 = 0x94D049BB133111EB
M64 = (1 << 64) - 1

PHASE = 1
ANDERSON = 2
VACANCY = 3
MLP = 5


def mix_int(z: int) -> int:
    """Scalar SplitMix64 finaliser on Python integers."""
    z &= M64
    z = ((z ^ (z >> 30)) * C1) & M64
    z = ((z ^ (z >> 27)) * C2) & M64
    return z ^ (z >> 31)


def stream_key(purpose: int, seed: int, a: int = 0, b: int = 0) -> int:
    k = mix_int(seed + purpose * GAMMA)
    k = mix_int(k + a * GAMMA)
    return mix_int(k + b * GAMMA)


def _mix_vec(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(C1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(C2)
        z = z ^ (z >> np.uint64(31))
    return z


def raw(key: int, counters: np.ndarray) -> np.ndarray:
    """x_i = mix(key + (i+1)*gamma) for an array of counters i (uint64)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key & M64) + (c + np.uint64(1)) * np.uint64(GAMMA)
    return _mix_vec(z)


def uniform(key: int, counters: np.ndarray) -> np.ndarray:
    """u_i = (x_i >> 11) * 2^-53, exactly representable doubles in [0, 1)."""
    x = raw(key, counters)
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
