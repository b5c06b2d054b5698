"""Pins for the oracle's SplitMix64 streams (published test vector + independent code)."""
import os

import numpy as np

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def _load_golden():
    seed, vals = None, []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("seed"):
                seed = int(line.split()[1])
            else:
                vals.append(int(line))
    return seed, vals


def test_splitmix64_published_vector():
    seed, vals = _load_golden()
    got = rng.raw(seed, np.arange(len(vals)))
    assert [int(x) for x in got] == vals


def test_vectorised_matches_bigint_arithmetic():
    g = np.random.default_rng(0)
    for key in [0, 1, 2**63 + 12345, int(g.integers(0, 2**62)) * 3]:
        counters = g.integers(0, 2**40, size=64).astype(np.uint64)
        got = rng.raw(key, counters)
        for c, x in zip(counters, got):
            z = (key + (int(c) + 1) * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & ((1 << 64) - 1)
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & ((1 << 64) - 1)
            z = z ^ (z >> 31)
            assert int(x) == z


def test_uniform_statistics():
    n = 1 << 20
    u = rng.uniform(rng.stream_key(rng.PHASE, 5194, 0, 0), np.arange(n, dtype=np.uint64))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
    hist, _ = np.histogram(u, bins=64, range=(0, 1))
    chi2 = np.sum((hist - n / 64) ** 2 / (n / 64))
    assert chi2 < 63 + 6 * np.sqrt(2 * 63)


def test_streams_are_distinct_and_uncorrelated():
    n = 1 << 18
    c = np.arange(n, dtype=np.uint64)
    keys = [rng.stream_key(p, s, a, b) for p, s, a, b in
            [(1, 5194, 0, 0), (1, 5194, 0, 1), (1, 5194, 1, 0), (2, 1910, 0, 0), (3, 1910, 0, 0)]]
    assert len(set(keys)) == len(keys)
    us = [rng.uniform(k, c) - 0.5 for k in keys]
    for i in range(len(us)):
        for j in range(i + 1, len(us)):
            corr = np.mean(us[i] * us[j]) / (1 / 12)
            assert abs(corr) < 5 / np.sqrt(n)
