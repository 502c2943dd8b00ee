"""Rademacher probe signs from the counter-based SplitMix64 generator.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the k-th output (k = 0, 1, ...) of the stream with
initial state `seed` is obtained by advancing the state by k+1 times the golden
gamma 0x9E3779B97F4A7C15 (mod 2^64) and applying the mix function
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
    z ^= z >> 31.
Probe s at user-order point u uses counter k = s * 2^40 + u and is +1 when bit 63
of the output is 0, else -1. Indexing by the user-order point keeps the probes
independent of any internal reordering of the points.

Pinned by the generator's published first output in tests/test_oracle_probes.py.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, k):
    """Output number k (uint64 array) of the SplitMix64 stream seeded with `seed`."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (k + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def rademacher_probes(seed, n_probes, n):
    """(n_probes, n) float64 array of +-1 in user order."""
    s = np.arange(n_probes, dtype=np.uint64)[:, None]
    u = np.arange(n, dtype=np.uint64)[None, :]
    z = splitmix64(seed, s * np.uint64(1 << 40) + u)
    neg = (z >> np.uint64(63)).astype(bool)
    return np.where(neg, -1.0, 1.0)


def probe_sign_masks(seed, n_probes, n):
    """(n,) uint64: bit s set when probe s is -1 at that point."""
    z = rademacher_probes(seed, n_probes, n)
    out = np.zeros(n, dtype=np.uint64)
    for s in range(n_probes):
        out |= (z[s] < 0).astype(np.uint64) << np.uint64(s)
    return out
