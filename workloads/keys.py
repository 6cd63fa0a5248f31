"""Seeded synthetic key generator shared by the tests and the benchmark.

This module draws input keys only.  It holds none of the filter's arithmetic
(no hashing, fingerprints or bucket indices) and imports neither the oracle nor
the GPU library.

Keys are uniformly distributed 64-bit integers, the input distribution of the
paper's synthetic throughput runs.  Key number ``c`` of a stream with seed
``s`` is output ``c`` of SplitMix64 (Steele, Lea and Flood, 2014) started at
state ``s``: ``mix(s + (c + 1) * gamma)``.  The map from counter to key is a
bijection of the 64-bit integers, so distinct counters give distinct keys.
Positive keys use counters ``[0, N)``; negative keys use counters at and above
``NEG_BASE`` (2**63), which can therefore never collide with a positive key.
The GPU library carries its own implementation of the same published
generator (``cf_keygen``) for inputs too large to copy from the host.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
NEG_BASE = 1 << 63
U64 = 0xFFFFFFFFFFFFFFFF


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, counters) -> np.ndarray:
    """Outputs number ``counters`` of the SplitMix64 stream starting at ``seed``."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & U64) + (c + np.uint64(1)) * GAMMA
        return _mix(z)


def keys(seed: int, start: int, n: int) -> np.ndarray:
    """``n`` keys from counters ``start .. start+n-1`` (wrapping mod 2**64)."""
    with np.errstate(over="ignore"):
        c = np.uint64(start & U64) + np.arange(n, dtype=np.uint64)
    return splitmix64(seed, c)


def negatives(seed: int, start: int, n: int) -> np.ndarray:
    """``n`` keys disjoint from every positive key of the same seed."""
    return keys(seed, NEG_BASE + start, n)


def seeded_subset(seed: int, n: int, k: int) -> np.ndarray:
    """A seeded random subset of ``k`` indices of ``range(n)``, in index order.

    Indices are ranked by a SplitMix64 output keyed on the index and the seed;
    the ``k`` lowest ranks are taken.  Deterministic and library-independent.
    """
    rank = splitmix64(seed ^ 0xDE1E7E, np.arange(n, dtype=np.uint64))
    idx = np.argsort(rank, kind="stable")[:k]
    return np.sort(idx)


def seeded_permutation(seed: int, n: int) -> np.ndarray:
    """A seeded random permutation of ``range(n)``."""
    rank = splitmix64(seed ^ 0x5E4F1E, np.arange(n, dtype=np.uint64))
    return np.argsort(rank, kind="stable")


def seeded_coin(seed: int, n: int, p_true: float) -> np.ndarray:
    """A seeded boolean mask with ``P(True) = p_true`` per element."""
    u = splitmix64(seed ^ 0xC0FFEE, np.arange(n, dtype=np.uint64))
    thr = np.uint64(min(int(p_true * 2.0**64), U64))
    return u < thr


def workload_seed(k: int) -> int:
    """Seed for workload number k."""
    return 0x5EED0000 + k
