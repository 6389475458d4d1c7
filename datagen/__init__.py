"""Seeded synthetic workloads for the static hash-table path.

This module generates inputs only.  It holds none of the hash-table
arithmetic (no hashing into buckets, no probing, no placement), so both the
CPU oracle and the GPU library can be fed from it without sharing any of the
method's code.

Workload shape (paper, Section VII): unique keys drawn uniformly from the
32-bit unsigned range, random 32-bit values, positive queries that are the
inserted keys in shuffled order and negative queries that are uniform keys
absent from the table.  The paper draws keys with a Mersenne Twister and
rejects duplicates; here a keyed Feistel permutation of a counter is used
instead, which yields a uniform set of distinct keys by construction (no
duplicate rejection pass is needed, so 2^28-key workloads build in seconds).
The reserved empty-key sentinel (all ones) never appears as a key.

Hash constants are random numbers the method draws (Section VII: a and b are
random integers below the prime p); they are drawn here and passed to both
sides explicitly.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 0x2108072320210807
P32 = 4294967291            # prime modulus of the 32-bit hash family (Section VII)
P61 = (1 << 61) - 1         # prime modulus used for 64-bit keys (not in the paper)
SENTINEL32 = 0xFFFFFFFF
SENTINEL64 = 0xFFFFFFFFFFFFFFFF

# Purpose tags: each stream of random numbers is derived from seed ^ tag.
TAG_KEYS = 0x01
TAG_VALUES = 0x02
TAG_PERM = 0x04
TAG_HASH = 0x05
TAG_RNG = 0x06
TAG_MIX = 0x07
TAG_SIZES = 0x08
TAG_ARRIVALS = 0x09

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start..start+count-1 of Steele/Lea/Flood's splitmix64 stream.

    Output i is mix(seed + (i + 1) * gamma); vectorised, wraps mod 2^64.
    """
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _seed(seed: int, tag: int) -> int:
    return (SEED_BASE ^ int(seed) ^ (tag << 56)) & 0xFFFFFFFFFFFFFFFF


def _fmix32(x: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        x = x ^ (x >> np.uint32(16))
        x = x * np.uint32(0x85EBCA6B)
        x = x ^ (x >> np.uint32(13))
        x = x * np.uint32(0xC2B2AE35)
        x = x ^ (x >> np.uint32(16))
    return x


def feistel32(x: np.ndarray, round_keys) -> np.ndarray:
    """Keyed bijection of [0, 2^32): four Feistel rounds over 16-bit halves."""
    x = np.asarray(x, dtype=np.uint32)
    left = x >> np.uint32(16)
    right = x & np.uint32(0xFFFF)
    for rk in round_keys:
        with np.errstate(over="ignore"):
            f = _fmix32(right * np.uint32(0x9E3779B1) + np.uint32(rk & 0xFFFFFFFF))
        left, right = right, (left ^ (f >> np.uint32(16))) & np.uint32(0xFFFF)
    return (left << np.uint32(16)) | right


def _fmix64(x: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        x = x ^ (x >> np.uint64(33))
        x = x * np.uint64(0xFF51AFD7ED558CCD)
        x = x ^ (x >> np.uint64(33))
        x = x * np.uint64(0xC4CEB9FE1A85EC53)
        x = x ^ (x >> np.uint64(33))
    return x


def feistel64(x: np.ndarray, round_keys) -> np.ndarray:
    """Keyed bijection of [0, 2^64): four Feistel rounds over 32-bit halves."""
    x = np.asarray(x, dtype=np.uint64)
    left = x >> np.uint64(32)
    right = x & np.uint64(0xFFFFFFFF)
    for rk in round_keys:
        with np.errstate(over="ignore"):
            f = _fmix64(right * np.uint64(0x9E3779B97F4A7C15) + np.uint64(rk))
        left, right = right, (left ^ (f >> np.uint64(32))) & np.uint64(0xFFFFFFFF)
    return (left << np.uint64(32)) | right


def _round_keys(seed: int, tag: int) -> list:
    return [int(v) for v in splitmix64(_seed(seed, tag), 4)]


def _distinct32(idx: np.ndarray, seed: int) -> np.ndarray:
    """Images of distinct indices under a bijection of [0,2^32) minus the sentinel.

    The sentinel is cycle-walked: the one index mapped onto it is sent to the
    image of the sentinel itself, which no other index in range can reach.
    """
    rk = _round_keys(seed, TAG_KEYS)
    y = feistel32(idx, rk)
    hit = y == np.uint32(SENTINEL32)
    if hit.any():
        y[hit] = feistel32(np.array([SENTINEL32], dtype=np.uint32), rk)[0]
    return y


def unique_keys(n: int, seed: int) -> np.ndarray:
    """n distinct uniform uint32 keys, none equal to the sentinel."""
    if n >= SENTINEL32:
        raise ValueError("too many keys for the 32-bit key space")
    return _distinct32(np.arange(n, dtype=np.uint32), seed)


def negative_keys(count: int, n_inserted: int, seed: int) -> np.ndarray:
    """count uniform uint32 keys disjoint from unique_keys(n_inserted, seed)."""
    if n_inserted + count >= SENTINEL32:
        raise ValueError("key space exhausted")
    idx = np.arange(n_inserted, n_inserted + count, dtype=np.uint64).astype(np.uint32)
    return _distinct32(idx, seed)


def values(n: int, seed: int) -> np.ndarray:
    """n uniform uint32 values (any value, the sentinel included)."""
    return (splitmix64(_seed(seed, TAG_VALUES), n) >> np.uint64(32)).astype(np.uint32)


def permutation(n: int, seed: int, tag: int = TAG_PERM) -> np.ndarray:
    """A seeded uniform permutation of 0..n-1 (int64 indices)."""
    return np.random.Generator(np.random.PCG64(_seed(seed, tag))).permutation(n)


def positive_queries(keys: np.ndarray, seed: int) -> np.ndarray:
    """The inserted keys in shuffled order."""
    return keys[permutation(len(keys), seed)]


def mixed_queries(keys: np.ndarray, count: int, positive_fraction: float, seed: int):
    """count queries, floor(fraction*count) of them inserted keys, the rest absent.

    Positives are a prefix of a shuffle of the inserted keys (repeating the
    shuffle if count exceeds the key count); negatives come from the disjoint
    key stream.  The union is shuffled again.  Returns the query array.
    """
    n = len(keys)
    npos = int(math.floor(positive_fraction * count))
    if npos > 0 and n == 0:
        raise ValueError("positive queries requested from an empty key set")
    pos_idx = permutation(n, seed)[: min(npos, n)] if n else np.zeros(0, np.int64)
    if npos > n:
        pos_idx = np.resize(pos_idx, npos)
    pos = keys[pos_idx]
    neg = negative_keys(count - npos, n, seed)
    q = np.concatenate([pos, neg])
    return q[permutation(count, seed, TAG_MIX)]


def hash_constants(seed: int, h: int):
    """h pairs (a_i, b_i) with a_i in [1, p-1] and b_i in [0, p-1], p = 4294967291.

    Drawn by rejection from the seed's splitmix64 stream (32-bit draws)."""
    out_a, out_b = [], []
    stream = splitmix64(_seed(seed, TAG_HASH), 64 * h)
    it = iter(int(v) for v in stream)
    while len(out_a) < h:
        a = next(it) & 0xFFFFFFFF
        b = next(it) & 0xFFFFFFFF
        if 1 <= a < P32 and b < P32:
            out_a.append(a)
            out_b.append(b)
    return out_a, out_b


def hash_constants64(seed: int, h: int):
    """h pairs (a_i, b_i) with a_i in [1, q-1], b_i in [0, q-1], q = 2^61 - 1."""
    out_a, out_b = [], []
    stream = splitmix64(_seed(seed, TAG_HASH), 64 * h)
    it = iter(int(v) for v in stream)
    while len(out_a) < h:
        a = next(it) >> 3
        b = next(it) >> 3
        if 1 <= a < P61 and b < P61:
            out_a.append(a)
            out_b.append(b)
    return out_a, out_b


def rng_seed(seed: int) -> int:
    """Nonzero 32-bit seed for the eviction-victim generator."""
    s = int(splitmix64(_seed(seed, TAG_RNG), 1)[0]) & 0xFFFFFFFF
    return s or 0x9E3779B9


def unique_keys64(n: int, seed: int) -> np.ndarray:
    """n distinct uniform uint64 keys, none equal to the all-ones sentinel."""
    rk = _round_keys(seed, TAG_KEYS)
    y = feistel64(np.arange(n, dtype=np.uint64), rk)
    hit = y == np.uint64(SENTINEL64)
    if hit.any():
        y[hit] = feistel64(np.array([SENTINEL64], dtype=np.uint64), rk)[0]
    return y


def negative_keys64(count: int, n_inserted: int, seed: int) -> np.ndarray:
    rk = _round_keys(seed, TAG_KEYS)
    y = feistel64(np.arange(n_inserted, n_inserted + count, dtype=np.uint64), rk)
    hit = y == np.uint64(SENTINEL64)
    if hit.any():
        y[hit] = feistel64(np.array([SENTINEL64], dtype=np.uint64), rk)[0]
    return y


def values64(n: int, seed: int) -> np.ndarray:
    return splitmix64(_seed(seed, TAG_VALUES), n)


def mixed_queries64(keys: np.ndarray, count: int, positive_fraction: float, seed: int):
    n = len(keys)
    npos = int(math.floor(positive_fraction * count))
    pos_idx = permutation(n, seed)[: min(npos, n)] if n else np.zeros(0, np.int64)
    if npos > n:
        pos_idx = np.resize(pos_idx, npos)
    q = np.concatenate([keys[pos_idx], negative_keys64(count - npos, n, seed)])
    return q[permutation(count, seed, TAG_MIX)]


def capacity_for(n: int, load_factor: float) -> int:
    """Slots needed to hold n keys at the given load factor: ceil(n / lf)."""
    from fractions import Fraction
    lf = Fraction(str(load_factor))
    return int(-(-Fraction(n) // lf))


def log_uniform_sizes(count: int, lo_log2: int, hi_log2: int, seed: int,
                      tag: int = TAG_SIZES) -> np.ndarray:
    """count sizes floor(2^(lo + (hi - lo) * u)) with u uniform in [0, 1)."""
    u = (splitmix64(_seed(seed, tag), count) >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    return np.floor(np.exp2(lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def uniform01(count: int, seed: int, tag: int) -> np.ndarray:
    """count doubles uniform in [0, 1) from the tagged stream."""
    return (splitmix64(_seed(seed, tag), count) >> np.uint64(11)).astype(np.float64) / float(1 << 53)
