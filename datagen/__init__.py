"""Seeded synthetic workloads for the static hash-table path.

This module generates inputs only.  It holds none of the hash-table
arithmetic (no hashing into buckets, no probing, no placement), so both the
CPU oracle and the GPU library can be fed from it without sharing any of the
method's code.

The bulk generators run in ``gen.c`` (plain C with OpenMP), loaded with
ctypes; 2^28-key workloads take about a second.

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

import ctypes
import math
import os
import subprocess

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


# ----------------------------------------------------- native generator

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libdatagen.so")
_lib = None


def build_library(force: bool = False) -> str:
    """Compile gen.c with gcc (OpenMP) into libdatagen.so next to the source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _native():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build_library())
        u32, u64, p = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
        _lib.dg_splitmix64.argtypes = [u64, u64, u64, p]
        _lib.dg_values32.argtypes = [u64, u64, p]
        _lib.dg_feistel32.restype = u32
        _lib.dg_feistel32.argtypes = [u32, u32, u32, u32, u32]
        _lib.dg_feistel64.restype = u64
        _lib.dg_feistel64.argtypes = [u64, u64, u64, u64, u64]
        _lib.dg_keys32.argtypes = [p, u64, u64, p]
        _lib.dg_keys64.argtypes = [p, u64, u64, p]
        _lib.dg_permutation.argtypes = [p, u64, p]
        _lib.dg_queries32.argtypes = [p, p, u64, p, u64, u64, ctypes.c_int, p]
        _lib.dg_queries64.argtypes = [p, p, u64, p, u64, u64, ctypes.c_int, p]
        _lib.dg_query_sources.argtypes = [p, u64, p, u64, u64, ctypes.c_int, p]
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def splitmix64_native(seed: int, count: int, start: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    if count:
        _native().dg_splitmix64(seed & 0xFFFFFFFFFFFFFFFF, start, count, _ptr(out))
    return out


def _round_keys(seed: int, tag: int) -> np.ndarray:
    return splitmix64(_seed(seed, tag), 4)


def feistel32(x: int, seed: int) -> int:
    """The keyed 32-bit permutation used for keys (one value)."""
    rk = [int(v) & 0xFFFFFFFF for v in _round_keys(seed, TAG_KEYS)]
    return int(_native().dg_feistel32(x, *rk))


def _keys32(start: int, count: int, seed: int) -> np.ndarray:
    rk = (_round_keys(seed, TAG_KEYS) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    out = np.empty(count, dtype=np.uint32)
    if count:
        _native().dg_keys32(_ptr(rk), start, count, _ptr(out))
    return out


def unique_keys(n: int, seed: int) -> np.ndarray:
    """n distinct uniform uint32 keys, none equal to the sentinel."""
    if n >= SENTINEL32:
        raise ValueError("too many keys for the 32-bit key space")
    return _keys32(0, n, seed)


def negative_keys(count: int, n_inserted: int, seed: int) -> np.ndarray:
    """count uniform uint32 keys disjoint from unique_keys(n_inserted, seed)."""
    if n_inserted + count >= SENTINEL32:
        raise ValueError("key space exhausted")
    return _keys32(n_inserted, count, seed)


def values(n: int, seed: int) -> np.ndarray:
    """n uniform uint32 values (any value, the sentinel included)."""
    out = np.empty(n, dtype=np.uint32)
    if n:
        _native().dg_values32(_seed(seed, TAG_VALUES), n, _ptr(out))
    return out


def permutation(n: int, seed: int, tag: int = TAG_PERM) -> np.ndarray:
    """A seeded permutation of 0..n-1 (int64): a keyed Feistel bijection."""
    out = np.empty(n, dtype=np.int64)
    if n:
        rk = _round_keys(seed, tag)
        _native().dg_permutation(_ptr(rk), n, _ptr(out))
    return out


def _queries(n: int, count: int, npos: int, seed: int, shuffle: bool, wide: bool,
             shuffle_seed=None):
    rk_keys = _round_keys(seed, TAG_KEYS)
    if not wide:
        rk_keys = (rk_keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    ss = seed if shuffle_seed is None else shuffle_seed
    rk_pos = _round_keys(ss, TAG_PERM)
    rk_mix = _round_keys(ss, TAG_MIX)
    out = np.empty(count, dtype=np.uint64 if wide else np.uint32)
    if count:
        fn = _native().dg_queries64 if wide else _native().dg_queries32
        fn(_ptr(rk_keys), _ptr(rk_pos), n, _ptr(rk_mix), count, npos, int(shuffle), _ptr(out))
    return out


def positive_queries(n: int, seed: int, wide: bool = False) -> np.ndarray:
    """The n inserted keys of the seed's key stream, in shuffled order."""
    return _queries(n, n, n, seed, False, wide)


def mixed_queries(n: int, count: int, positive_fraction: float, seed: int,
                  wide: bool = False, shuffle_seed=None) -> np.ndarray:
    """count queries against the first n keys of the seed's key stream.

    floor(fraction * count) of them are inserted keys (a prefix of the
    positive shuffle, repeated if it exceeds n); the rest are the keys that
    follow the n inserted ones in the stream, hence absent.  The union is
    shuffled.  shuffle_seed (default: seed) selects which positives and
    negatives are drawn and their order, over the same key stream.
    """
    npos = int(math.floor(positive_fraction * count))
    if npos > 0 and n == 0:
        raise ValueError("positive queries requested from an empty key set")
    return _queries(n, count, npos, seed, True, wide, shuffle_seed)


def query_sources(n: int, count: int, positive_fraction, seed: int,
                  shuffle_seed=None) -> np.ndarray:
    """Key-stream position of each query of mixed_queries(n, count, fraction,
    seed, shuffle_seed), or of positive_queries(n, seed) when
    positive_fraction is None: below n the query is inserted key number i
    (its expected value is values(n, seed)[i]); from n on it is absent."""
    ss = seed if shuffle_seed is None else shuffle_seed
    if positive_fraction is None:
        npos, shuffle = n, False
        assert count == n
    else:
        npos, shuffle = int(math.floor(positive_fraction * count)), True
    rk_pos, rk_mix = _round_keys(ss, TAG_PERM), _round_keys(ss, TAG_MIX)
    out = np.empty(count, dtype=np.int64)
    if count:
        _native().dg_query_sources(_ptr(rk_pos), n, _ptr(rk_mix), count, npos, int(shuffle),
                                   _ptr(out))
    return out


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


def _keys64(start: int, count: int, seed: int) -> np.ndarray:
    rk = _round_keys(seed, TAG_KEYS)
    out = np.empty(count, dtype=np.uint64)
    if count:
        _native().dg_keys64(_ptr(rk), start, count, _ptr(out))
    return out


def unique_keys64(n: int, seed: int) -> np.ndarray:
    """n distinct uniform uint64 keys, none equal to the all-ones sentinel."""
    return _keys64(0, n, seed)


def negative_keys64(count: int, n_inserted: int, seed: int) -> np.ndarray:
    return _keys64(n_inserted, count, seed)


def values64(n: int, seed: int) -> np.ndarray:
    return splitmix64_native(_seed(seed, TAG_VALUES), n)


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
