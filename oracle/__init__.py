"""CPU oracle for static bucketed hash tables — TEST INFRASTRUCTURE ONLY.

Python face of ``oracle.c``: a plain, serial statement of what the method of
"Better GPU Hash Tables" (arXiv 2108.07232) computes, used to check the GPU
library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import it.  It shares no code with the GPU library
(``paper_2108_07232_amd``) and never imports it.

Every function is pinned by ``tests/test_oracle_pins.py`` to something other
than itself: hand-derived hash values and congruences, a GF(2) matrix form of
the xorshift generator, the paper's worked example (Fig. 1), brute force,
balls-into-bins counts, textbook cuckoo thresholds and the paper's printed
probe counts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SCHEMES = {"bcht": 0, "bp2ht": 1, "iht": 2, "cht1": 3, "bcht_lb": 4}
OK, FAILED, SENTINEL, BADARG = 0, 1, 2, 3
EMPTY32 = 0xFFFFFFFF
EMPTY64 = 0xFFFFFFFFFFFFFFFF


def build_library(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int32),
        ("b", ctypes.c_uint32),
        ("m", ctypes.c_uint64),
        ("h", ctypes.c_uint32),
        ("max_chain", ctypes.c_uint32),
        ("a", ctypes.c_uint64 * 4),
        ("c", ctypes.c_uint64 * 4),
        ("threshold", ctypes.c_uint32),
        ("b2", ctypes.c_uint32),
        ("m2", ctypes.c_uint64),
        ("rng_seed", ctypes.c_uint32),
        ("mock_n", ctypes.c_uint32),
        ("mock_hash", ctypes.POINTER(ctypes.c_uint32)),
        ("iht_early_exit", ctypes.c_uint32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build_library())
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        _lib.orc_hash32.restype = u64
        _lib.orc_hash32.argtypes = [u64, u64, u32, u64]
        _lib.orc_hash64.restype = u64
        _lib.orc_hash64.argtypes = [u64, u64, u64, u64]
        _lib.orc_hash32_many.argtypes = [u64, u64, p, u64, u64, p]
        _lib.orc_hash64_many.argtypes = [u64, u64, p, u64, u64, p]
        _lib.orc_xorshift32.restype = u32
        _lib.orc_xorshift32.argtypes = [u32]
        _lib.orc_table_words.restype = u64
        _lib.orc_table_words.argtypes = [p, ctypes.c_int]
        for name in ("orc_build32", "orc_build64"):
            getattr(_lib, name).restype = ctypes.c_int
            getattr(_lib, name).argtypes = [p, p, p, u64, p, p]
        _lib.orc_insert32.restype = ctypes.c_int
        _lib.orc_insert32.argtypes = [p, p, u32, u32, p, p]
        _lib.orc_exchange32.restype = ctypes.c_int
        _lib.orc_exchange32.argtypes = [p, p, u32, u32, p, p, p]
        _lib.orc_continue32.restype = ctypes.c_int
        _lib.orc_continue32.argtypes = [p, p, u32, u32, u64, u32, p, p]
        _lib.orc_find32.argtypes = [p, p, p, u64, p, p, p, p]
        _lib.orc_find64.argtypes = [p, p, p, u64, p, p, p, p]
        _lib.orc_brute_find32.argtypes = [p, p, u64, p, u64, p, p]
        _lib.orc_brute_find64.argtypes = [p, p, u64, p, u64, p, p]
        _lib.orc_join_find32.argtypes = [p, p, u64, p, u64, p, p]
        _lib.orc_join_find64.argtypes = [p, p, u64, p, u64, p, p]
        for name in ("orc_check32", "orc_check64"):
            getattr(_lib, name).restype = ctypes.c_int
            getattr(_lib, name).argtypes = [p, p, p, p, u64, ctypes.c_char_p, ctypes.c_int]
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


@dataclass
class Params:
    """Table geometry and hash constants (all explicit, no hidden draws)."""
    scheme: str
    b: int
    m: int
    h: int
    a: list
    c: list
    max_chain: int = 128
    threshold: int = 0
    b2: int = 0
    m2: int = 0
    rng_seed: int = 0x9E3779B9
    mock: np.ndarray | None = None   # (mock_n, h) uint32 bucket table, tests only
    early_exit: bool = False         # iceberg find: stop after a primary below t
    _keep: list = field(default_factory=list, repr=False)

    def to_c(self) -> _Params:
        p = _Params()
        p.scheme = SCHEMES[self.scheme]
        p.b, p.m, p.h, p.max_chain = self.b, self.m, self.h, self.max_chain
        for i in range(4):
            p.a[i] = int(self.a[i]) if i < len(self.a) else 0
            p.c[i] = int(self.c[i]) if i < len(self.c) else 0
        p.threshold, p.b2, p.m2, p.rng_seed = self.threshold, self.b2, self.m2, self.rng_seed
        p.iht_early_exit = 1 if self.early_exit else 0
        if self.mock is not None:
            mk = np.ascontiguousarray(self.mock, dtype=np.uint32)
            self._keep = [mk]
            p.mock_n = mk.shape[0]
            p.mock_hash = mk.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        else:
            p.mock_n = 0
        return p

    def slots(self) -> int:
        s = self.m * self.b
        if self.scheme == "iht" and self.b2:
            s += self.m2 * self.b2
        return s


def hash32(a: int, c: int, k: int, m: int) -> int:
    return int(lib().orc_hash32(a, c, k, m))


def hash64(a: int, c: int, k: int, m: int) -> int:
    return int(lib().orc_hash64(a, c, k, m))


def hash32_many(a: int, c: int, keys: np.ndarray, m: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    out = np.empty(len(keys), dtype=np.uint64)
    lib().orc_hash32_many(a, c, _ptr(keys), len(keys), m, _ptr(out))
    return out


def hash64_many(a: int, c: int, keys: np.ndarray, m: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.empty(len(keys), dtype=np.uint64)
    lib().orc_hash64_many(a, c, _ptr(keys), len(keys), m, _ptr(out))
    return out


def xorshift32(x: int) -> int:
    return int(lib().orc_xorshift32(x))


def empty_table(params: Params, wide: bool = False) -> np.ndarray:
    pc = params.to_c()
    words = int(lib().orc_table_words(ctypes.byref(pc), int(wide)))
    return np.full(words, EMPTY64, dtype=np.uint64)


def build32(params: Params, keys: np.ndarray, vals: np.ndarray):
    """Serial build.  Returns (status, table uint64[slots], bucket reads)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    pc = params.to_c()
    table = empty_table(params)
    probes = ctypes.c_uint64(0)
    st = lib().orc_build32(ctypes.byref(pc), _ptr(keys), _ptr(vals), len(keys),
                           _ptr(table), ctypes.byref(probes))
    return st, table, probes.value


def insert32(params: Params, table: np.ndarray, key: int, val: int, rng_state: int):
    """One insertion into an existing layout (modified in place).

    Returns (status, new rng state, bucket reads)."""
    pc = params.to_c()
    rng = ctypes.c_uint32(rng_state)
    probes = ctypes.c_uint64(0)
    st = lib().orc_insert32(ctypes.byref(pc), _ptr(table), key, val, ctypes.byref(rng),
                            ctypes.byref(probes))
    return st, rng.value, probes.value


def exchange32(params: Params, table: np.ndarray, key: int, val: int, rng_state: int):
    """First cuckoo step of inserting (key, val) whose first bucket is full:
    exchange with a random slot there (table modified in place).  Returns
    (status, new rng state, evicted key, evicted value)."""
    pc = params.to_c()
    rng = ctypes.c_uint32(rng_state)
    ek, ev = ctypes.c_uint32(0), ctypes.c_uint32(0)
    st = lib().orc_exchange32(ctypes.byref(pc), _ptr(table), key, val, ctypes.byref(rng),
                              ctypes.byref(ek), ctypes.byref(ev))
    return st, rng.value, ek.value, ev.value


def continue32(params: Params, table: np.ndarray, key: int, val: int, from_bucket: int,
               chain: int, rng_state: int):
    """Rest of the insertion of a pair just evicted from bucket from_bucket
    after `chain` exchanges.  Returns (status, new rng state, bucket reads)."""
    pc = params.to_c()
    rng = ctypes.c_uint32(rng_state)
    probes = ctypes.c_uint64(0)
    st = lib().orc_continue32(ctypes.byref(pc), _ptr(table), key, val, from_bucket, chain,
                              ctypes.byref(rng), ctypes.byref(probes))
    return st, rng.value, probes.value


def find32(params: Params, table: np.ndarray, queries: np.ndarray):
    """Serial find.  Returns (values, found, total probes, per-query probes)."""
    q = np.ascontiguousarray(queries, dtype=np.uint32)
    table = np.ascontiguousarray(table, dtype=np.uint64)
    pc = params.to_c()
    out_v = np.empty(len(q), dtype=np.uint32)
    out_f = np.empty(len(q), dtype=np.uint8)
    per = np.empty(len(q), dtype=np.uint8)
    probes = ctypes.c_uint64(0)
    lib().orc_find32(ctypes.byref(pc), _ptr(table), _ptr(q), len(q), _ptr(out_v), _ptr(out_f),
                     ctypes.byref(probes), _ptr(per))
    return out_v, out_f, probes.value, per


def brute_find32(keys: np.ndarray, vals: np.ndarray, queries: np.ndarray):
    """The plain definition of lookup: (value, 1) for a stored key, else (all ones, 0)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    q = np.ascontiguousarray(queries, dtype=np.uint32)
    out_v = np.empty(len(q), dtype=np.uint32)
    out_f = np.empty(len(q), dtype=np.uint8)
    lib().orc_brute_find32(_ptr(keys), _ptr(vals), len(keys), _ptr(q), len(q), _ptr(out_v),
                           _ptr(out_f))
    return out_v, out_f


def join_find32(keys: np.ndarray, vals: np.ndarray, queries: np.ndarray):
    """brute_find32's results by a sort-merge join (linear time: every query
    of a 2^28-query batch in seconds)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    q = np.ascontiguousarray(queries, dtype=np.uint32)
    assert len(q) < (1 << 32)
    out_v = np.empty(len(q), dtype=np.uint32)
    out_f = np.empty(len(q), dtype=np.uint8)
    lib().orc_join_find32(_ptr(keys), _ptr(vals), len(keys), _ptr(q), len(q), _ptr(out_v),
                          _ptr(out_f))
    return out_v, out_f


def check32(params: Params, table: np.ndarray, keys: np.ndarray, vals: np.ndarray):
    """Layout invariants.  Returns (0, 'ok') or (invariant number, message)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    table = np.ascontiguousarray(table, dtype=np.uint64)
    pc = params.to_c()
    buf = ctypes.create_string_buffer(512)
    code = lib().orc_check32(ctypes.byref(pc), _ptr(table), _ptr(keys), _ptr(vals), len(keys),
                             buf, 512)
    return code, buf.value.decode()


def build64(params: Params, keys: np.ndarray, vals: np.ndarray):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    vals = np.ascontiguousarray(vals, dtype=np.uint64)
    pc = params.to_c()
    table = empty_table(params, wide=True)
    probes = ctypes.c_uint64(0)
    st = lib().orc_build64(ctypes.byref(pc), _ptr(keys), _ptr(vals), len(keys),
                           _ptr(table), ctypes.byref(probes))
    return st, table, probes.value


def find64(params: Params, table: np.ndarray, queries: np.ndarray):
    """Serial find.  Returns (values, found, total probes, per-query probes)."""
    q = np.ascontiguousarray(queries, dtype=np.uint64)
    table = np.ascontiguousarray(table, dtype=np.uint64)
    pc = params.to_c()
    out_v = np.empty(len(q), dtype=np.uint64)
    out_f = np.empty(len(q), dtype=np.uint8)
    per = np.empty(len(q), dtype=np.uint8)
    probes = ctypes.c_uint64(0)
    lib().orc_find64(ctypes.byref(pc), _ptr(table), _ptr(q), len(q), _ptr(out_v), _ptr(out_f),
                     ctypes.byref(probes), _ptr(per))
    return out_v, out_f, probes.value, per


def brute_find64(keys: np.ndarray, vals: np.ndarray, queries: np.ndarray):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    vals = np.ascontiguousarray(vals, dtype=np.uint64)
    q = np.ascontiguousarray(queries, dtype=np.uint64)
    out_v = np.empty(len(q), dtype=np.uint64)
    out_f = np.empty(len(q), dtype=np.uint8)
    lib().orc_brute_find64(_ptr(keys), _ptr(vals), len(keys), _ptr(q), len(q), _ptr(out_v),
                           _ptr(out_f))
    return out_v, out_f


def join_find64(keys: np.ndarray, vals: np.ndarray, queries: np.ndarray):
    """brute_find64's results by a sort-merge join (linear time)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    vals = np.ascontiguousarray(vals, dtype=np.uint64)
    q = np.ascontiguousarray(queries, dtype=np.uint64)
    out_v = np.empty(len(q), dtype=np.uint64)
    out_f = np.empty(len(q), dtype=np.uint8)
    lib().orc_join_find64(_ptr(keys), _ptr(vals), len(keys), _ptr(q), len(q), _ptr(out_v),
                          _ptr(out_f))
    return out_v, out_f


def check64(params: Params, table: np.ndarray, keys: np.ndarray, vals: np.ndarray):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    vals = np.ascontiguousarray(vals, dtype=np.uint64)
    table = np.ascontiguousarray(table, dtype=np.uint64)
    pc = params.to_c()
    buf = ctypes.create_string_buffer(512)
    code = lib().orc_check64(ctypes.byref(pc), _ptr(table), _ptr(keys), _ptr(vals), len(keys),
                             buf, 512)
    return code, buf.value.decode()


def params_for(scheme: str, n: int, load_factor: float, seed: int, b: int = 16, h: int | None = None,
               max_chain: int = 128, threshold: int = 0, wide: bool = False) -> Params:
    """Geometry for n keys at a load factor: m = ceil(ceil(n / lf) / b)."""
    import datagen
    if h is None:
        h = {"bcht": 3, "bp2ht": 2, "iht": 3, "cht1": 3, "bcht_lb": 3}[scheme]
    cap = datagen.capacity_for(n, load_factor)
    m = max(1, -(-cap // b))
    a, c = (datagen.hash_constants64 if wide else datagen.hash_constants)(seed, h)
    return Params(scheme=scheme, b=b, m=m, h=h, a=a, c=c, max_chain=max_chain,
                  threshold=threshold, rng_seed=datagen.rng_seed(seed))
