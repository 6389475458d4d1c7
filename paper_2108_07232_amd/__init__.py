"""Static bucketed hash tables for AMD Instinct MI355X (gfx950).

Thin ctypes binding of ``libbht.so`` (C ABI in ``include/bht.h``): argument
marshalling only.  Building and querying run in the library's HIP kernels;
PyTorch supplies device memory and streams.  If the library has not been
built, importing this package raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbht.so")

BHT_BCHT, BHT_BP2HT, BHT_IHT, BHT_CHT1, BHT_BCHT_LB = 0, 1, 2, 3, 4
SCHEMES = {"bcht": BHT_BCHT, "bp2ht": BHT_BP2HT, "iht": BHT_IHT, "cht1": BHT_CHT1,
           "bcht_lb": BHT_BCHT_LB}

STATUS = {
    0: "BHT_OK", 1: "BHT_ERR_INVALID_ARG", 2: "BHT_ERR_CAPACITY", 3: "BHT_ERR_SENTINEL_KEY",
    4: "BHT_ERR_BUILD_FAILED", 5: "BHT_ERR_NOT_BUILT", 6: "BHT_ERR_OOM", 7: "BHT_ERR_HIP",
    8: "BHT_ERR_UNSUPPORTED",
}
BHT_OK, BHT_ERR_INVALID_ARG, BHT_ERR_CAPACITY, BHT_ERR_SENTINEL_KEY = 0, 1, 2, 3
BHT_ERR_BUILD_FAILED, BHT_ERR_NOT_BUILT, BHT_ERR_OOM, BHT_ERR_HIP, BHT_ERR_UNSUPPORTED = 4, 5, 6, 7, 8


class BhtError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__("%s: %s (%s)" % (where, STATUS.get(status, status), detail))
        self.status = status


class bht_params(ctypes.Structure):
    _fields_ = [
        ("num_hashes", ctypes.c_uint32),
        ("key_bits", ctypes.c_uint32),
        ("a", ctypes.c_uint64 * 4),
        ("b", ctypes.c_uint64 * 4),
        ("rng_seed", ctypes.c_uint32),
        ("max_chain", ctypes.c_uint32),
        ("iht_threshold", ctypes.c_uint32),
        ("iht_secondary_b", ctypes.c_uint32),
        ("iht_secondary_m", ctypes.c_uint64),
    ]


class bht_tuning(ctypes.Structure):
    _fields_ = [("tile_width", ctypes.c_uint32), ("find_schedule", ctypes.c_uint32),
                ("grid_blocks", ctypes.c_uint32), ("build_mode", ctypes.c_uint32),
                ("iht_early_exit", ctypes.c_uint32), ("query_unroll", ctypes.c_uint32)]


class bht_batch_entry(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("d_keys", ctypes.c_void_p),
                ("d_values", ctypes.c_void_p), ("n_keys", ctypes.c_uint64),
                ("d_queries", ctypes.c_void_p), ("n_queries", ctypes.c_uint64),
                ("d_out_values", ctypes.c_void_p), ("d_out_found", ctypes.c_void_p)]


class bht_find_request(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("d_queries", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("d_out_values", ctypes.c_void_p), ("d_out_found", ctypes.c_void_p)]


BHT_FIND_DEFAULT, BHT_FIND_REFILL, BHT_FIND_CHUNK, BHT_FIND_PARALLEL = 0, 1, 2, 3
FIND_SCHEDULES = {"default": 0, "refill": 1, "chunk": 2, "parallel": 3}
BHT_BUILD_AUTO, BHT_BUILD_CONCURRENT, BHT_BUILD_PARTITIONED = 0, 1, 2
BUILD_MODES = {"auto": 0, "concurrent": 1, "partitioned": 2}

if not os.path.exists(LIB_PATH):
    raise ImportError("libbht.so is not built; run __graft_entry__.build() "
                      "(or python paper_2108_07232_amd/build.py) first")

_lib = ctypes.CDLL(LIB_PATH)
_u32, _u64, _p, _st = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
_pp = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "bht_create": (_st, [_u64, _u32, ctypes.c_int, ctypes.POINTER(bht_params), _pp]),
    "bht_destroy": (None, [_p]),
    "bht_table_bytes": (_u64, [_u64, _u32, ctypes.c_int, ctypes.POINTER(bht_params)]),
    "bht_create_in": (_st, [_u64, _u32, ctypes.c_int, ctypes.POINTER(bht_params), _p, _u64, _pp]),
    "bht_reseed": (_st, [_p, ctypes.POINTER(bht_params)]),
    "bht_build": (_st, [_p, _p, _p, _u64, _p]),
    "bht_build_async": (_st, [_p, _p, _p, _u64, _p]),
    "bht_build_wait": (_st, [_p, _p]),
    "bht_find": (_st, [_p, _p, _u64, _p, _p, _p]),
    "bht_build64": (_st, [_p, _p, _p, _u64, _p]),
    "bht_find64": (_st, [_p, _p, _u64, _p, _p, _p]),
    "bht_build_counted": (_st, [_p, _p, _p, _u64, _p, _p]),
    "bht_build_workspace_bytes": (_u64, [_p, _u64]),
    "bht_build_async_in": (_st, [_p, _p, _p, _u64, _p, _u64, _p]),
    "bht_build_noalloc_max_bytes": (_u64, []),
    "bht_build_async_noalloc": (_st, [_p, _p, _p, _u64, _p]),
    "bht_build_stats": (_st, [_p, ctypes.POINTER(_u32), ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "bht_build_padding": (_st, [_p, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "bht_params_from_seed": (_st, [_u64, ctypes.c_int, _u32, ctypes.POINTER(bht_params)]),
    "bht_build_retry": (_st, [_p, _p, _p, _u64, _u64, _u32, ctypes.POINTER(_u32), _p]),
    "bht_find_counted": (_st, [_p, _p, _u64, _p, _p, _p, _p]),
    "bht_find64_counted": (_st, [_p, _p, _u64, _p, _p, _p, _p]),
    "bht_get_probe_stats": (_st, [_p, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "bht_set_tuning": (_st, [_p, ctypes.POINTER(bht_tuning)]),
    "bht_get_tuning": (_st, [_p, ctypes.POINTER(bht_tuning)]),
    "bht_enable_timing": (_st, [_p, ctypes.c_int]),
    "bht_kernel_ms": (_st, [_p, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "bht_info": (_st, [_p, ctypes.POINTER(_u64), ctypes.POINTER(_u32), ctypes.POINTER(_u64),
                       ctypes.POINTER(_u64)]),
    "bht_download": (_st, [_p, _p]),
    "bht_upload": (_st, [_p, _p, _u64]),
    "bht_device_slots": (_st, [_p, _pp]),
    "bht_diag_gather": (_st, [_p, _u64, _u64, _u32, _u64, _p, _p]),
    "bht_diag_cas": (_st, [_p, _u64, _u64, _u64, _p, _p]),
    "bht_diag_stream": (_st, [_p, _p, _u64, _p, _p]),
    "bht_hash32": (_u64, [_u64, _u64, _u32, _u64]),
    "bht_hash64": (_u64, [_u64, _u64, _u64, _u64]),
    "bht_batch_create": (_st, [ctypes.POINTER(bht_batch_entry), _u32, _u32, _pp]),
    "bht_batch_run": (_st, [_p, _p]),
    "bht_batch_wait": (_st, [_p, _p, ctypes.POINTER(ctypes.c_int)]),
    "bht_batch_destroy": (None, [_p]),
    "bht_batch_build_find": (_st, [ctypes.POINTER(bht_batch_entry), _u32, _u32,
                                   ctypes.POINTER(ctypes.c_int), _p]),
    "bht_find_ctx_create": (_st, [_u32, _u64, _pp]),
    "bht_multi_find": (_st, [_p, ctypes.POINTER(bht_find_request), _u32, _u32, _p]),
    "bht_find_ctx_destroy": (None, [_p]),
    "bht_status_string": (ctypes.c_char_p, [_st]),
    "bht_last_error": (ctypes.c_char_p, []),
}

for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = sorted(_SIGS)


def _check(status: int, where: str):
    if status != BHT_OK:
        raise BhtError(status, where, (_lib.bht_last_error() or b"").decode())


def _dptr(t, dtype=None, name="tensor"):
    """Device address of a contiguous tensor (marshalling only)."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        if not t.is_cuda:
            raise ValueError("%s must be a device tensor" % name)
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if dtype is not None and t.dtype != dtype:
            raise ValueError("%s must have dtype %s, not %s" % (name, dtype, t.dtype))
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(int(t))


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def make_params(a, b, num_hashes=None, key_bits=32, rng_seed=0x9E3779B9, max_chain=128,
                iht_threshold=0, iht_secondary_b=0, iht_secondary_m=0) -> bht_params:
    p = bht_params()
    p.num_hashes = len(a) if num_hashes is None else num_hashes
    p.key_bits = key_bits
    for i in range(4):
        p.a[i] = int(a[i]) if i < len(a) else 0
        p.b[i] = int(b[i]) if i < len(b) else 0
    p.rng_seed = rng_seed & 0xFFFFFFFF
    p.max_chain = max_chain
    p.iht_threshold = iht_threshold
    p.iht_secondary_b = iht_secondary_b
    p.iht_secondary_m = iht_secondary_m
    return p


# ---------------------------------------------------- C ABI, same names

def bht_create(capacity_slots: int, bucket_size: int, scheme, params: bht_params):
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    out = ctypes.c_void_p()
    _check(_lib.bht_create(capacity_slots, bucket_size, scheme, ctypes.byref(params),
                           ctypes.byref(out)), "bht_create")
    return out


def bht_table_bytes(capacity_slots: int, bucket_size: int, scheme, params: bht_params) -> int:
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    return int(_lib.bht_table_bytes(capacity_slots, bucket_size, scheme, ctypes.byref(params)))


def bht_create_in(capacity_slots: int, bucket_size: int, scheme, params: bht_params, buffer,
                  nbytes: int = None):
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    nbytes = buffer.numel() * buffer.element_size() if nbytes is None else nbytes
    out = ctypes.c_void_p()
    _check(_lib.bht_create_in(capacity_slots, bucket_size, scheme, ctypes.byref(params),
                              _dptr(buffer, None, "buffer"), nbytes, ctypes.byref(out)),
           "bht_create_in")
    return out


def bht_destroy(table):
    _lib.bht_destroy(table)


def bht_reseed(table, params: bht_params):
    _check(_lib.bht_reseed(table, ctypes.byref(params)), "bht_reseed")


def bht_build(table, keys, values, n=None, stream=None) -> int:
    """Returns the status (BUILD_FAILED and SENTINEL_KEY are returned, not raised)."""
    n = keys.numel() if n is None else n
    st = _lib.bht_build(table, _dptr(keys, None, "keys"), _dptr(values, None, "values"), n,
                        _stream(stream))
    if st not in (BHT_OK, BHT_ERR_BUILD_FAILED, BHT_ERR_SENTINEL_KEY):
        _check(st, "bht_build")
    return st


def bht_build_async(table, keys, values, n=None, stream=None):
    n = keys.numel() if n is None else n
    _check(_lib.bht_build_async(table, _dptr(keys, None, "keys"), _dptr(values, None, "values"),
                                n, _stream(stream)), "bht_build_async")


def bht_build_workspace_bytes(table, n: int) -> int:
    return int(_lib.bht_build_workspace_bytes(table, n))


def bht_build_async_in(table, keys, values, workspace, n=None, stream=None):
    """Enqueues a build using the caller's device workspace (a uint8 tensor
    of at least bht_build_workspace_bytes(table, n) bytes)."""
    n = keys.numel() if n is None else n
    nbytes = workspace.numel() * workspace.element_size()
    _check(_lib.bht_build_async_in(table, _dptr(keys, None, "keys"), _dptr(values, None, "values"),
                                   n, _dptr(workspace, None, "workspace"), nbytes, _stream(stream)),
           "bht_build_async_in")


def bht_build_noalloc_max_bytes() -> int:
    return int(_lib.bht_build_noalloc_max_bytes())


def bht_build_async_noalloc(table, keys, values, n=None, stream=None) -> int:
    """Enqueues a build whose workspace is the library's fixed per-GPU array
    (no device allocation); returns the status (CAPACITY when the build
    needs more workspace than the array holds)."""
    n = keys.numel() if n is None else n
    st = _lib.bht_build_async_noalloc(table, _dptr(keys, None, "keys"),
                                      _dptr(values, None, "values"), n, _stream(stream))
    if st not in (BHT_OK, BHT_ERR_CAPACITY):
        _check(st, "bht_build_async_noalloc")
    return st


def bht_build_wait(table, stream=None) -> int:
    st = _lib.bht_build_wait(table, _stream(stream))
    if st not in (BHT_OK, BHT_ERR_BUILD_FAILED, BHT_ERR_SENTINEL_KEY):
        _check(st, "bht_build_wait")
    return st


def bht_find(table, queries, out_values, out_found, n=None, stream=None):
    n = queries.numel() if n is None else n
    _check(_lib.bht_find(table, _dptr(queries, None, "queries"), n,
                         _dptr(out_values, None, "out_values"),
                         _dptr(out_found, None, "out_found"), _stream(stream)), "bht_find")


def bht_build64(table, keys, values, n=None, stream=None) -> int:
    n = keys.numel() if n is None else n
    st = _lib.bht_build64(table, _dptr(keys, None, "keys"), _dptr(values, None, "values"), n,
                          _stream(stream))
    if st not in (BHT_OK, BHT_ERR_BUILD_FAILED, BHT_ERR_SENTINEL_KEY):
        _check(st, "bht_build64")
    return st


def bht_find64(table, queries, out_values, out_found, n=None, stream=None):
    n = queries.numel() if n is None else n
    _check(_lib.bht_find64(table, _dptr(queries, None, "queries"), n,
                           _dptr(out_values, None, "out_values"),
                           _dptr(out_found, None, "out_found"), _stream(stream)), "bht_find64")


def bht_build_stats(table):
    """(partitioned, evicted pairs, overflow bucket reads) of the last build."""
    part, ev, pr = _u32(0), _u64(0), _u64(0)
    _check(_lib.bht_build_stats(table, ctypes.byref(part), ctypes.byref(ev), ctypes.byref(pr)),
           "bht_build_stats")
    return bool(part.value), ev.value, pr.value


def bht_build_padding(table):
    """(first-pass, second-pass) padding pairs of the last build's radix passes."""
    p1, p2 = _u64(0), _u64(0)
    _check(_lib.bht_build_padding(table, ctypes.byref(p1), ctypes.byref(p2)), "bht_build_padding")
    return p1.value, p2.value


def bht_params_from_seed(seed: int, scheme, key_bits: int = 32) -> bht_params:
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    p = bht_params()
    _check(_lib.bht_params_from_seed(seed & (2**64 - 1), scheme, key_bits, ctypes.byref(p)),
           "bht_params_from_seed")
    return p


def bht_build_retry(table, keys, values, seed: int, max_attempts: int = 50, n=None, stream=None):
    """Returns (status, builds run)."""
    n = keys.numel() if n is None else n
    attempts = _u32(0)
    st = _lib.bht_build_retry(table, _dptr(keys, None, "keys"), _dptr(values, None, "values"), n,
                              seed & (2**64 - 1), max_attempts, ctypes.byref(attempts),
                              _stream(stream))
    if st not in (BHT_OK, BHT_ERR_BUILD_FAILED, BHT_ERR_SENTINEL_KEY):
        _check(st, "bht_build_retry")
    return st, attempts.value


def bht_build_counted(table, keys, values, probe_total, n=None, stream=None) -> int:
    n = keys.numel() if n is None else n
    st = _lib.bht_build_counted(table, _dptr(keys, None, "keys"), _dptr(values, None, "values"),
                                n, _dptr(probe_total, None, "probe_total"), _stream(stream))
    if st not in (BHT_OK, BHT_ERR_BUILD_FAILED, BHT_ERR_SENTINEL_KEY):
        _check(st, "bht_build_counted")
    return st


def bht_find_counted(table, queries, out_values, out_found, probes, n=None, stream=None):
    n = queries.numel() if n is None else n
    _check(_lib.bht_find_counted(table, _dptr(queries, None, "queries"), n,
                                 _dptr(out_values, None, "out_values"),
                                 _dptr(out_found, None, "out_found"),
                                 _dptr(probes, None, "probes"), _stream(stream)),
           "bht_find_counted")


def bht_get_probe_stats(table):
    """(bucket reads of the last build if it was counted, bucket reads of the
    counted finds since the previous call)."""
    bp, fp = _u64(0), _u64(0)
    _check(_lib.bht_get_probe_stats(table, ctypes.byref(bp), ctypes.byref(fp)),
           "bht_get_probe_stats")
    return bp.value, fp.value


def bht_find64_counted(table, queries, out_values, out_found, probes, n=None, stream=None):
    n = queries.numel() if n is None else n
    _check(_lib.bht_find64_counted(table, _dptr(queries, None, "queries"), n,
                                   _dptr(out_values, None, "out_values"),
                                   _dptr(out_found, None, "out_found"),
                                   _dptr(probes, None, "probes"), _stream(stream)),
           "bht_find64_counted")


def bht_set_tuning(table, tile_width: int = 0, find_schedule=0, grid_blocks: int = 0,
                   build_mode=0, iht_early_exit: bool = False, query_unroll: int = 0):
    if isinstance(find_schedule, str):
        find_schedule = FIND_SCHEDULES[find_schedule]
    if isinstance(build_mode, str):
        build_mode = BUILD_MODES[build_mode]
    tu = bht_tuning(tile_width, find_schedule, grid_blocks, build_mode, int(bool(iht_early_exit)),
                    query_unroll)
    _check(_lib.bht_set_tuning(table, ctypes.byref(tu)), "bht_set_tuning")


def bht_get_tuning(table):
    tu = bht_tuning()
    _check(_lib.bht_get_tuning(table, ctypes.byref(tu)), "bht_get_tuning")
    return (tu.tile_width, tu.find_schedule, tu.grid_blocks, tu.build_mode, tu.iht_early_exit,
            tu.query_unroll)


def bht_enable_timing(table, on: bool = True):
    _check(_lib.bht_enable_timing(table, int(on)), "bht_enable_timing")


def bht_kernel_ms(table):
    b, f = ctypes.c_float(), ctypes.c_float()
    _check(_lib.bht_kernel_ms(table, ctypes.byref(b), ctypes.byref(f)), "bht_kernel_ms")
    return b.value, f.value


def bht_info(table):
    m, b, n, nbytes = _u64(), _u32(), _u64(), _u64()
    _check(_lib.bht_info(table, ctypes.byref(m), ctypes.byref(b), ctypes.byref(n),
                         ctypes.byref(nbytes)), "bht_info")
    return m.value, b.value, n.value, nbytes.value


def bht_download(table):
    import numpy as np
    _, _, _, nbytes = bht_info(table)
    out = np.empty(nbytes // 8, dtype=np.uint64)
    _check(_lib.bht_download(table, ctypes.c_void_p(out.ctypes.data)), "bht_download")
    return out


def bht_upload(table, host_words, n_stored: int):
    import numpy as np
    host_words = np.ascontiguousarray(host_words, dtype=np.uint64)
    _check(_lib.bht_upload(table, ctypes.c_void_p(host_words.ctypes.data), n_stored), "bht_upload")


def bht_device_slots(table) -> int:
    out = ctypes.c_void_p()
    _check(_lib.bht_device_slots(table, ctypes.byref(out)), "bht_device_slots")
    return out.value


def bht_diag_gather(d_buf: int, nbytes: int, n_reads: int, line_bytes: int, seed, sink,
                    stream=None):
    _check(_lib.bht_diag_gather(ctypes.c_void_p(d_buf), nbytes, n_reads, line_bytes, seed,
                                _dptr(sink, None, "sink"), _stream(stream)), "bht_diag_gather")


def bht_diag_cas(d_buf: int, nbytes: int, n_ops: int, seed, sink, stream=None):
    _check(_lib.bht_diag_cas(ctypes.c_void_p(d_buf), nbytes, n_ops, seed,
                             _dptr(sink, None, "sink"), _stream(stream)), "bht_diag_cas")


def bht_diag_stream(d_src: int, d_dst, nbytes: int, sink, stream=None):
    """Streaming ceiling: copy nbytes from d_src to d_dst, or read them when
    d_dst is None (raw device addresses)."""
    _check(_lib.bht_diag_stream(ctypes.c_void_p(d_src),
                                None if d_dst is None else ctypes.c_void_p(d_dst), nbytes,
                                _dptr(sink, None, "sink"), _stream(stream)), "bht_diag_stream")


def bht_hash32(a: int, b: int, k: int, m: int) -> int:
    return int(_lib.bht_hash32(a, b, k, m))


def bht_hash64(a: int, b: int, k: int, m: int) -> int:
    return int(_lib.bht_hash64(a, b, k, m))


def _ptr_of(t):
    if t is None:
        return None
    return t.data_ptr() if hasattr(t, "data_ptr") else int(t)


def _batch_entries(entries):
    arr = (bht_batch_entry * len(entries))()
    for i, (table, keys, vals, queries, out_v, out_f) in enumerate(entries):
        arr[i].table = table.value if isinstance(table, ctypes.c_void_p) else table
        arr[i].d_keys = _ptr_of(keys)
        arr[i].d_values = _ptr_of(vals)
        arr[i].n_keys = 0 if keys is None else keys.numel()
        arr[i].d_queries = _ptr_of(queries)
        arr[i].n_queries = 0 if queries is None else queries.numel()
        arr[i].d_out_values = _ptr_of(out_v)
        arr[i].d_out_found = _ptr_of(out_f)
    return arr


def bht_batch_create(entries, item_size: int = 0):
    """entries: sequence of (table handle, keys, values, queries, out_values,
    out_found) with device tensors (queries/outputs may be None)."""
    arr = _batch_entries(entries)
    out = ctypes.c_void_p()
    _check(_lib.bht_batch_create(arr, len(entries), item_size, ctypes.byref(out)),
           "bht_batch_create")
    return out


def bht_batch_run(batch, stream=None):
    _check(_lib.bht_batch_run(batch, _stream(stream)), "bht_batch_run")


def bht_batch_wait(batch, count: int, stream=None):
    """Returns (overall status, list of per-table statuses)."""
    st = (ctypes.c_int * count)()
    rc = _lib.bht_batch_wait(batch, _stream(stream), st)
    if rc not in (BHT_OK, BHT_ERR_BUILD_FAILED, BHT_ERR_SENTINEL_KEY):
        _check(rc, "bht_batch_wait")
    return rc, list(st)


def bht_batch_destroy(batch):
    _lib.bht_batch_destroy(batch)


def bht_batch_build_find(entries, item_size: int = 0, stream=None):
    """One synchronous batched build and query pass (entries as for
    bht_batch_create).  Returns (overall status, per-table statuses)."""
    arr = _batch_entries(entries)
    st = (ctypes.c_int * len(entries))()
    rc = _lib.bht_batch_build_find(arr, len(entries), item_size, st, _stream(stream))
    if rc not in (BHT_OK, BHT_ERR_BUILD_FAILED, BHT_ERR_SENTINEL_KEY):
        _check(rc, "bht_batch_build_find")
    return rc, list(st)


def bht_find_ctx_create(max_requests: int, max_items: int):
    out = ctypes.c_void_p()
    _check(_lib.bht_find_ctx_create(max_requests, max_items, ctypes.byref(out)),
           "bht_find_ctx_create")
    return out


def bht_multi_find(ctx, requests, item_size: int = 0, stream=None):
    """requests: sequence of (table handle, queries, out_values, out_found)."""
    arr = (bht_find_request * len(requests))()
    for i, (table, q, ov, of) in enumerate(requests):
        arr[i].table = table.value if isinstance(table, ctypes.c_void_p) else table
        arr[i].d_queries = _ptr_of(q)
        arr[i].n = q.numel()
        arr[i].d_out_values = _ptr_of(ov)
        arr[i].d_out_found = _ptr_of(of)
    _check(_lib.bht_multi_find(ctx, arr, len(requests), item_size, _stream(stream)),
           "bht_multi_find")


def bht_find_ctx_destroy(ctx):
    _lib.bht_find_ctx_destroy(ctx)


def bht_status_string(status: int) -> str:
    return _lib.bht_status_string(status).decode()


# ------------------------------------------------------- convenience

class Table:
    """One device table: owns the C handle, takes and returns torch tensors."""

    def __init__(self, capacity_slots: int, bucket_size: int, scheme="bcht", a=(), b=(),
                 key_bits=32, rng_seed=0x9E3779B9, max_chain=128, iht_threshold=0,
                 iht_secondary_b=0, iht_secondary_m=0, tile=None, find_schedule=0,
                 grid_blocks=0, buffer=None, build_mode=0, iht_early_exit=False,
                 query_unroll=0):
        self.params = make_params(a, b, key_bits=key_bits, rng_seed=rng_seed,
                                  max_chain=max_chain, iht_threshold=iht_threshold,
                                  iht_secondary_b=iht_secondary_b,
                                  iht_secondary_m=iht_secondary_m)
        self.key_bits = key_bits
        self.buffer = buffer          # caller-owned device memory kept alive with the table
        if buffer is None:
            self.handle = bht_create(capacity_slots, bucket_size, scheme, self.params)
        else:
            self.handle = bht_create_in(capacity_slots, bucket_size, scheme, self.params, buffer)
        if (tile is not None or find_schedule or grid_blocks or build_mode or iht_early_exit
                or query_unroll):
            bht_set_tuning(self.handle, tile or 0, find_schedule, grid_blocks, build_mode,
                           iht_early_exit, query_unroll)

    def close(self):
        if self.handle:
            bht_destroy(self.handle)
            self.handle = None
        self.buffer = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self):
        return bht_info(self.handle)

    def build(self, keys, values, stream=None) -> int:
        if self.key_bits == 64:
            return bht_build64(self.handle, keys, values, stream=stream)
        return bht_build(self.handle, keys, values, stream=stream)

    def find(self, queries, stream=None):
        import torch
        if self.key_bits == 64:
            out_v = torch.empty(queries.numel(), dtype=torch.int64, device=queries.device)
            out_f = torch.empty(queries.numel(), dtype=torch.uint8, device=queries.device)
            bht_find64(self.handle, queries, out_v, out_f, stream=stream)
        else:
            out_v = torch.empty(queries.numel(), dtype=torch.int32, device=queries.device)
            out_f = torch.empty(queries.numel(), dtype=torch.uint8, device=queries.device)
            bht_find(self.handle, queries, out_v, out_f, stream=stream)
        return out_v, out_f

    def download(self):
        return bht_download(self.handle)

    def upload(self, host_words, n_stored):
        bht_upload(self.handle, host_words, n_stored)
