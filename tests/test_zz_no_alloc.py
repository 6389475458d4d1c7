"""The no-allocation build (bht_build_async_noalloc) against the build with a
caller workspace (bht_build_async_in) through the C ABI.

Two calls in a row on the library's fixed per-GPU array, the second with a
smaller input: each layout passes the oracle's invariant checker and every
lookup equals the workspace build's and the plain lookup definition (brute
force), bit for bit.  A build needing more than the array is refused."""
import numpy as np
import pytest

import datagen
import oracle
from tests._util import dev, host_u32, host_u8

pytestmark = pytest.mark.gpu


def bht():
    import paper_2108_07232_amd
    return paper_2108_07232_amd


def make_table(params):
    B = bht()
    return B.Table(params.m * params.b, params.b, params.scheme, params.a, params.c,
                   rng_seed=params.rng_seed, max_chain=params.max_chain)


def lookups(t, q):
    import torch
    v, f = t.find(dev(q))
    torch.cuda.synchronize()
    return host_u32(v), host_u8(f)


def test_noalloc_matches_workspace_build_twice():
    import torch
    B = bht()
    for n, seed in ((1 << 22, 41), (300007, 42)):
        print("no-alloc build: %d pairs, seed %d" % (n, seed), flush=True)
        keys, vals = datagen.unique_keys(n, seed), datagen.values(n, seed)
        params = oracle.params_for("bcht", n, 0.9, seed)
        q = datagen.mixed_queries(n, n, 0.5, seed)
        dk, dv = dev(keys), dev(vals)

        ref = make_table(params)
        ws = torch.empty(B.bht_build_workspace_bytes(ref.handle, n), dtype=torch.uint8,
                         device="cuda")
        B.bht_build_async_in(ref.handle, dk, dv, ws)
        assert B.bht_build_wait(ref.handle) == B.BHT_OK
        rv, rf = lookups(ref, q)

        t = make_table(params)
        st = B.bht_build_async_noalloc(t.handle, dk, dv)
        assert st == B.BHT_OK, B.bht_status_string(st)
        assert B.bht_build_wait(t.handle) == B.BHT_OK
        assert B.bht_build_stats(t.handle)[0] == 1          # the partitioned path ran
        code, msg = oracle.check32(params, t.download(), keys, vals)
        assert code == 0, msg
        v, f = lookups(t, q)
        np.testing.assert_array_equal(f, rf)
        np.testing.assert_array_equal(v, rv)
        ev, ef = oracle.brute_find32(keys, vals, q)
        np.testing.assert_array_equal(f, ef)
        np.testing.assert_array_equal(v, ev)
        t.close()
        ref.close()
        del ws, dk, dv


def test_noalloc_small_and_oversize():
    B = bht()
    # a small build takes the concurrent kernel, which needs no workspace
    n = 5000
    keys, vals = datagen.unique_keys(n, 43), datagen.values(n, 43)
    params = oracle.params_for("bcht", n, 0.9, 43)
    t = make_table(params)
    assert B.bht_build_async_noalloc(t.handle, dev(keys), dev(vals)) == B.BHT_OK
    assert B.bht_build_wait(t.handle) == B.BHT_OK
    code, msg = oracle.check32(params, t.download(), keys, vals)
    assert code == 0, msg
    t.close()
    # a build whose workspace exceeds the fixed array is refused before any work
    n = B.bht_build_noalloc_max_bytes() // 8
    params = oracle.params_for("bcht", n, 0.9, 44)
    t = make_table(params)
    keys = datagen.unique_keys(n, 44)
    dk = dev(keys)
    assert B.bht_build_async_noalloc(t.handle, dk, dk) == B.BHT_ERR_CAPACITY
    t.close()
