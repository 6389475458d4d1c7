"""GPU parity of the 64-bit-key bucketed cuckoo table (16-byte slots, 8 per
128-byte bucket): layouts checked with the oracle's invariant checker,
lookups bit-exact against brute force."""
import numpy as np
import pytest

import datagen
import oracle
from tests._util import dev, host_u64, host_u8

pytestmark = pytest.mark.gpu


def build(n, lf, seed, tries=10):
    import paper_2108_07232_amd as bht
    keys, vals = datagen.unique_keys64(n, seed), datagen.values64(n, seed)
    for s in range(tries):
        p = oracle.params_for("bcht", n, lf, seed * 100 + s, b=8, wide=True)
        t = bht.Table(p.m * p.b, 8, "bcht", p.a, p.c, key_bits=64, rng_seed=p.rng_seed,
                      max_chain=p.max_chain)
        st = t.build(dev(keys), dev(vals))
        if st == bht.BHT_OK:
            return t, p, keys, vals
        assert st == bht.BHT_ERR_BUILD_FAILED, bht.bht_status_string(st)
        t.close()
    pytest.fail("no successful 64-bit build")


def check(t, keys, vals, q):
    import torch
    v, f = t.find(dev(q))
    torch.cuda.synchronize()
    bv, bf = oracle.brute_find64(keys, vals, q)
    np.testing.assert_array_equal(host_u8(f), bf)
    np.testing.assert_array_equal(host_u64(v), bv)


@pytest.mark.parametrize("n,lf", [(1 << 20, 0.9), (1 << 16, 0.95), (50001, 0.85), (1000, 0.9),
                                  (40, 0.9), (3000, 0.97)])
def test_wide_build_invariants_and_find(n, lf):
    t, p, keys, vals = build(n, lf, 3)
    layout = t.download()
    code, msg = oracle.check64(p, layout, keys, vals)
    assert code == 0, msg
    for frac in (1.0, 0.5, 0.0):
        check(t, keys, vals, datagen.mixed_queries(n, n, frac, 3, wide=True))
    t.close()


def test_wide_find_on_oracle_layout():
    n = 30000
    keys, vals = datagen.unique_keys64(n, 4), datagen.values64(n, 4)
    p = oracle.params_for("bcht", n, 0.9, 4, b=8, wide=True)
    st, layout, _ = oracle.build64(p, keys, vals)
    assert st == oracle.OK
    import paper_2108_07232_amd as bht
    t = bht.Table(p.m * p.b, 8, "bcht", p.a, p.c, key_bits=64)
    t.upload(layout, n)
    check(t, keys, vals, datagen.mixed_queries(n, 2 * n, 0.5, 4, wide=True))
    edge = np.array([0, 1, (1 << 64) - 1, (1 << 64) - 2, int(keys[0]), (1 << 61) - 1, 1 << 61],
                    dtype=np.uint64)
    check(t, keys, vals, edge)
    t.close()


def test_wide_reserved_keys_rejected_and_contention():
    import paper_2108_07232_amd as bht
    n = 1000
    keys, vals = datagen.unique_keys64(n, 5), datagen.values64(n, 5)
    p = oracle.params_for("bcht", n, 0.9, 5, b=8, wide=True)
    t = bht.Table(p.m * p.b, 8, "bcht", p.a, p.c, key_bits=64)
    for bad in ((1 << 64) - 1, (1 << 64) - 2):
        k = keys.copy()
        k[17] = bad
        assert t.build(dev(k), dev(vals)) == bht.BHT_ERR_SENTINEL_KEY
    t.close()
    # tiny tables: every slot contended by many lanes at once
    for n, lf in [(15, 1.0), (200, 0.97), (2000, 0.98)]:
        t, p, keys, vals = build(n, lf, 6, tries=40)
        assert oracle.check64(p, t.download(), keys, vals)[0] == 0
        check(t, keys, vals, datagen.mixed_queries(n, 4 * n, 0.5, 6, wide=True))
        t.close()
