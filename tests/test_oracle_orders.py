"""The insertion orders the partitioned GPU builds realise, run through the
serial oracle (Section III: a bulk build takes an unordered list, so any
order of the same pairs is a valid build).  Cuckoo: every pair whose first
bucket still has room, then the pairs that meet a full first bucket.
Iceberg: every pair whose primary holds fewer than t pairs, then the rest.
Each order gives a layout the invariant checker accepts and the same
lookup results as the input order, and the number of pairs that leave their
first bucket / primary is the overflow sum max(0, X_j - cap)."""
import numpy as np
import pytest

import datagen
import oracle


def first_come_order(h0, cap):
    """Indices of pairs whose bucket h0 has fewer than cap earlier pairs (in
    input order), followed by the others."""
    seen = {}
    first, rest = [], []
    for i, h in enumerate(h0.tolist()):
        c = seen.get(h, 0)
        (first if c < cap else rest).append(i)
        seen[h] = c + 1
    return np.array(first + rest, dtype=np.int64), len(rest)


def build_ok(p, keys, vals):
    st, table, _ = oracle.build32(p, keys, vals)
    return st, table


@pytest.mark.parametrize("b,lf,n", [(16, 0.9, 20000), (8, 0.85, 12000), (1, 0.8, 8000)])
def test_cuckoo_first_bucket_order(b, lf, n):
    keys, vals = datagen.unique_keys(n, 61), datagen.values(n, 61)
    scheme = "cht1" if b == 1 else "bcht"
    for s in range(10):
        p = oracle.params_for(scheme, n, lf, 6100 + s, b=b)
        st, t_in = build_ok(p, keys, vals)
        if st != oracle.OK:
            continue
        h0 = oracle.hash32_many(p.a[0], p.c[0], keys, p.m).astype(np.int64)
        idx, sent = first_come_order(h0, b)
        counts = np.bincount(h0, minlength=p.m)
        assert sent == int(np.maximum(counts - b, 0).sum())
        st2, t_ord = build_ok(p, keys[idx], vals[idx])
        if st2 != oracle.OK:
            continue
        assert oracle.check32(p, t_ord, keys, vals)[0] == 0
        q = datagen.mixed_queries(n, 2 * n, 0.5, 61)
        v1, f1, _, _ = oracle.find32(p, t_in, q)
        v2, f2, _, _ = oracle.find32(p, t_ord, q)
        np.testing.assert_array_equal(f1, f2)
        np.testing.assert_array_equal(v1, v2)
        bv, bf = oracle.brute_find32(keys, vals, q)
        np.testing.assert_array_equal(f2, bf)
        np.testing.assert_array_equal(v2, bv)
        return
    pytest.fail("no seed built in both orders")


@pytest.mark.parametrize("b2,t,lf,n", [(0, 13, 0.85, 20000), (8, 16, 0.8, 20000), (0, 8, 0.7, 10000)])
def test_iceberg_primary_first_order(b2, t, lf, n):
    keys, vals = datagen.unique_keys(n, 62), datagen.values(n, 62)
    for s in range(10):
        p = oracle.params_for("iht", n, lf, 6200 + s, b=16)
        if b2:
            cap = datagen.capacity_for(n, lf)
            p.m = max(4, int(np.ceil(cap / (16 + 16 / 8.0))))
            p.b2 = b2
            p.m2 = max(1, p.m * 16 // 8 // b2)
        p.threshold = t
        st, t_in = build_ok(p, keys, vals)
        if st != oracle.OK:
            continue
        hp = oracle.hash32_many(p.a[0], p.c[0], keys, p.m).astype(np.int64)
        idx, sent = first_come_order(hp, t)
        counts = np.bincount(hp, minlength=p.m)
        assert sent == int(np.maximum(counts - t, 0).sum())
        st2, t_ord = build_ok(p, keys[idx], vals[idx])
        if st2 != oracle.OK:
            continue
        # includes the threshold invariant: a secondary key's primary holds >= t
        assert oracle.check32(p, t_ord, keys, vals)[0] == 0
        q = datagen.mixed_queries(n, 2 * n, 0.5, 62)
        v2, f2, _, _ = oracle.find32(p, t_ord, q)
        bv, bf = oracle.brute_find32(keys, vals, q)
        np.testing.assert_array_equal(f2, bf)
        np.testing.assert_array_equal(v2, bv)
        return
    pytest.fail("no seed built in both orders")
