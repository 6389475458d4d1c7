"""The schedules of the partitioned GPU builds, replayed step by step with
the serial oracle (Section III: a bulk build takes an unordered list; the
cuckoo insertion of Section III-A is a sequence of bucket visits, each
ending in a claim of slot = load or an exchange with a random resident).

Cuckoo (deferred victims): every pair whose first bucket still has room
claims its slot; then every pair that meets a full first bucket exchanges
itself with a random resident there; then each evicted pair continues its
insertion from the bucket it left.  The GPU runs the last phase's chains
concurrently (Section V's concurrent insertion); here they run one after
another.  Iceberg: every pair whose primary holds fewer than t pairs, then
the rest through the secondary step.  Each schedule gives a layout the
invariant checker accepts and the lookups of the plain definition, and the
number of pairs that leave their first bucket / primary is the overflow sum
max(0, X_j - cap)."""
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


def deferred_victim_build(p, keys, vals, rng):
    """The partitioned cuckoo build's schedule through the serial oracle.
    Returns (status, table, pairs that met a full first bucket)."""
    table = oracle.empty_table(p)
    h0 = oracle.hash32_many(p.a[0], p.c[0], keys, p.m).astype(np.int64)
    idx, sent = first_come_order(h0, p.b)
    first, rest = idx[:len(idx) - sent], idx[len(idx) - sent:]
    for i in first.tolist():                 # claims in first buckets with room
        st, rng, probes = oracle.insert32(p, table, int(keys[i]), int(vals[i]), rng)
        assert st == oracle.OK and probes == 1
    victims = []
    for i in rest.tolist():                  # on-chip exchanges in full first buckets
        st, rng, ek, ev = oracle.exchange32(p, table, int(keys[i]), int(vals[i]), rng)
        assert st == oracle.OK
        victims.append((ek, ev, int(h0[i])))
    for ek, ev, bucket in victims:           # the victims' chains
        st, rng, _ = oracle.continue32(p, table, ek, ev, bucket, 1, rng)
        if st != oracle.OK:
            return st, table, sent
    return oracle.OK, table, sent


@pytest.mark.parametrize("b,lf,n", [(16, 0.9, 20000), (16, 0.97, 20000), (8, 0.85, 12000),
                                    (1, 0.8, 8000)])
def test_cuckoo_deferred_victim_schedule(b, lf, n):
    keys, vals = datagen.unique_keys(n, 63), datagen.values(n, 63)
    scheme = "cht1" if b == 1 else "bcht"
    for s in range(10):
        p = oracle.params_for(scheme, n, lf, 6300 + s, b=b)
        st, table, sent = deferred_victim_build(p, keys, vals, p.rng_seed)
        if st != oracle.OK:
            continue
        h0 = oracle.hash32_many(p.a[0], p.c[0], keys, p.m).astype(np.int64)
        assert sent == int(np.maximum(np.bincount(h0, minlength=p.m) - b, 0).sum())
        assert sent > 0
        assert oracle.check32(p, table, keys, vals) == (0, "ok")
        q = datagen.mixed_queries(n, 2 * n, 0.5, 63)
        v, f, _, _ = oracle.find32(p, table, q)
        bv, bf = oracle.brute_find32(keys, vals, q)
        np.testing.assert_array_equal(f, bf)
        np.testing.assert_array_equal(v, bv)
        return
    pytest.fail("no seed built with the deferred-victim schedule")


def test_exchange_and_continue_compose_to_one_insertion():
    """Inserting a pair whose first bucket is full equals its exchange
    followed by the evicted pair's continuation, slot for slot (same
    generator draws), and the split refuses a first bucket with room."""
    n = 3000
    keys, vals = datagen.unique_keys(n + 200, 64), datagen.values(n + 200, 64)
    p = oracle.params_for("bcht", n, 0.95, 64)
    st, base, _ = oracle.build32(p, keys[:n], vals[:n])
    assert st == oracle.OK
    h0 = oracle.hash32_many(p.a[0], p.c[0], keys, p.m).astype(np.int64)
    loads = [(base[bk * 16:(bk + 1) * 16] != np.uint64(oracle.EMPTY64)).sum()
             for bk in range(p.m)]
    done_full = done_room = False
    for i in range(n, n + 200):
        k, v, bk = int(keys[i]), int(vals[i]), int(h0[i])
        if loads[bk] == 16 and not done_full:
            t1 = base.copy()
            st1, r1, _ = oracle.insert32(p, t1, k, v, 12345)
            t2 = base.copy()
            st2, r2, ek, ev = oracle.exchange32(p, t2, k, v, 12345)
            assert st2 == oracle.OK
            st3, r3, _ = oracle.continue32(p, t2, ek, ev, bk, 1, r2)
            assert st1 == st3 == oracle.OK and r1 == r3
            np.testing.assert_array_equal(t1, t2)
            done_full = True
        elif loads[bk] < 16 and not done_room:
            t2 = base.copy()
            assert oracle.exchange32(p, t2, k, v, 1)[0] == oracle.BADARG
            np.testing.assert_array_equal(t2, base)
            done_room = True
    assert done_full and done_room


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
