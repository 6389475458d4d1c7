"""Pins of the CPU oracle to facts other than itself.

Each test checks the oracle against something the paper or mathematics fixes:
hand-derived hash values and congruences, a GF(2) matrix form of the
xorshift generator, the worked example of Fig. 1, brute force, a balls-into-
bins count, textbook cuckoo-hashing thresholds and the paper's printed probe
counts.  Mistakes are planted in layouts (never in the GPU path) to show the
invariant checker catches them.
"""
import json
import os

import numpy as np
import pytest

import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
P = 4294967291
P61 = (1 << 61) - 1


# ----------------------------------------------------------------- hashing

def test_hash32_hand_values():
    # (2*5 + 3) mod p = 13, 13 mod 7 = 6
    assert oracle.hash32(2, 3, 5, 7) == 6
    # a = 1, b = 0 and k < p: the hash is k mod m
    assert oracle.hash32(1, 0, 10, 3) == 1
    assert oracle.hash32(1, 0, 123456789, 1000) == 789
    # k = p: a*p + b is b mod p
    assert oracle.hash32(17, 99, P, 1 << 40) == 99
    # a = b = p - 1, k = 2^32 - 1: (p-1)(2^32-1) + (p-1) = (p-1) 2^32
    # and 2^32 = 5 (mod p), so the residue is -5 mod p = p - 5
    assert oracle.hash32(P - 1, P - 1, 0xFFFFFFFF, 1 << 40) == P - 5
    assert oracle.hash32(P - 1, P - 1, 0xFFFFFFFF, 1000) == (P - 5) % 1000
    # m = 1 puts every key in bucket 0
    assert oracle.hash32(12345, 678, 0xDEADBEEF, 1) == 0


def test_hash32_is_affine_mod_p_then_reduced_mod_m():
    rng = np.random.default_rng(1)
    big = 1 << 40          # m above p: the outer reduction is the identity
    for _ in range(200):
        a = int(rng.integers(1, P))
        c = int(rng.integers(0, P))
        k = int(rng.integers(0, 0xFFFFFFFE))
        h0 = oracle.hash32(a, c, k, big)
        h1 = oracle.hash32(a, c, k + 1, big)
        assert 0 <= h0 < P
        # consecutive keys differ by a modulo p
        assert (h1 - h0 - a) % P == 0
        # the bucket index is the residue reduced modulo m, for any m
        for m in (1, 2, 3, 72818, 18641352, (1 << 31) - 1):
            assert oracle.hash32(a, c, k, m) == h0 % m


def test_hash32_keys_above_p_wrap():
    # keys p .. 2^32 - 2 are congruent to 0 .. 4 (reading of Section VII:
    # the modulus is applied to a*k + b, so such keys share buckets)
    for off in range(4):
        for (a, c, m) in [(3, 7, 1000), (P - 2, 5, 72818)]:
            assert oracle.hash32(a, c, P + off, m) == oracle.hash32(a, c, off, m)


def test_hash32_buckets_are_uniform():
    keys = datagen.unique_keys(1 << 16, seed=3)
    a, c = datagen.hash_constants(3, 1)
    m = 64
    counts = np.bincount(oracle.hash32_many(a[0], c[0], keys, m).astype(np.int64), minlength=m)
    expected = len(keys) / m
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    assert chi2 < 120.0          # 63 degrees of freedom; 99.999% quantile ~ 115


def test_hash64_hand_values():
    assert oracle.hash64(2, 3, 5, 7) == 6
    assert oracle.hash64(1, 0, 10, 3) == 1
    # k = q: a*q + b reduces to b
    assert oracle.hash64(17, 99, P61, 1 << 62) == 99
    # keys above q wrap: 2^64 = 8 (q + 1), so 2^64 - 2 = 8 q + 6 is 6 mod q
    assert oracle.hash64(1, 0, (1 << 64) - 2, 1 << 62) == 6
    rng = np.random.default_rng(2)
    for _ in range(100):
        a = int(rng.integers(1, P61))
        c = int(rng.integers(0, P61))
        k = int(rng.integers(0, 1 << 62))
        h0 = oracle.hash64(a, c, k, 1 << 62)
        h1 = oracle.hash64(a, c, k + 1, 1 << 62)
        assert (h1 - h0 - a) % P61 == 0
        assert oracle.hash64(a, c, k, 9320676) == h0 % 9320676


# ------------------------------------------------------- eviction generator

def _gf2_matrix_shift(left: bool, s: int) -> np.ndarray:
    T = np.zeros((32, 32), dtype=np.uint8)
    for i in range(32):       # output bit i
        j = i - s if left else i + s
        if 0 <= j < 32:
            T[i, j] = 1
    return T


def test_xorshift32_is_marsaglias_linear_map():
    # x -> (I + L^5)(I + R^17)(I + L^13) x over GF(2) (Marsaglia 2003)
    I = np.eye(32, dtype=np.uint8)
    T = ((I + _gf2_matrix_shift(True, 5)) @ (I + _gf2_matrix_shift(False, 17)) % 2
         @ (I + _gf2_matrix_shift(True, 13))) % 2
    rng = np.random.default_rng(5)
    for x in [1, 2463534242] + [int(v) for v in rng.integers(1, 1 << 32, 50)]:
        bits = np.array([(x >> i) & 1 for i in range(32)], dtype=np.uint8)
        y_bits = (T @ bits) % 2
        y = int(sum(int(b) << i for i, b in enumerate(y_bits)))
        assert oracle.xorshift32(x) == y


# ------------------------------------------------------------ worked example

def _mock_params(scheme, fx, **kw):
    h = fx["h"]
    rows = max(int(k) for k in fx["hashes"]) + 1
    mock = np.zeros((rows, h), dtype=np.uint32)
    for k, hv in fx["hashes"].items():
        mock[int(k)] = hv
    return oracle.Params(scheme=scheme, b=fx["b"], m=fx["buckets"], h=h, a=[0] * h, c=[0] * h,
                         mock=mock, **kw)


def _layout(params, initial):
    t = oracle.empty_table(params)
    for bkt, keys in enumerate(initial):
        for s, k in enumerate(keys):
            t[bkt * params.b + s] = ((k + 1000) << 32) | k
    return t


def _bucket_keys(params, t, bkt):
    words = t[bkt * params.b:(bkt + 1) * params.b]
    return [int(w) & 0xFFFFFFFF for w in words if (int(w) & 0xFFFFFFFF) != 0xFFFFFFFF]


def test_fig1b_cuckoo_next_bucket_rule():
    fx = json.load(open(os.path.join(GOLDEN, "fig1_worked_example.json")))["bcht_fig1b"]
    params = _mock_params("bcht", fx)
    for seed in range(1, 20):          # whichever resident is evicted
        t = _layout(params, fx["initial"])
        st, _, probes = oracle.insert32(params, t, fx["insert"], fx["insert"] + 1000, seed)
        assert st == oracle.OK
        assert probes == fx["expect_probes"]
        b2 = _bucket_keys(params, t, fx["expect_bucket_of_new_key"])
        assert fx["insert"] in b2 and len(b2) == 4
        evicted = [k for k in fx["expect_evicted_from"] if k not in b2]
        assert len(evicted) == 1 and evicted[0] in fx["expect_evicted_from"]
        b1 = _bucket_keys(params, t, fx["expect_evicted_to_bucket"])
        assert b1 == fx["initial"][1] + evicted
        assert _bucket_keys(params, t, 0) == fx["initial"][0]
        # the moved pair kept its value
        slot = fx["expect_evicted_to_bucket"] * params.b + len(fx["initial"][1])
        assert int(t[slot]) >> 32 == evicted[0] + 1000


def test_fig1c_power_of_two_least_loaded():
    fx = json.load(open(os.path.join(GOLDEN, "fig1_worked_example.json")))["bp2ht_fig1c"]
    params = _mock_params("bp2ht", fx)
    for case in fx["cases"]:
        t = _layout(params, case["initial"])
        st, _, probes = oracle.insert32(params, t, 7, 1007, 1)
        assert st == oracle.OK and probes == 2
        assert int(t[case["expect_bucket"] * params.b + case["expect_slot"]]) & 0xFFFFFFFF == 7


def test_fig1d_iceberg_threshold_then_secondary():
    fx = json.load(open(os.path.join(GOLDEN, "fig1_worked_example.json")))["iht_fig1d"]
    params = _mock_params("iht", fx, threshold=fx["threshold"])
    for case in fx["cases"]:
        t = _layout(params, case["initial"])
        st, _, _ = oracle.insert32(params, t, case["insert"], case["insert"] + 1000, 1)
        assert st == oracle.OK
        w = int(t[case["expect_bucket"] * params.b + case["expect_slot"]])
        assert w & 0xFFFFFFFF == case["insert"]


# ------------------------------------------------------------- brute force

def test_brute_force_matches_dictionary():
    rng = np.random.default_rng(7)
    for n in [0, 1, 2, 5, 64, 1000]:
        keys = rng.choice(1 << 20, size=n, replace=False).astype(np.uint32)
        vals = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
        q = np.concatenate([keys, rng.integers(0, 1 << 20, 300).astype(np.uint32),
                            np.array([0xFFFFFFFF], dtype=np.uint32)])
        d = dict(zip(keys.tolist(), vals.tolist()))
        v, f = oracle.brute_find32(keys, vals, q)
        for qi, vi, fi in zip(q.tolist(), v.tolist(), f.tolist()):
            if qi in d:
                assert fi == 1 and vi == d[qi]
            else:
                assert fi == 0 and vi == 0xFFFFFFFF


def test_brute_force64_matches_dictionary():
    rng = np.random.default_rng(8)
    keys = rng.choice(1 << 40, size=500, replace=False).astype(np.uint64)
    vals = rng.integers(0, 1 << 63, size=500, dtype=np.uint64)
    q = np.concatenate([keys, rng.integers(0, 1 << 40, 300).astype(np.uint64)])
    d = dict(zip(keys.tolist(), vals.tolist()))
    v, f = oracle.brute_find64(keys, vals, q)
    for qi, vi, fi in zip(q.tolist(), v.tolist(), f.tolist()):
        assert (fi == 1 and vi == d[qi]) if qi in d else (fi == 0 and vi == (1 << 64) - 1)


def test_join_lookup_matches_dictionary():
    """The sort-merge join used for full-size checks answers like a Python
    dictionary: keys spanning all 32 bits (every radix digit), repeated
    queries, the reserved key, empty inputs."""
    rng = np.random.default_rng(9)
    for n, nq in [(0, 10), (1, 0), (1, 5), (7, 100), (5000, 20000), (100000, 300000)]:
        keys = np.unique(rng.integers(0, 0xFFFFFFFF, size=2 * n + 4, dtype=np.uint64))
        keys = rng.permutation(keys)[:n].astype(np.uint32)
        vals = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
        pool = np.concatenate([keys, rng.integers(0, 1 << 32, size=max(n, 8),
                                                   dtype=np.uint64).astype(np.uint32),
                               np.array([0xFFFFFFFF, 0], dtype=np.uint32)])
        q = pool[rng.integers(0, len(pool), size=nq)]
        d = dict(zip(keys.tolist(), vals.tolist()))
        v, f = oracle.join_find32(keys, vals, q)
        ev = np.array([d.get(x, 0xFFFFFFFF) for x in q.tolist()], dtype=np.uint32)
        ef = np.array([x in d for x in q.tolist()], dtype=np.uint8)
        np.testing.assert_array_equal(f, ef)
        np.testing.assert_array_equal(v, ev)


def test_join_lookup64_matches_dictionary():
    rng = np.random.default_rng(10)
    for n, nq in [(0, 10), (3, 50), (20000, 60000)]:
        keys = rng.integers(0, (1 << 64) - 2, size=n, dtype=np.uint64)
        keys = np.unique(keys)
        n = len(keys)
        keys = rng.permutation(keys)
        vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
        pool = np.concatenate([keys, rng.integers(0, 1 << 64, size=max(n, 8), dtype=np.uint64),
                               np.array([(1 << 64) - 1, 0], dtype=np.uint64)])
        q = pool[rng.integers(0, len(pool), size=nq)]
        d = dict(zip(keys.tolist(), vals.tolist()))
        v, f = oracle.join_find64(keys, vals, q)
        ev = np.array([d.get(x, (1 << 64) - 1) for x in q.tolist()], dtype=np.uint64)
        ef = np.array([x in d for x in q.tolist()], dtype=np.uint8)
        np.testing.assert_array_equal(f, ef)
        np.testing.assert_array_equal(v, ev)


# ---------------------------------------------- build + find vs brute force

GRID = [
    # scheme, b, h, lf, n
    ("bcht", 16, 3, 0.9, 4000), ("bcht", 16, 3, 0.97, 4000), ("bcht", 8, 3, 0.9, 3000),
    ("bcht", 4, 3, 0.85, 2000), ("bcht", 2, 3, 0.8, 2000), ("bcht", 32, 3, 0.95, 4000),
    ("bcht", 16, 2, 0.8, 3000), ("cht1", 1, 3, 0.8, 3000), ("cht1", 1, 4, 0.85, 3000),
    ("bp2ht", 16, 2, 0.75, 4000), ("bp2ht", 32, 2, 0.85, 4000), ("bp2ht", 8, 2, 0.6, 2000),
    ("iht", 16, 3, 0.8, 4000), ("iht", 32, 3, 0.88, 4000),
]


@pytest.mark.parametrize("scheme,b,h,lf,n", GRID)
def test_oracle_find_equals_brute_force(scheme, b, h, lf, n):
    ok = 0
    for seed in range(1, 12):
        keys = datagen.unique_keys(n, seed)
        vals = datagen.values(n, seed)
        thr = int(round(0.8 * b)) if scheme == "iht" else 0
        params = oracle.params_for(scheme, n, lf, seed, b=b, h=h, threshold=thr)
        st, table, _ = oracle.build32(params, keys, vals)
        if st != oracle.OK:
            continue           # a failed build is retried with new constants
        ok += 1
        assert oracle.check32(params, table, keys, vals) == (0, "ok")
        q = datagen.mixed_queries(n, 2 * n, 0.5, seed)
        v, f, _, _ = oracle.find32(params, table, q)
        bv, bf = oracle.brute_find32(keys, vals, q)
        np.testing.assert_array_equal(f, bf)
        np.testing.assert_array_equal(v, bv)
        if ok == 3:
            break
    assert ok >= 1


def test_two_level_iceberg_find_equals_brute_force():
    n = 20000
    for seed in range(1, 6):
        keys, vals = datagen.unique_keys(n, seed), datagen.values(n, seed)
        params = oracle.params_for("iht", n, 0.8, seed, b=16, threshold=16)
        params.b2 = 8
        params.m2 = max(1, params.m * 16 // 8 // 8)     # secondary slots = primary / 8
        st, table, _ = oracle.build32(params, keys, vals)
        if st != oracle.OK:
            continue
        assert oracle.check32(params, table, keys, vals) == (0, "ok")
        q = datagen.mixed_queries(n, n, 0.5, seed)
        v, f, probes, per = oracle.find32(params, table, q)
        bv, bf = oracle.brute_find32(keys, vals, q)
        np.testing.assert_array_equal(f, bf)
        np.testing.assert_array_equal(v, bv)
        assert np.all(per[f == 0] == 3)      # no early exit for iceberg
        return
    pytest.fail("no two-level iceberg build succeeded")


def test_oracle_64bit_find_equals_brute_force():
    n = 5000
    for seed in (1, 2):
        keys, vals = datagen.unique_keys64(n, seed), datagen.values64(n, seed)
        params = oracle.params_for("bcht", n, 0.9, seed, b=8, wide=True)
        st, table, _ = oracle.build64(params, keys, vals)
        assert st == oracle.OK
        assert oracle.check64(params, table, keys, vals) == (0, "ok")
        q = datagen.mixed_queries(n, 2 * n, 0.5, seed, wide=True)
        v, f, total, per = oracle.find64(params, table, q)
        assert int(per.sum(dtype=np.int64)) == total
        bv, bf = oracle.brute_find64(keys, vals, q)
        np.testing.assert_array_equal(f, bf)
        np.testing.assert_array_equal(v, bv)


def test_empty_and_single_inputs():
    for scheme in ("bcht", "bp2ht", "iht", "cht1"):
        b = 1 if scheme == "cht1" else 16
        params = oracle.params_for(scheme, 1, 0.5, 1, b=b, threshold=13)
        e = np.zeros(0, dtype=np.uint32)
        st, table, probes = oracle.build32(params, e, e)
        assert st == oracle.OK and probes == 0
        assert np.all(table == oracle.EMPTY64)
        v, f, _, _ = oracle.find32(params, table, np.array([5, 0xFFFFFFFF], dtype=np.uint32))
        assert list(f) == [0, 0] and list(v) == [0xFFFFFFFF, 0xFFFFFFFF]
        st, table, _ = oracle.build32(params, np.array([9], np.uint32), np.array([0xFFFFFFFF], np.uint32))
        assert st == oracle.OK
        v, f, _, _ = oracle.find32(params, table, np.array([9, 10], dtype=np.uint32))
        assert list(f) == [1, 0] and list(v) == [0xFFFFFFFF, 0xFFFFFFFF]


# ------------------------------------------------------ special-case pins

def test_single_hash_cuckoo_is_balls_into_bins():
    # h = 1: an evicted key returns to the same full bucket, so the build
    # succeeds iff no bucket receives more than b keys.
    for seed in range(1, 40):
        n, b = 600, 8
        keys, vals = datagen.unique_keys(n, seed), datagen.values(n, seed)
        params = oracle.params_for("bcht", n, 0.7, seed, b=b, h=1)
        counts = np.bincount(oracle.hash32_many(params.a[0], params.c[0], keys, params.m).astype(np.int64),
                             minlength=params.m)
        st, _, _ = oracle.build32(params, keys, vals)
        assert (st == oracle.OK) == bool(counts.max() <= b)


def test_textbook_cuckoo_threshold_two_hashes():
    # b = 1, h = 2 (Pagh-Rodler) supports load factors below 1/2 only
    n = 1 << 15
    keys, vals = datagen.unique_keys(n, 11), datagen.values(n, 11)
    lo = oracle.params_for("cht1", n, 0.35, 11, b=1, h=2, max_chain=1000)
    hi = oracle.params_for("cht1", n, 0.6, 11, b=1, h=2, max_chain=1000)
    assert oracle.build32(lo, keys, vals)[0] == oracle.OK
    assert oracle.build32(hi, keys, vals)[0] == oracle.FAILED


def test_three_hash_single_slot_below_threshold():
    # b = 1, h = 3: threshold about 0.918 (Section IV-B), LF 0.8 builds
    n = 1 << 15
    successes = 0
    for seed in range(1, 4):
        keys, vals = datagen.unique_keys(n, seed), datagen.values(n, seed)
        params = oracle.params_for("cht1", n, 0.8, seed, b=1, h=3, max_chain=1000)
        successes += oracle.build32(params, keys, vals)[0] == oracle.OK
    assert successes >= 2


def test_forced_failures():
    keys = np.arange(1, 40, dtype=np.uint32)
    vals = keys.copy()
    # every key in one bucket (a = 0, equal offsets), no evictions allowed
    params = oracle.Params(scheme="bcht", b=16, m=8, h=3, a=[0, 0, 0], c=[5, 5, 5], max_chain=0)
    assert oracle.build32(params, keys, vals)[0] == oracle.FAILED
    params.max_chain = 128
    assert oracle.build32(params, keys, vals)[0] == oracle.FAILED
    assert oracle.build32(params, keys[:16], vals[:16])[0] == oracle.OK
    p2 = oracle.Params(scheme="bp2ht", b=16, m=8, h=2, a=[0, 0], c=[5, 5])
    assert oracle.build32(p2, keys, vals)[0] == oracle.FAILED
    ih = oracle.Params(scheme="iht", b=16, m=8, h=3, a=[0, 0, 0], c=[5, 5, 5], threshold=13)
    assert oracle.build32(ih, keys, vals)[0] == oracle.FAILED
    bad = np.array([3, 0xFFFFFFFF], dtype=np.uint32)
    params.max_chain = 128
    assert oracle.build32(params, bad, bad)[0] == oracle.SENTINEL


# ----------------------------------------------------- invariant checker

def _built(seed=3, scheme="bcht", n=3000, lf=0.95, b=16):
    keys, vals = datagen.unique_keys(n, seed), datagen.values(n, seed)
    params = oracle.params_for(scheme, n, lf, seed, b=b, threshold=13)
    st, table, _ = oracle.build32(params, keys, vals)
    assert st == oracle.OK
    return params, table, keys, vals


def test_checker_catches_planted_mistakes():
    params, table, keys, vals = _built()
    assert oracle.check32(params, table, keys, vals)[0] == 0
    occ = np.nonzero((table & np.uint64(0xFFFFFFFF)) != np.uint64(0xFFFFFFFF))[0]
    # I1: a dropped pair
    t = table.copy(); t[occ[0]] = oracle.EMPTY64
    assert oracle.check32(params, t, keys, vals)[0] in (1, 4)
    # I1: a changed value
    t = table.copy(); t[occ[5]] ^= np.uint64(1 << 40)
    assert oracle.check32(params, t, keys, vals)[0] == 1
    # I6: empty key with a value
    empties = np.nonzero(table == np.uint64(oracle.EMPTY64))[0]
    t = table.copy(); t[empties[0]] = np.uint64(0x12345678FFFFFFFF)
    assert oracle.check32(params, t, keys, vals)[0] == 6
    # I2: a pair moved to a bucket none of its hashes names
    t = table.copy()
    src = occ[7]
    k = int(table[src]) & 0xFFFFFFFF
    cands = {int(oracle.hash32(params.a[i], params.c[i], k, params.m)) for i in range(3)}
    dst_bucket = next(bk for bk in range(params.m) if bk not in cands
                      and int(table[bk * 16 + 15]) == oracle.EMPTY64)
    load = int(np.sum((t[dst_bucket * 16:(dst_bucket + 1) * 16] & np.uint64(0xFFFFFFFF)) != np.uint64(0xFFFFFFFF)))
    # move k to the destination; fill the hole by moving the last pair of its bucket
    sb = src // 16
    last = sb * 16 + int(np.sum((t[sb * 16:(sb + 1) * 16] & np.uint64(0xFFFFFFFF)) != np.uint64(0xFFFFFFFF))) - 1
    t[dst_bucket * 16 + load] = table[src]
    t[src] = t[last]
    t[last] = oracle.EMPTY64
    assert oracle.check32(params, t, keys, vals)[0] == 2
    # I4: a hole inside a bucket
    t = table.copy()
    full_b = next(bk for bk in range(params.m) if int(table[bk * 16 + 15]) != oracle.EMPTY64)
    part_b = next(bk for bk in range(params.m) if int(table[bk * 16 + 15]) == oracle.EMPTY64
                  and int(table[bk * 16 + 1]) != oracle.EMPTY64)
    ld = int(np.sum((t[part_b * 16:(part_b + 1) * 16] & np.uint64(0xFFFFFFFF)) != np.uint64(0xFFFFFFFF)))
    t[part_b * 16 + ld] = t[part_b * 16]
    t[part_b * 16] = oracle.EMPTY64
    assert oracle.check32(params, t, keys, vals)[0] == 4
    assert full_b >= 0


def _occupied64(t, b, bucket):
    """Occupied slots of a 64-bit layout's bucket (key words not empty)."""
    keys = t[2 * bucket * b:2 * (bucket + 1) * b:2]
    return int(np.sum(keys != np.uint64(oracle.EMPTY64)))


def test_checker64_catches_planted_mistakes():
    """orc_check64 on a valid serial 64-bit layout, then with one mistake
    planted per copy; each returns the number of the invariant it breaks
    (Section III: every pair stored once with its value, in a candidate
    bucket, buckets filled as a prefix, empty slots wholly empty)."""
    n, b = 3000, 8
    keys, vals = datagen.unique_keys64(n, 5), datagen.values64(n, 5)
    params = oracle.params_for("bcht", n, 0.9, 5, b=b, wide=True)
    st, table, _ = oracle.build64(params, keys, vals)
    assert st == oracle.OK
    assert oracle.check64(params, table, keys, vals) == (0, "ok")
    E = np.uint64(oracle.EMPTY64)
    m = params.m
    loads = [_occupied64(table, b, bk) for bk in range(m)]
    part = [bk for bk in range(m) if 1 < loads[bk] < b]
    assert part, "the layout has no partly filled bucket"
    # I1: a dropped pair (the last one of a bucket, so no hole appears)
    bk = part[0]
    s = bk * b + loads[bk] - 1
    t = table.copy(); t[2 * s] = E; t[2 * s + 1] = E
    assert oracle.check64(params, t, keys, vals)[0] == 1
    # I1: a changed value word
    t = table.copy(); t[2 * (bk * b) + 1] ^= np.uint64(1 << 63)
    assert oracle.check64(params, t, keys, vals)[0] == 1
    # I1: a duplicated key (one stored pair copied over another)
    occ = [bb * b + i for bb in range(m) for i in range(loads[bb])]
    t = table.copy(); t[2 * occ[1]:2 * occ[1] + 2] = table[2 * occ[0]:2 * occ[0] + 2]
    assert oracle.check64(params, t, keys, vals)[0] == 1
    # I1: a slot left holding the slot-lock key (2^64 - 2) in place of its key
    t = table.copy(); t[2 * occ[3]] = np.uint64(oracle.EMPTY64 - 1)
    assert oracle.check64(params, t, keys, vals)[0] == 1
    # I6: the empty key with a value word
    empty = next(bb * b + loads[bb] for bb in range(m) if loads[bb] < b)
    t = table.copy(); t[2 * empty + 1] = np.uint64(12345)
    assert oracle.check64(params, t, keys, vals)[0] == 6
    # I4: a hole inside a bucket
    t = table.copy()
    ld = loads[bk]
    t[2 * (bk * b + ld):2 * (bk * b + ld) + 2] = t[2 * bk * b:2 * bk * b + 2]
    t[2 * bk * b] = E; t[2 * bk * b + 1] = E
    assert oracle.check64(params, t, keys, vals)[0] == 4
    # I2: a pair moved to a bucket none of its hashes names (Python big-int
    # hashes, independent of the oracle's)
    src = occ[7]
    k = int(table[2 * src])
    cands = {((params.a[i] * k + params.c[i]) % P61) % m for i in range(3)}
    dst = next(bb for bb in range(m) if bb not in cands and loads[bb] < b)
    t = table.copy()
    t[2 * (dst * b + loads[dst]):2 * (dst * b + loads[dst]) + 2] = table[2 * src:2 * src + 2]
    sb = src // b
    last = sb * b + loads[sb] - 1
    t[2 * src:2 * src + 2] = t[2 * last:2 * last + 2]
    t[2 * last] = E; t[2 * last + 1] = E
    assert oracle.check64(params, t, keys, vals)[0] == 2


@pytest.mark.parametrize("via", [1, 2])
def test_checker64_catches_early_exit_violation(via):
    """A key stored in the bucket of hash `via` while the bucket of hash 0
    has room breaks I3, the property early-exit lookups rely on."""
    b, m = 8, 5
    a, c = datagen.hash_constants64(9, 3)
    params = oracle.Params(scheme="bcht", b=b, m=m, h=3, a=a, c=c)

    def H(i, k):
        return ((a[i] * k + c[i]) % P61) % m

    k = next(k for k in range(1, 1 << 20)
             if len({H(0, k), H(1, k), H(2, k)}) == 3)
    t = oracle.empty_table(params, wide=True)
    slot = H(via, k) * b
    t[2 * slot] = np.uint64(k); t[2 * slot + 1] = np.uint64(77)
    keys = np.array([k], dtype=np.uint64)
    vals = np.array([77], dtype=np.uint64)
    assert oracle.check64(params, t, keys, vals)[0] == 3
    # the same key in its first bucket is valid
    t = oracle.empty_table(params, wide=True)
    slot = H(0, k) * b
    t[2 * slot] = np.uint64(k); t[2 * slot + 1] = np.uint64(77)
    assert oracle.check64(params, t, keys, vals) == (0, "ok")


def test_checker_catches_early_exit_violation():
    # key 1 sits in its second bucket while its first has room (I3)
    mock = np.array([[0, 0, 0], [0, 1, 2], [0, 1, 2]], dtype=np.uint32)
    params = oracle.Params(scheme="bcht", b=2, m=3, h=3, a=[0] * 3, c=[0] * 3, mock=mock)
    keys = np.array([1, 2], dtype=np.uint32)
    vals = np.array([10, 20], dtype=np.uint32)
    t = oracle.empty_table(params)
    t[0] = (20 << 32) | 2        # bucket 0: [2, empty]
    t[2] = (10 << 32) | 1        # bucket 1: [1, empty]
    assert oracle.check32(params, t, keys, vals)[0] == 3
    # and the early-exit query then misses key 1: the reason I3 matters
    v, f, _, _ = oracle.find32(params, t, keys)
    assert list(f) == [0, 1]


def test_checker_catches_iceberg_threshold_violation():
    mock = np.array([[0, 1, 2], [0, 1, 2]], dtype=np.uint32)
    params = oracle.Params(scheme="iht", b=4, m=3, h=3, a=[0] * 3, c=[0] * 3, mock=mock, threshold=3)
    keys = np.array([1], dtype=np.uint32)
    vals = np.array([10], dtype=np.uint32)
    t = oracle.empty_table(params)
    t[4] = (10 << 32) | 1        # in secondary bucket 1 while primary 0 is empty
    assert oracle.check32(params, t, keys, vals)[0] == 5


# -------------------------------------------------- probe counts (Section VII-E)

def _probe_stats(scheme, n, lf, b, h=None, threshold=0, seeds=range(1, 8)):
    for seed in seeds:
        keys, vals = datagen.unique_keys(n, seed), datagen.values(n, seed)
        params = oracle.params_for(scheme, n, lf, seed, b=b, h=h, threshold=threshold)
        st, table, ins = oracle.build32(params, keys, vals)
        if st != oracle.OK:
            continue
        pos = datagen.positive_queries(n, seed)
        neg = datagen.negative_keys(n, n, seed)
        _, _, pp, per_pos = oracle.find32(params, table, pos)
        _, _, pn, _ = oracle.find32(params, table, neg)
        return dict(params=params, table=table, keys=keys, vals=vals, insert=ins / n,
                    pos=pp / n, neg=pn / n, per_pos=per_pos, pos_q=pos)
    pytest.fail("no successful build")


PC = json.load(open(os.path.join(GOLDEN, "paper_probe_counts.json")))


def test_positive_probes_equal_bucket_rank_from_layout():
    s = _probe_stats("bcht", 1 << 16, 0.95, 16)
    params, table = s["params"], s["table"]
    keys_at = (table & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    slot_of = {int(k): i for i, k in enumerate(keys_at) if k != 0xFFFFFFFF}
    # probes of a positive query = 1 + index of the hash that names its bucket
    hv = [oracle.hash32_many(params.a[i], params.c[i], s["pos_q"], params.m) for i in range(3)]
    expect = np.empty(len(s["pos_q"]), dtype=np.int64)
    for j, q in enumerate(s["pos_q"].tolist()):
        bkt = slot_of[q] // 16
        expect[j] = 1 + next(i for i in range(3) if int(hv[i][j]) == bkt)
    np.testing.assert_array_equal(s["per_pos"].astype(np.int64), expect)


def test_bcht_probe_counts_match_paper():
    c = PC["bcht"]
    s90 = _probe_stats("bcht", 1 << 18, 0.9, 16)
    assert abs(s90["insert"] - c["insert_b16_lf090"]["value"]) <= 0.06
    s8 = _probe_stats("bcht", 1 << 17, 0.9, 8)
    assert abs(s8["insert"] - c["insert_b8_lf090"]["value"]) <= 0.08
    s32 = _probe_stats("bcht", 1 << 17, 0.9, 32)
    assert abs(s32["insert"] - c["insert_b32_lf090"]["value"]) <= 0.05
    s99 = _probe_stats("bcht", 1 << 18, 0.99, 16)
    assert 1.2 <= s99["insert"] <= c["insert_b16_lf099_max"]["value"] * 1.1
    assert s99["pos"] <= c["positive_b16_max"]["value"] * 1.05
    assert abs(s99["neg"] - c["negative_b16_lf099"]["value"]) <= 0.15


def test_negative_probes_follow_full_bucket_fraction():
    # independent hashes: a negative query reads 1 + f + f^2 buckets on
    # average, f being the fraction of full buckets
    s = _probe_stats("bcht", 1 << 18, 0.97, 16)
    t = s["table"].reshape(-1, 16)
    f = float(np.mean((t[:, 15] & np.uint64(0xFFFFFFFF)) != np.uint64(0xFFFFFFFF)))
    assert abs(s["neg"] - (1 + f + f * f)) < 0.02


def test_single_slot_cuckoo_probe_counts_match_paper():
    s = _probe_stats("cht1", 1 << 17, 0.9, 1, h=4)
    assert abs(s["insert"] - PC["bcht"]["insert_b1h4_lf090"]["value"]) <= 0.3


def test_power_of_two_probe_counts_match_paper():
    c = PC["bp2ht"]
    s = _probe_stats("bp2ht", 1 << 17, 0.9, 32)
    assert s["insert"] == c["insert"]["value"]
    assert s["neg"] == c["negative"]["value"]
    assert abs(s["pos"] - c["positive"]["value"]) <= 0.05
    assert abs((s["pos"] + s["neg"]) / 2 - c["half_positive"]["value"]) <= 0.05


def test_iceberg_probe_counts_match_paper():
    c = PC["iht"]
    n = 1 << 17
    for pct, ins, pos in zip(c["b16_lf086_thresholds_percent"], c["b16_lf086_insert"]["value"],
                             c["b16_lf086_positive"]["value"]):
        # threshold = floor(pct * b / 100) keys and "primary while load < t"
        # reproduce all eight printed values to within 0.02; the listing's
        # "load > t" comparison or rounding up would be off by over 0.1
        t = (16 * pct) // 100
        s = _probe_stats("iht", n, 0.86, 16, threshold=t)
        assert s["neg"] == c["negative"]["value"]
        assert abs(s["insert"] - ins) <= 0.03, (pct, s["insert"], ins)
        assert abs(s["pos"] - pos) <= 0.03, (pct, s["pos"], pos)


@pytest.mark.parametrize("b2,t,lf,both", [(0, 13, 0.86, True), (0, 6, 0.8, False),
                                           (8, 16, 0.8, True)])
def test_iceberg_early_exit_find_equals_brute_force(b2, t, lf, both):
    """Early exit after a primary below the threshold loses no key (results
    equal the plain definition), leaves positive probe counts unchanged, and
    cuts a negative query to one probe exactly when its primary holds fewer
    than t keys."""
    n = 20000
    for seed in range(1, 8):
        keys, vals = datagen.unique_keys(n, seed), datagen.values(n, seed)
        params = oracle.params_for("iht", n, lf, seed, b=16, threshold=t)
        if b2:
            params.b2 = b2
            params.m2 = max(1, params.m * 16 // 8 // b2)
        st, table, _ = oracle.build32(params, keys, vals)
        if st == oracle.OK:
            break
    else:
        pytest.fail("no iceberg build succeeded")
    q = datagen.mixed_queries(n, 2 * n, 0.5, seed)
    _, _, _, per_plain = oracle.find32(params, table, q)
    params.early_exit = True
    v, f, _, per = oracle.find32(params, table, q)
    bv, bf = oracle.brute_find32(keys, vals, q)
    np.testing.assert_array_equal(f, bf)
    np.testing.assert_array_equal(v, bv)
    np.testing.assert_array_equal(per[f == 1], per_plain[f == 1])
    prim = oracle.hash32_many(params.a[0], params.c[0], q, params.m).astype(np.int64)
    loads = (table[:params.m * 16].reshape(-1, 16) & np.uint64(0xFFFFFFFF)) != np.uint64(0xFFFFFFFF)
    below = loads.sum(axis=1)[prim] < t
    neg = f == 0
    assert np.all(per[neg & below] == 1) and np.all(per[neg & ~below] == 3)
    assert (neg & ~below).any()
    if both:        # a low threshold leaves (almost) no primary below it
        assert (neg & below).any()


# ------------------------------------------- load-balanced cuckoo table

@pytest.mark.parametrize("b,h,lf", [(16, 3, 0.9), (16, 3, 0.97), (16, 2, 0.9), (8, 3, 0.9),
                                    (32, 2, 0.95), (16, 4, 0.98)])
def test_load_balanced_cuckoo_find_equals_brute_force(b, h, lf):
    """Layouts satisfy the invariants that hold without early exit, lookups
    equal the plain definition, a negative query reads all h buckets, and
    insertion reads h buckets per placement attempt."""
    n = 20000
    s = _probe_stats("bcht_lb", n, lf, b, h=h)
    params, table, keys, vals = s["params"], s["table"], s["keys"], s["vals"]
    assert oracle.check32(params, table, keys, vals) == (0, "ok")
    q = datagen.mixed_queries(n, 2 * n, 0.5, 3)
    v, f, _, per = oracle.find32(params, table, q)
    bv, bf = oracle.brute_find32(keys, vals, q)
    np.testing.assert_array_equal(f, bf)
    np.testing.assert_array_equal(v, bv)
    assert np.all(per[f == 0] == h)
    assert s["neg"] == h
    ins = int(round(s["insert"] * n))
    assert ins >= h * n and ins % h == 0


def test_load_balanced_two_hashes_equals_power_of_two_without_evictions():
    """With two hashes and no bucket pair ever full, the load-balanced rule
    (least loaded, ties to H0) is the power-of-two rule: both serial builds
    give the same layout, word for word, though written separately."""
    n = 30000
    keys, vals = datagen.unique_keys(n, 5), datagen.values(n, 5)
    lb = oracle.params_for("bcht_lb", n, 0.7, 5, b=16, h=2)
    p2 = oracle.params_for("bp2ht", n, 0.7, 5, b=16)
    assert lb.a == p2.a and lb.c == p2.c and lb.m == p2.m
    st1, t1, ins1 = oracle.build32(lb, keys, vals)
    st2, t2, ins2 = oracle.build32(p2, keys, vals)
    assert st1 == st2 == oracle.OK and ins1 == ins2 == 2 * n
    np.testing.assert_array_equal(t1, t2)


def test_load_balanced_eviction_fires_and_stays_valid():
    """Past the two-choice limit the load-balanced table must evict (insert
    probes above h per key) and its layout stays valid; plain power-of-two
    fails at the same load."""
    n = 1 << 16
    keys, vals = datagen.unique_keys(n, 6), datagen.values(n, 6)
    p2 = oracle.params_for("bp2ht", n, 0.95, 6, b=8)
    assert oracle.build32(p2, keys, vals)[0] == oracle.FAILED
    lb = oracle.params_for("bcht_lb", n, 0.95, 6, b=8, h=2)
    st, table, ins = oracle.build32(lb, keys, vals)
    assert st == oracle.OK and ins > 2 * n
    assert oracle.check32(lb, table, keys, vals) == (0, "ok")
