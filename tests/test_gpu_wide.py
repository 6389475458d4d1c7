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


def build_mode64(n, lf, seed, mode, tries=8):
    import paper_2108_07232_amd as bht
    keys, vals = datagen.unique_keys64(n, seed), datagen.values64(n, seed)
    for s in range(tries):
        p = oracle.params_for("bcht", n, lf, seed * 100 + s, b=8, wide=True)
        t = bht.Table(p.m * p.b, 8, "bcht", p.a, p.c, key_bits=64, rng_seed=p.rng_seed,
                      max_chain=p.max_chain, build_mode=mode)
        st = t.build(dev(keys), dev(vals))
        if st == bht.BHT_OK:
            return t, p, keys, vals
        assert st == bht.BHT_ERR_BUILD_FAILED, bht.bht_status_string(st)
        t.close()
    pytest.fail("no successful 64-bit %s build" % mode)


def plan_levels64(m):
    """Radix passes the library plans for m buckets of 8 16-byte slots."""
    return 1 if -(-m // 512) <= 1024 else 2


@pytest.mark.parametrize("n,lf", [(1 << 20, 0.9), (100003, 0.95), (50000, 0.98), (3000, 0.9),
                                  (1, 0.5), (9, 0.9), (1 << 18, 0.85)])
def test_wide_partitioned_build(n, lf):
    """Partitioned 64-bit build (radix passes, placement in LDS with evictions
    in ranked rounds, overflow insertion): valid layout, exact lookups, and
    the on-chip eviction count equals the first-bucket overflow."""
    import paper_2108_07232_amd as bht
    print("wide partitioned n=%d lf=%g" % (n, lf), flush=True)
    t, p, keys, vals = build_mode64(n, lf, 7, "partitioned")
    code, msg = oracle.check64(p, t.download(), keys, vals)
    assert code == 0, msg
    check(t, keys, vals, datagen.mixed_queries(n, max(2 * n, 64), 0.5, 7, wide=True))
    h0 = oracle.hash64_many(p.a[0], p.c[0], keys, p.m)
    counts = np.bincount(h0.astype(np.int64), minlength=p.m)
    part, evicted, probes = bht.bht_build_stats(t.handle)
    assert part and evicted == int(np.maximum(counts - 8, 0).sum())
    assert probes >= evicted
    t.close()


@pytest.mark.parametrize("n,padded", [(4_500_000, (True, False)), (1 << 25, (True, True))])
def test_wide_partitioned_two_passes(n, padded):
    """4,500,000 pairs at load 0.9: 1,221 bins of 512 buckets, two radix
    passes (the first through the slot array); 2^25 pairs: 9,103 bins.  A
    pass writes whole 128-byte lines of 16 keys (ranges padded with the
    empty key) unless its padding would be heavy (the second pass of the
    smaller build, with 16 K-pair chunks)."""
    import paper_2108_07232_amd as bht
    print("wide partitioned two-pass n=%d" % n, flush=True)
    t, p, keys, vals = build_mode64(n, 0.9, 8, "partitioned")
    assert plan_levels64(p.m) == 2
    code, msg = oracle.check64(p, t.download(), keys, vals)
    assert code == 0, msg
    check(t, keys, vals, datagen.mixed_queries(n, 1 << 21, 0.5, 8, wide=True))
    ranges = -(-n // 16384) * 256
    for pad, on in zip(bht.bht_build_padding(t.handle), padded):
        if on:
            assert 0 < pad <= 15 * ranges and (n + pad) % 16 == 0
        else:
            assert pad == 0
    t.close()


def test_wide_build_modes_agree():
    """Default, concurrent and partitioned 64-bit builds of 2^20 pairs give
    valid layouts and identical lookups; the default takes the partitioned
    path at this size."""
    import torch
    import paper_2108_07232_amd as bht
    n = 1 << 20
    keys, vals = datagen.unique_keys64(n, 9), datagen.values64(n, 9)
    p = oracle.params_for("bcht", n, 0.9, 900, b=8, wide=True)
    q = datagen.mixed_queries(n, n, 0.5, 9, wide=True)
    results = []
    for mode in ("auto", "concurrent", "partitioned"):
        t = bht.Table(p.m * p.b, 8, "bcht", p.a, p.c, key_bits=64, rng_seed=p.rng_seed,
                      build_mode=mode)
        assert t.build(dev(keys), dev(vals)) == bht.BHT_OK
        assert oracle.check64(p, t.download(), keys, vals)[0] == 0
        assert bht.bht_build_stats(t.handle)[0] == (mode != "concurrent")
        v, f = t.find(dev(q))
        torch.cuda.synchronize()
        results.append((host_u64(v), host_u8(f)))
        t.close()
    for v, f in results[1:]:
        np.testing.assert_array_equal(v, results[0][0])
        np.testing.assert_array_equal(f, results[0][1])


def test_wide_partitioned_crowded_bucket_and_status_paths():
    """Keys that all share one first bucket (H_0 = k mod m for a = 1, c = 0):
    one bin takes 6,000 pairs, 8 stay and the rest leave through thousands of
    ranked eviction rounds.  Reserved keys are refused, and one hash for all
    three choices fails the build instead of looping."""
    import paper_2108_07232_amd as bht
    n, m = 6000, 4000                       # 32,000 slots, load 0.19
    keys = np.arange(1, n + 1, dtype=np.uint64) * np.uint64(m)
    vals = datagen.values64(n, 10)
    a, c = datagen.hash_constants64(10, 3)
    a, c = [1] + [int(x) for x in a[1:]], [0] + [int(x) for x in c[1:]]
    p = oracle.Params(scheme="bcht", b=8, m=m, h=3, a=a, c=c)
    t = bht.Table(m * 8, 8, "bcht", a, c, key_bits=64, build_mode="partitioned")
    assert t.build(dev(keys), dev(vals)) == bht.BHT_OK
    assert oracle.check64(p, t.download(), keys, vals)[0] == 0
    check(t, keys, vals, datagen.mixed_queries(n, 2 * n, 0.5, 10, wide=True))
    t.close()
    n = 1 << 16
    keys, vals = datagen.unique_keys64(n, 12), datagen.values64(n, 12)
    p = oracle.params_for("bcht", n, 0.9, 12, b=8, wide=True)
    for bad in ((1 << 64) - 1, (1 << 64) - 2):
        k = keys.copy()
        k[n // 2] = bad
        t = bht.Table(p.m * 8, 8, "bcht", p.a, p.c, key_bits=64, build_mode="partitioned")
        assert t.build(dev(k), dev(vals)) == bht.BHT_ERR_SENTINEL_KEY
        t.close()
    same = [int(p.a[0])] * 3, [int(p.c[0])] * 3
    t = bht.Table(p.m * 8, 8, "bcht", same[0], same[1], key_bits=64, build_mode="partitioned")
    assert t.build(dev(keys), dev(vals)) == bht.BHT_ERR_BUILD_FAILED
    t.close()


@pytest.mark.parametrize("n,lf,mode", [(1 << 20, 0.9, "partitioned"), (50001, 0.95, "concurrent"),
                                       (3000, 0.9, "partitioned")])
def test_wide_counted_find_probes_equal_oracle(n, lf, mode):
    """Per-query bucket reads of the counted 64-bit find equal the oracle's
    find replayed on the GPU's own layout (Section VII-E's probe); results
    equal brute force."""
    import torch
    import paper_2108_07232_amd as bht
    t, p, keys, vals = build_mode64(n, lf, 11, mode)
    layout = t.download()
    for frac in (1.0, 0.5, 0.0):
        q = datagen.mixed_queries(n, n, frac, 11, wide=True)
        out_v = torch.empty(n, dtype=torch.int64, device="cuda")
        out_f = torch.empty(n, dtype=torch.uint8, device="cuda")
        pr = torch.empty(n, dtype=torch.uint8, device="cuda")
        bht.bht_find64_counted(t.handle, dev(q), out_v, out_f, pr)
        torch.cuda.synchronize()
        bv, bf = oracle.brute_find64(keys, vals, q)
        np.testing.assert_array_equal(host_u8(out_f), bf)
        np.testing.assert_array_equal(host_u64(out_v), bv)
        _, _, _, per = oracle.find64(p, layout, q)
        np.testing.assert_array_equal(host_u8(pr), per)
    with pytest.raises(bht.BhtError):
        bht.bht_find64_counted(t.handle, dev(q), out_v, out_f, None)
    t.close()
