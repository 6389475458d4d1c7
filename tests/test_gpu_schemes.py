"""GPU parity of the comparison schemes on the shared tile skeleton:
bucketed power-of-two choices, iceberg (one level, and two levels with an
8-slot secondary array of 1/8 the primary's slots), and the bucket-size-1
cuckoo table with three and four hashes."""
import numpy as np
import pytest

import datagen
import oracle
from tests._util import dev, host_u32, host_u8, workload

pytestmark = pytest.mark.gpu


def bht():
    import paper_2108_07232_amd
    return paper_2108_07232_amd


def iceberg_params(n, lf, seed, b=16, b2=0, threshold=None):
    """Two-level geometry: secondary slots = primary slots / 8, load factor
    over all slots; one level when b2 = 0."""
    p = oracle.params_for("iht", n, lf, seed, b=b)
    if b2:
        cap = datagen.capacity_for(n, lf)
        per_primary = b + b / 8.0      # slots per primary bucket incl. its secondary share
        p.m = max(4, int(np.ceil(cap / per_primary)))
        p.b2 = b2
        p.m2 = max(1, p.m * b // 8 // b2)
    p.threshold = b if threshold is None else threshold
    return p


def gpu_table(p, schedule=0):
    return bht().Table(p.m * p.b, p.b, p.scheme, p.a, p.c, rng_seed=p.rng_seed,
                       max_chain=p.max_chain, iht_threshold=p.threshold, iht_secondary_b=p.b2,
                       iht_secondary_m=p.m2, find_schedule=schedule)


def check_find(t, p, keys, vals, q):
    import torch
    import paper_2108_07232_amd as B
    n = len(q)
    out_v = torch.empty(n, dtype=torch.int32, device="cuda")
    out_f = torch.empty(n, dtype=torch.uint8, device="cuda")
    probes = torch.empty(n, dtype=torch.uint8, device="cuda")
    B.bht_find_counted(t.handle, dev(q), out_v, out_f, probes)
    torch.cuda.synchronize()
    bv, bf = oracle.brute_find32(keys, vals, q)
    np.testing.assert_array_equal(host_u8(out_f), bf)
    np.testing.assert_array_equal(host_u32(out_v), bv)
    # per-query probes equal the oracle's on the GPU's own layout
    _, _, _, per = oracle.find32(p, t.download(), q)
    np.testing.assert_array_equal(host_u8(probes), per)


CASES = [
    # scheme, b, b2, threshold, lf, n
    ("bp2ht", 16, 0, 0, 0.8, 1 << 18),
    ("bp2ht", 32, 0, 0, 0.88, 1 << 18),
    ("bp2ht", 8, 0, 0, 0.6, 50000),
    ("bp2ht", 16, 0, 0, 0.7, 999),
    ("iht", 16, 0, 12, 0.8, 1 << 18),
    ("iht", 16, 0, 12, 0.85, 30001),
    ("iht", 32, 0, 25, 0.9, 1 << 18),
    ("iht", 16, 8, 16, 0.8, 1 << 18),
    ("iht", 16, 8, 16, 0.75, 4097),
    ("iht", 32, 8, 32, 0.85, 1 << 17),
    ("cht1", 1, 0, 0, 0.8, 1 << 18),
]


@pytest.mark.parametrize("scheme,b,b2,thr,lf,n", CASES)
def test_scheme_build_find_parity(scheme, b, b2, thr, lf, n):
    import torch
    B = bht()
    keys, vals = workload(n, 31)
    for s in range(12):
        if scheme == "iht":
            p = iceberg_params(n, lf, 3100 + s, b=b, b2=b2, threshold=thr)
        else:
            p = oracle.params_for(scheme, n, lf, 3100 + s, b=b)
        t = gpu_table(p)
        total = torch.zeros(1, dtype=torch.int64, device="cuda")
        st = B.bht_build_counted(t.handle, dev(keys), dev(vals), total)
        if st == B.BHT_OK:
            break
        assert st == B.BHT_ERR_BUILD_FAILED
        t.close()
    assert st == B.BHT_OK
    layout = t.download()
    code, msg = oracle.check32(p, layout, keys, vals)
    assert code == 0, msg
    ins = int(total.item())
    if scheme == "bp2ht":
        # Section VII-A: two buckets per placement decision; a slot lost to a
        # concurrent placement makes the pair read both again and re-decide
        assert ins >= 2 * n and ins % 2 == 0
    elif scheme == "iht":
        # one primary read per pair, two secondary reads per secondary choice
        # (made again when a concurrent placement took the chosen slot)
        assert ins >= n and (ins - n) % 2 == 0
    for frac in (1.0, 0.5, 0.0):
        check_find(t, p, keys, vals, datagen.mixed_queries(n, n, frac, 31))
    t.close()


@pytest.mark.parametrize("scheme,b,b2,thr", [("bp2ht", 16, 0, 0), ("iht", 16, 0, 12),
                                             ("iht", 16, 8, 16), ("cht1", 1, 0, 0)])
def test_scheme_find_on_oracle_layout(scheme, b, b2, thr):
    n = 20000
    keys, vals = workload(n, 41)
    for s in range(20):
        if scheme == "iht":
            p = iceberg_params(n, 0.75, 4100 + s, b=b, b2=b2, threshold=thr)
        else:
            p = oracle.params_for(scheme, n, 0.75, 4100 + s, b=b)
        st, layout, _ = oracle.build32(p, keys, vals)
        if st == oracle.OK:
            break
    assert st == oracle.OK
    t = gpu_table(p)
    t.upload(layout, n)
    check_find(t, p, keys, vals, datagen.mixed_queries(n, 2 * n, 0.5, 41))
    t.close()


def test_scheme_failures_are_reported():
    B = bht()
    n = 20000
    keys, vals = workload(n, 5)
    # power of two choices cannot reach LF 0.97 with 8-slot buckets
    p = oracle.params_for("bp2ht", n, 0.97, 5, b=8)
    t = gpu_table(p)
    assert t.build(dev(keys), dev(vals)) == B.BHT_ERR_BUILD_FAILED
    t.close()
    # two-level iceberg at full load overflows its small secondary level
    p = iceberg_params(n, 0.99, 5, b=16, b2=8, threshold=16)
    t = gpu_table(p)
    assert t.build(dev(keys), dev(vals)) == B.BHT_ERR_BUILD_FAILED
    t.close()


def test_power_of_two_places_in_less_loaded_bucket_when_uncontended():
    # one wave's worth of keys on a large table: no two keys share a bucket,
    # so every key lands in H0 exactly (both buckets empty, ties to H0)
    n = 64
    for seed in range(6, 100):
        keys, vals = workload(n, seed)
        p = oracle.params_for("bp2ht", n, 0.001, seed, b=16)
        cands = np.concatenate([oracle.hash32_many(p.a[i], p.c[i], keys, p.m) for i in range(2)])
        if len(np.unique(cands)) == 2 * n:     # no candidate bucket shared by two keys
            break
    t = gpu_table(p)
    assert t.build(dev(keys), dev(vals)) == bht().BHT_OK
    layout = t.download()
    b0 = oracle.hash32_many(p.a[0], p.c[0], keys, p.m).astype(np.int64)
    occ = np.nonzero((layout & np.uint64(0xFFFFFFFF)) != np.uint64(0xFFFFFFFF))[0]
    stored_keys = (layout[occ] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    where = dict(zip(stored_keys.tolist(), (occ // 16).tolist()))
    assert all(where[int(k)] == int(b) for k, b in zip(keys, b0))
    t.close()


@pytest.mark.parametrize("b,b2,thr,lf,n", [(16, 0, 13, 0.86, 1 << 18), (16, 0, 8, 0.8, 50001),
                                           (16, 8, 16, 0.8, 1 << 18), (32, 0, 25, 0.9, 1 << 17)])
def test_iceberg_early_exit_find(b, b2, thr, lf, n):
    """Iceberg finds that stop after a miss in a primary below the threshold:
    results equal brute force, and per-query probes equal the oracle's
    early-exit find on the GPU's own layout (one probe for a negative query
    whose primary holds fewer than t keys)."""
    import torch
    B = bht()
    keys, vals = workload(n, 51)
    for s in range(12):
        p = iceberg_params(n, lf, 5100 + s, b=b, b2=b2, threshold=thr)
        t = gpu_table(p)
        st = t.build(dev(keys), dev(vals))
        if st == B.BHT_OK:
            break
        t.close()
    assert st == B.BHT_OK
    B.bht_set_tuning(t.handle, iht_early_exit=True)
    assert B.bht_get_tuning(t.handle)[4] == 1
    p.early_exit = True
    for frac in (1.0, 0.5, 0.0):
        check_find(t, p, keys, vals, datagen.mixed_queries(n, n, frac, 52))
    t.close()
    # other schemes refuse the setting
    pc = oracle.params_for("bcht", 1000, 0.5, 1)
    t = B.Table(pc.m * 16, 16, "bcht", pc.a, pc.c)
    with pytest.raises(B.BhtError):
        B.bht_set_tuning(t.handle, iht_early_exit=True)
    t.close()


@pytest.mark.parametrize("b,h,lf,n", [(16, 3, 0.9, 1 << 18), (16, 3, 0.97, 1 << 17),
                                      (16, 2, 0.9, 100003), (8, 3, 0.9, 1 << 17),
                                      (32, 2, 0.95, 1 << 17), (16, 4, 0.98, 50000)])
def test_load_balanced_cuckoo_build_find_parity(b, h, lf, n):
    """Load-balanced cuckoo table on the GPU: the layout satisfies the
    oracle's invariants (no early-exit property is claimed), lookups equal
    brute force, per-query probes equal the oracle's on the GPU layout, and
    insertion reads h buckets per placement attempt."""
    import torch
    B = bht()
    keys, vals = workload(n, 61)
    for s in range(10):
        p = oracle.params_for("bcht_lb", n, lf, 6100 + s, b=b, h=h)
        t = gpu_table(p)
        total = torch.zeros(1, dtype=torch.int64, device="cuda")
        st = B.bht_build_counted(t.handle, dev(keys), dev(vals), total)
        if st == B.BHT_OK:
            break
        assert st == B.BHT_ERR_BUILD_FAILED
        t.close()
    assert st == B.BHT_OK
    code, msg = oracle.check32(p, t.download(), keys, vals)
    assert code == 0, msg
    ins = int(total.item())
    assert ins >= h * n and ins % h == 0
    for frac in (1.0, 0.5, 0.0):
        check_find(t, p, keys, vals, datagen.mixed_queries(n, n, frac, 62))
    # an uninstrumented rebuild is valid too
    assert t.build(dev(keys), dev(vals)) == B.BHT_OK
    assert oracle.check32(p, t.download(), keys, vals)[0] == 0
    t.close()


def test_load_balanced_cuckoo_reaches_loads_power_of_two_cannot():
    """With two hashes and 8-slot buckets, power-of-two choices fails at load
    0.95 while the load-balanced table, which can evict, builds."""
    B = bht()
    n = 1 << 16
    keys, vals = workload(n, 63)
    p = oracle.params_for("bp2ht", n, 0.95, 63, b=8)
    t = gpu_table(p)
    assert t.build(dev(keys), dev(vals)) == B.BHT_ERR_BUILD_FAILED
    t.close()
    for s in range(6):
        p = oracle.params_for("bcht_lb", n, 0.95, 6300 + s, b=8, h=2)
        t = gpu_table(p)
        st = t.build(dev(keys), dev(vals))
        if st == B.BHT_OK:
            break
        t.close()
    assert st == B.BHT_OK
    assert oracle.check32(p, t.download(), keys, vals)[0] == 0
    t.close()


ICEBERG_PARTITIONED = [
    # b, b2, threshold, lf, n
    (16, 0, 12, 0.8, 1 << 18),
    (16, 0, 9, 0.86, 100003),
    (32, 0, 25, 0.9, 1 << 18),
    (16, 8, 16, 0.8, 1 << 18),
    (16, 8, 16, 0.86, 300007),
    (32, 8, 32, 0.85, 1 << 17),
    (16, 8, 16, 0.86, 1 << 23),          # 1,059 bins: two radix passes
    (16, 0, 4, 0.5, 5000),               # low threshold, a single bin
    (16, 8, 16, 0.8, 3),
]


@pytest.mark.parametrize("b,b2,thr,lf,n", ICEBERG_PARTITIONED)
def test_iceberg_partitioned_build(b, b2, thr, lf, n):
    """Partitioned iceberg build (primaries filled on chip up to t pairs, the
    rest inserted at their secondary choices): the oracle's invariant checker
    (including: every secondary key's primary holds at least t keys), exact
    lookups and per-query probes, and the number of pairs sent on from the
    primaries equals the primary overflow sum max(0, X_j - t)."""
    B = bht()
    print("iceberg partitioned b=%d b2=%d t=%d lf=%g n=%d" % (b, b2, thr, lf, n), flush=True)
    keys, vals = workload(n, 41)
    for s in range(12):
        p = iceberg_params(n, lf, 4100 + s, b=b, b2=b2, threshold=thr)
        t = B.Table(p.m * p.b, p.b, p.scheme, p.a, p.c, rng_seed=p.rng_seed,
                    max_chain=p.max_chain, iht_threshold=p.threshold, iht_secondary_b=p.b2,
                    iht_secondary_m=p.m2, build_mode="partitioned")
        st = t.build(dev(keys), dev(vals))
        if st == B.BHT_OK:
            break
        assert st == B.BHT_ERR_BUILD_FAILED
        t.close()
    assert st == B.BHT_OK
    code, msg = oracle.check32(p, t.download(), keys, vals)
    assert code == 0, msg
    part, sent_on, _ = B.bht_build_stats(t.handle)
    h0 = oracle.hash32_many(p.a[0], p.c[0], keys, p.m)
    counts = np.bincount(h0.astype(np.int64), minlength=p.m)
    assert part and sent_on == int(np.maximum(counts - min(thr, b), 0).sum())
    nq = min(n, 1 << 20)
    for frac in (1.0, 0.0):
        check_find(t, p, keys, vals, datagen.mixed_queries(n, nq, frac, 41))
    t.close()


def test_iceberg_build_modes_agree():
    """Concurrent and partitioned iceberg builds of the same input give valid
    layouts and identical lookups; from 2^18 pairs the default takes the
    partitioned path for a two-level table."""
    import torch
    B = bht()
    n = 1 << 19
    keys, vals = workload(n, 42)
    p = iceberg_params(n, 0.8, 4200, b=16, b2=8, threshold=16)
    q = datagen.mixed_queries(n, n, 0.5, 42)
    results = []
    for mode in ("concurrent", "auto", "partitioned"):
        t = B.Table(p.m * p.b, p.b, p.scheme, p.a, p.c, rng_seed=p.rng_seed,
                    iht_threshold=p.threshold, iht_secondary_b=p.b2, iht_secondary_m=p.m2,
                    build_mode=mode)
        assert t.build(dev(keys), dev(vals)) == B.BHT_OK
        assert oracle.check32(p, t.download(), keys, vals)[0] == 0
        assert B.bht_build_stats(t.handle)[0] == (mode != "concurrent")
        v, f = t.find(dev(q))
        torch.cuda.synchronize()
        results.append((host_u32(v), host_u8(f)))
        t.close()
    for v, f in results[1:]:
        np.testing.assert_array_equal(v, results[0][0])
        np.testing.assert_array_equal(f, results[0][1])
