"""GPU parity of the bucketed cuckoo table (and its bucket-size-1 form).

Lookups must equal the plain definition (brute force over the input pairs)
bit for bit; layouts may differ from the oracle's, so GPU layouts are
checked with the oracle's invariant checker instead.
"""
import numpy as np
import pytest

import datagen
import oracle
from tests._util import dev, host_u32, host_u8, workload

pytestmark = pytest.mark.gpu


def bht():
    import paper_2108_07232_amd
    return paper_2108_07232_amd


def gpu_table(params: oracle.Params, tile=None, schedule=0):
    t = bht().Table(params.m * params.b, params.b, params.scheme, params.a, params.c,
                    rng_seed=params.rng_seed, max_chain=params.max_chain, tile=tile,
                    find_schedule=schedule)
    return t


def build_ok(table, keys, vals):
    st = table.build(dev(keys), dev(vals))
    return st


def assert_find_matches_bruteforce(table, keys, vals, queries):
    import torch
    v, f = table.find(dev(queries))
    torch.cuda.synchronize()
    bv, bf = oracle.brute_find32(keys, vals, queries)
    np.testing.assert_array_equal(host_u8(f), bf)
    np.testing.assert_array_equal(host_u32(v), bv)


def build_with_retries(scheme, n, lf, b, seed0, h=None, tile=None, tries=8):
    keys, vals = workload(n, seed0)
    for s in range(tries):
        params = oracle.params_for(scheme, n, lf, seed0 * 100 + s, b=b, h=h)
        t = gpu_table(params, tile)
        st = build_ok(t, keys, vals)
        if st == bht().BHT_OK:
            return t, params, keys, vals
        assert st == bht().BHT_ERR_BUILD_FAILED
        t.close()
    pytest.fail("no successful GPU build in %d tries" % tries)


# -------------------------------------------- find on oracle-built layouts

@pytest.mark.parametrize("schedule", ["refill", "chunk", "parallel", "chunk_unroll2"])
@pytest.mark.parametrize("b,tile,n,lf", [
    (16, 8, 1 << 20, 0.9), (16, 4, 5000, 0.95), (16, 16, 4097, 0.9), (8, 8, 3001, 0.85),
    (8, 4, 777, 0.9), (32, 16, 6000, 0.95), (32, 8, 1000, 0.9), (4, 4, 2000, 0.8),
    (1, 1, 3000, 0.8),
])
def test_find_on_oracle_layout(b, tile, n, lf, schedule):
    scheme = "cht1" if b == 1 else "bcht"
    keys, vals = workload(n, 21)
    for s in range(10):
        params = oracle.params_for(scheme, n, lf, 2100 + s, b=b)
        st, layout, _ = oracle.build32(params, keys, vals)
        if st == oracle.OK:
            break
    assert st == oracle.OK
    if schedule == "chunk_unroll2":
        t = gpu_table(params, tile, "chunk")
        bht().bht_set_tuning(t.handle, tile, "chunk", 0, 0, False, 2)
    else:
        t = gpu_table(params, tile, schedule)
    t.upload(layout, n)
    for frac in (1.0, 0.5, 0.0):
        q = datagen.mixed_queries(n, n, frac, 21)
        assert_find_matches_bruteforce(t, keys, vals, q)
    # sentinel query, and queries equal to p..p+3 (hash like 0..3)
    q = np.array([0xFFFFFFFF, 4294967291, 4294967292, 0, 1, 2, 3, int(keys[0])], dtype=np.uint32)
    assert_find_matches_bruteforce(t, keys, vals, q)
    t.close()


# ------------------------------------------------ GPU build: invariants + find

@pytest.mark.parametrize("b,tile,n,lf", [
    (16, 8, 1 << 20, 0.9), (16, 4, 1 << 16, 0.9), (16, 16, 1 << 16, 0.9),
    (16, 8, 50000, 0.95), (16, 8, 40000, 0.98), (16, 8, 1000, 0.9), (16, 8, 63, 0.5),
    (8, 8, 30000, 0.9), (32, 16, 30000, 0.95), (32, 8, 30001, 0.9), (4, 4, 20000, 0.85),
    (1, 1, 30000, 0.8),
])
def test_gpu_build_invariants_and_find(b, tile, n, lf):
    scheme = "cht1" if b == 1 else "bcht"
    t, params, keys, vals = build_with_retries(scheme, n, lf, b, 7, tile=tile)
    layout = t.download()
    code, msg = oracle.check32(params, layout, keys, vals)
    assert code == 0, msg
    for frac in (1.0, 0.5, 0.0):
        q = datagen.mixed_queries(n, n, frac, 7)
        assert_find_matches_bruteforce(t, keys, vals, q)
    t.close()


def test_gpu_build_lf_sweep_and_ragged_sizes():
    for n, lf in [(1 << 18, 0.6), (1 << 18, 0.7), (1 << 18, 0.8), (1 << 18, 0.95),
                  (1 << 18, 0.99), (100003, 0.9), (1, 0.9), (17, 0.9)]:
        t, params, keys, vals = build_with_retries("bcht", n, lf, 16, 3, tries=12)
        code, msg = oracle.check32(params, t.download(), keys, vals)
        assert code == 0, (n, lf, msg)
        q = datagen.mixed_queries(n, max(n, 64), 0.5, 3)
        assert_find_matches_bruteforce(t, keys, vals, q)
        t.close()


def test_small_table_high_contention():
    # a 2-bucket .. 64-bucket table built by thousands of lanes at once: every
    # CAS and exchange contends; the layout must still hold every pair once
    for n, lf, b in [(31, 1.0, 16), (500, 0.98, 16), (1024, 0.97, 8), (4000, 0.99, 32)]:
        t, params, keys, vals = build_with_retries("bcht", n, lf, b, 5, tries=30)
        code, msg = oracle.check32(params, t.download(), keys, vals)
        assert code == 0, (n, lf, b, msg)
        assert_find_matches_bruteforce(t, keys, vals, datagen.mixed_queries(n, 4 * n, 0.5, 5))
        t.close()


# ---------------------------------------------------- status and edge cases

def test_build_status_paths():
    B = bht()
    keys, vals = workload(1000, 2)
    params = oracle.params_for("bcht", 1000, 0.9, 2)
    t = gpu_table(params)
    # find before build
    with pytest.raises(B.BhtError) as e:
        t.find(dev(keys))
    assert e.value.status == B.BHT_ERR_NOT_BUILT
    # empty build, then every query misses
    assert t.build(dev(keys[:0]), dev(vals[:0])) == B.BHT_OK
    v, f = t.find(dev(keys))
    assert not host_u8(f).any() and np.all(host_u32(v) == 0xFFFFFFFF)
    # sentinel key is rejected
    bad = keys.copy()
    bad[500] = 0xFFFFFFFF
    assert t.build(dev(bad), dev(vals)) == B.BHT_ERR_SENTINEL_KEY
    # more pairs than slots
    with pytest.raises(B.BhtError) as e:
        B.bht_build(t.handle, dev(np.arange(2000, dtype=np.uint32)), dev(np.arange(2000, dtype=np.uint32)))
    assert e.value.status == B.BHT_ERR_CAPACITY
    # a good build after failures works
    assert t.build(dev(keys), dev(vals)) == B.BHT_OK
    assert_find_matches_bruteforce(t, keys, vals, datagen.mixed_queries(1000, 3000, 0.5, 2))
    t.close()


def test_single_hash_build_fails_exactly_on_overflow():
    # h = 1: an evicted pair returns to the same full bucket, so the build
    # fails exactly when some bucket receives more than b keys
    B = bht()
    for seed in range(1, 25):
        n = 700
        keys, vals = workload(n, seed)
        params = oracle.params_for("bcht", n, 0.75, seed, b=8, h=1)
        counts = np.bincount(oracle.hash32_many(params.a[0], params.c[0], keys, params.m).astype(np.int64),
                             minlength=params.m)
        t = gpu_table(params)
        st = t.build(dev(keys), dev(vals))
        assert (st == B.BHT_OK) == bool(counts.max() <= 8), seed
        if st == B.BHT_OK:
            assert oracle.check32(params, t.download(), keys, vals)[0] == 0
        t.close()


def test_reseed_after_failure_and_zero_chain():
    B = bht()
    n = 60000
    keys, vals = workload(n, 9)
    params = oracle.params_for("bcht", n, 0.99, 9, max_chain=0)
    t = gpu_table(params)
    assert t.build(dev(keys), dev(vals)) == B.BHT_ERR_BUILD_FAILED
    p2 = oracle.params_for("bcht", n, 0.99, 10)
    B.bht_reseed(t.handle, B.make_params(p2.a, p2.c, max_chain=128))
    for s in range(11, 20):
        if t.build(dev(keys), dev(vals)) == B.BHT_OK:
            break
        p2 = oracle.params_for("bcht", n, 0.99, s)
        B.bht_reseed(t.handle, B.make_params(p2.a, p2.c, max_chain=128))
    p2.max_chain = 128
    assert oracle.check32(p2, t.download(), keys, vals)[0] == 0
    t.close()


# ---------------------------------------------------------- probe counters

@pytest.mark.parametrize("schedule", ["refill", "chunk"])
def test_find_probe_counts_equal_oracle_on_gpu_layout(schedule):
    import torch
    B = bht()
    n = 1 << 18
    t, params, keys, vals = build_with_retries("bcht", n, 0.95, 16, 4)
    B.bht_set_tuning(t.handle, 0, schedule)
    layout = t.download()
    for frac in (1.0, 0.5, 0.0):
        q = datagen.mixed_queries(n, n, frac, 4)
        dq = dev(q)
        out_v = torch.empty(n, dtype=torch.int32, device="cuda")
        out_f = torch.empty(n, dtype=torch.uint8, device="cuda")
        probes = torch.empty(n, dtype=torch.uint8, device="cuda")
        B.bht_find_counted(t.handle, dq, out_v, out_f, probes)
        torch.cuda.synchronize()
        ov, of, total, per = oracle.find32(params, layout, q)
        np.testing.assert_array_equal(host_u8(probes), per)
        np.testing.assert_array_equal(host_u8(out_f), of)
        np.testing.assert_array_equal(host_u32(out_v), ov)
    t.close()


def test_build_probe_counts_near_paper():
    import torch
    B = bht()
    n = 1 << 20
    keys, vals = workload(n, 12)
    params = oracle.params_for("bcht", n, 0.9, 12)
    t = gpu_table(params)
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert B.bht_build_counted(t.handle, dev(keys), dev(vals), total) == B.BHT_OK
    per_key = int(total.item()) / n
    # Section VII-A: 1.11 bucket reads per insertion at b = 16, LF 0.9
    assert 1.0 <= per_key <= 1.25, per_key
    t.close()


def test_probe_stats_totals():
    """bht_get_probe_stats reports the counted build's bucket reads (as the
    caller's counter saw them) and the sum of the per-query counts of the
    counted finds since the previous call; the oracle's find on the GPU
    layout gives the same find total."""
    import torch
    B = bht()
    n = 1 << 17
    keys, vals = workload(n, 14)
    params = oracle.params_for("bcht", n, 0.9, 14)
    t = gpu_table(params)
    total = torch.full((1,), 1000, dtype=torch.int64, device="cuda")
    assert B.bht_build_counted(t.handle, dev(keys), dev(vals), total) == B.BHT_OK
    bp, fp = B.bht_get_probe_stats(t.handle)
    assert bp == int(total.item()) - 1000 and n <= bp < 2 * n
    assert fp == 0
    layout = t.download()
    expect = 0
    for frac in (1.0, 0.0, 0.5):
        q = datagen.mixed_queries(n, n, frac, 14)
        out_v = torch.empty(n, dtype=torch.int32, device="cuda")
        out_f = torch.empty(n, dtype=torch.uint8, device="cuda")
        probes = torch.empty(n, dtype=torch.uint8, device="cuda")
        B.bht_find_counted(t.handle, dev(q), out_v, out_f, probes)
        B.bht_find(t.handle, dev(q), out_v, out_f)      # uncounted: adds nothing
        expect += oracle.find32(params, layout, q)[2]
    bp2, fp = B.bht_get_probe_stats(t.handle)
    assert bp2 == bp and fp == expect
    assert B.bht_get_probe_stats(t.handle) == (bp, 0)
    assert B.bht_build(t.handle, dev(keys), dev(vals)) == B.BHT_OK
    assert B.bht_get_probe_stats(t.handle) == (0, 0)    # the last build was not counted
    t.close()


# ------------------------------------------------ build with reseeding

def test_build_retry_recovers_from_constants_that_cannot_build():
    """Three equal hash functions give every key a single bucket, so at load
    factor 0.9 some bucket overflows and the first build fails; the retry
    draws new constants (Section VII) and the rebuilt table is valid."""
    B = bht()
    n, seed = 20000, 99
    keys, vals = workload(n, 77)
    cap = datagen.capacity_for(n, 0.9)
    t = B.Table(cap, 16, "bcht", [5, 5, 5], [7, 7, 7])
    st, attempts = B.bht_build_retry(t.handle, dev(keys), dev(vals), seed, max_attempts=10)
    assert st == B.BHT_OK and attempts >= 2
    drawn = B.bht_params_from_seed(seed + attempts - 2, "bcht")
    m = t.info[0]
    params = oracle.Params(scheme="bcht", b=16, m=m, h=3, a=list(drawn.a)[:3],
                           c=list(drawn.b)[:3], rng_seed=drawn.rng_seed)
    code, msg = oracle.check32(params, t.download(), keys, vals)
    assert code == 0, msg
    q = datagen.mixed_queries(n, 3 * n, 0.5, 5)
    assert_find_matches_bruteforce(t, keys, vals, q)
    t.close()


def test_build_retry_gives_up_after_max_attempts():
    """With no evictions allowed a build at load factor 0.95 always meets a
    full bucket and fails: every attempt runs and the failure is reported."""
    B = bht()
    n = 20000
    keys, vals = workload(n, 78)
    cap = datagen.capacity_for(n, 0.95)
    a, c = datagen.hash_constants(3, 3)
    t = B.Table(cap, 16, "bcht", a, c, max_chain=0)
    st, attempts = B.bht_build_retry(t.handle, dev(keys), dev(vals), 5, max_attempts=3)
    assert st == B.BHT_ERR_BUILD_FAILED and attempts == 3
    t.close()


@pytest.mark.parametrize("b,h", [(16, 3), (16, 2), (8, 4), (1, 3)])
def test_parallel_probing_reads_every_candidate(b, h):
    """Parallel probing reads all h buckets of every query (h probes, none
    for the sentinel) and answers exactly as brute force."""
    import torch
    B = bht()
    n = 40000
    scheme = "cht1" if b == 1 else "bcht"
    t, params, keys, vals = build_with_retries(scheme, n, 0.8, b, 9, h=h)
    B.bht_set_tuning(t.handle, 0, "parallel")
    q = datagen.mixed_queries(n, 2 * n, 0.5, 9)
    q[5] = 0xFFFFFFFF
    out_v = torch.empty(len(q), dtype=torch.int32, device="cuda")
    out_f = torch.empty(len(q), dtype=torch.uint8, device="cuda")
    pr = torch.empty(len(q), dtype=torch.uint8, device="cuda")
    B.bht_find_counted(t.handle, dev(q), out_v, out_f, pr)
    torch.cuda.synchronize()
    bv, bf = oracle.brute_find32(keys, vals, q)
    np.testing.assert_array_equal(host_u8(out_f), bf)
    np.testing.assert_array_equal(host_u32(out_v), bv)
    expect = np.full(len(q), h, dtype=np.uint8)
    expect[5] = 0
    np.testing.assert_array_equal(host_u8(pr), expect)
    t.close()
