"""GPU parity of the partitioned build (radix passes by first-bucket region,
first-bucket placement in on-chip memory, cuckoo insertion of the rest).

The insertion runs under a deferred-victim schedule (first-bucket claims
and on-chip exchanges, then the evicted pairs' chains concurrently), and
its layout is judged like every GPU layout: the oracle's invariant checker
(each pair stored once, in a candidate bucket, occupied slots a prefix,
early-exit property) and lookups equal to brute force, bit for bit."""
import numpy as np
import pytest

import datagen
import oracle
from tests._util import dev, host_u32, host_u8, workload

pytestmark = pytest.mark.gpu


def bht():
    import paper_2108_07232_amd
    return paper_2108_07232_amd


def build_partitioned(params, keys, vals, mode="partitioned", tile=None):
    B = bht()
    t = B.Table(params.m * params.b, params.b, params.scheme, params.a, params.c,
                rng_seed=params.rng_seed, max_chain=params.max_chain, tile=tile,
                build_mode=mode)
    st = t.build(dev(keys), dev(vals))
    return t, st


def check_table(t, params, keys, vals, n_queries=None, seed=3):
    import torch
    code, msg = oracle.check32(params, t.download(), keys, vals)
    assert code == 0, msg
    n = len(keys)
    q = datagen.mixed_queries(n, n_queries or 2 * n, 0.5, seed)
    v, f = t.find(dev(q))
    torch.cuda.synchronize()
    ev, ef = oracle.brute_find32(keys, vals, q)
    np.testing.assert_array_equal(host_u8(f), ef)
    np.testing.assert_array_equal(host_u32(v), ev)


def plan_levels(m, b):
    """Radix passes the library plans for m buckets of b slots."""
    r = (4096 if b == 1 else 8192) // b
    nbins = -(-m // r)
    return 1 if nbins <= 1024 else 2


@pytest.mark.parametrize("scheme,b,tile,n,lf", [
    ("bcht", 16, 8, 1 << 20, 0.9),        # one pass, 143 bins
    ("bcht", 16, 8, 100003, 0.95),        # ragged last bin
    ("bcht", 16, 4, 50000, 0.98),         # heavy overflow
    ("bcht", 16, 16, 3000, 0.9),          # a single bin
    ("bcht", 8, 8, 300007, 0.9),
    ("bcht", 8, 4, 1 << 18, 0.85),
    ("bcht", 32, 16, 400009, 0.95),
    ("bcht", 32, 8, 1 << 17, 0.9),
    ("bcht", 4, 4, 200003, 0.8),
    ("cht1", 1, 1, 300000, 0.8),
])
def test_partitioned_build_invariants_and_find(scheme, b, tile, n, lf):
    print("partitioned %s b=%d tile=%d n=%d lf=%g" % (scheme, b, tile, n, lf), flush=True)
    keys, vals = workload(n, 11)
    for s in range(6):
        params = oracle.params_for(scheme, n, lf, 500 + s, b=b)
        t, st = build_partitioned(params, keys, vals, tile=tile)
        if st == bht().BHT_OK:
            break
        assert st == bht().BHT_ERR_BUILD_FAILED
        t.close()
    else:
        pytest.fail("no partitioned build succeeded")
    assert plan_levels(params.m, b) == 1
    check_table(t, params, keys, vals)
    t.close()


@pytest.mark.parametrize("scheme,b,n,lf,padded", [
    ("bcht", 16, 9_000_011, 0.9, (True, False)),   # two passes: 1,221 bins of 512 buckets
    ("bcht", 32, 8_000_000, 0.9, (True, False)),
    ("cht1", 1, 4_000_037, 0.8, (True, False)),    # two passes: 1,221 bins of 4,096 slots
    ("bcht", 16, 1 << 25, 0.9, (True, True)),      # 4,552 bins, 64 K-pair chunks
])
def test_partitioned_build_two_passes(scheme, b, n, lf, padded):
    print("partitioned two-pass %s b=%d n=%d lf=%g" % (scheme, b, n, lf), flush=True)
    keys, vals = workload(n, 12)
    params = oracle.params_for(scheme, n, lf, 600, b=b)
    assert plan_levels(params.m, b) == 2
    t, st = build_partitioned(params, keys, vals)
    assert st == bht().BHT_OK, bht().bht_status_string(st)
    check_table(t, params, keys, vals, n_queries=1 << 21)
    # a pass of at most 256 digits pads its ranges to whole 128-byte lines
    # unless that padding would be heavy (small chunks): it then writes a
    # multiple of 32 words, less than a line more per (chunk, digit) range
    pads = bht().bht_build_padding(t.handle)
    ranges = -(-n // 16384) * 256
    for pad, on in zip(pads, padded):
        if on:
            assert 0 < pad <= 31 * ranges and (n + pad) % 32 == 0
        else:
            assert pad == 0
    t.close()


def test_partitioned_first_pass_unpadded_when_slots_are_short():
    """At 2^27 pairs and LF 0.99 the padded first-pass output could exceed
    the slot array it is written to (up to 2.1 M padding pairs, 1.4 M spare
    slots), so only the second pass pads; the layout is valid and lookups
    equal brute force.  (Near its load limit the build runs with an
    eviction cap of 1024.)"""
    B = bht()
    n = 1 << 27
    keys, vals = workload(n, 13)
    for s in range(4):
        params = oracle.params_for("bcht", n, 0.99, 620 + s, max_chain=1024)
        t, st = build_partitioned(params, keys, vals)
        if st == B.BHT_OK:
            break
        assert st == B.BHT_ERR_BUILD_FAILED
        t.close()
    else:
        pytest.fail("no partitioned build succeeded")
    pad1, pad2 = B.bht_build_padding(t.handle)
    assert pad1 == 0 and pad2 > 0 and (n + pad2) % 32 == 0
    check_table(t, params, keys, vals, n_queries=1 << 21)
    t.close()


def test_build_modes_give_valid_layouts_and_identical_lookups():
    """Default, concurrent and partitioned builds of 2^21 pairs: every layout
    is valid and every lookup result is the same."""
    import torch
    n = 1 << 21
    keys, vals = workload(n, 13)
    params = oracle.params_for("bcht", n, 0.9, 700)
    q = datagen.mixed_queries(n, n, 0.5, 9)
    results = []
    for mode in ("auto", "concurrent", "partitioned"):
        t, st = build_partitioned(params, keys, vals, mode=mode)
        assert st == bht().BHT_OK
        assert oracle.check32(params, t.download(), keys, vals)[0] == 0
        v, f = t.find(dev(q))
        torch.cuda.synchronize()
        results.append((host_u32(v), host_u8(f)))
        t.close()
    for v, f in results[1:]:
        np.testing.assert_array_equal(v, results[0][0])
        np.testing.assert_array_equal(f, results[0][1])


def test_bin_with_more_pairs_than_one_placement_round():
    """All pairs share their first bucket (H_0 = identity mod m on multiples of
    m): one bin receives 20,000 pairs (three rounds of 8,192), 16 are placed
    and the rest go through eviction to their other buckets."""
    n = 20000
    m = 12500                                    # 200,000 slots, load 0.1
    keys = (np.arange(n, dtype=np.uint64) * m).astype(np.uint32)
    assert len(np.unique(keys)) == n and int(keys.max()) < 4294967291
    vals = datagen.values(n, 14)
    _, c = datagen.hash_constants(14, 3)
    a = [1] + list(datagen.hash_constants(15, 3)[0][1:])
    c = [0] + list(c[1:])
    params = oracle.Params(scheme="bcht", b=16, m=m, h=3, a=a, c=c)
    t, st = build_partitioned(params, keys, vals)
    assert st == bht().BHT_OK, bht().bht_status_string(st)
    check_table(t, params, keys, vals)
    t.close()


def test_line_writing_passes_with_skewed_digits():
    """2^25 pairs whose first buckets all lie in the first quarter of a
    table of 2^27 slots (16 of the first pass's 64 digits, 512 pairs per
    digit and sub-tile, 16 lines per digit): both radix passes write whole
    lines, carry remainders and pad, and the layout is valid with lookups
    equal to brute force."""
    B = bht()
    n = 1 << 25
    params = oracle.params_for("bcht", n, 0.25, 640)
    keys = datagen.unique_keys(5 * n, 41)
    h0 = oracle.hash32_many(params.a[0], params.c[0], keys, params.m)
    keys = keys[h0 < params.m // 4][:n]
    assert len(keys) == n
    vals = datagen.values(n, 41)
    t, st = build_partitioned(params, keys, vals)
    assert st == B.BHT_OK, B.bht_status_string(st)
    pad1, pad2 = B.bht_build_padding(t.handle)
    assert pad1 > 0 and pad2 > 0 and (n + pad1) % 32 == 0 and (n + pad2) % 32 == 0
    check_table(t, params, keys, vals, n_queries=1 << 21)
    t.close()


def test_repeated_builds_reuse_the_workspace():
    """Rebuilding a table (larger, then smaller inputs) gives a fresh valid
    layout each time."""
    B = bht()
    params = oracle.params_for("bcht", 1 << 20, 0.9, 800)
    t = B.Table(params.m * params.b, 16, "bcht", params.a, params.c, rng_seed=params.rng_seed,
                build_mode="partitioned")
    for n, seed in ((1 << 19, 21), (1 << 20, 22), (77777, 23)):
        keys, vals = workload(n, seed)
        assert t.build(dev(keys), dev(vals)) == B.BHT_OK
        check_table(t, params, keys, vals, n_queries=n)
    t.close()


def test_partitioned_status_paths():
    B = bht()
    n = 1 << 16
    keys, vals = workload(n, 24)
    params = oracle.params_for("bcht", n, 0.9, 900)
    bad = keys.copy()
    bad[n // 3] = 0xFFFFFFFF
    t, st = build_partitioned(params, bad, vals)
    assert st == B.BHT_ERR_SENTINEL_KEY
    t.close()
    # one hash for all three choices: overflow can never leave its bucket
    same = oracle.Params(scheme="bcht", b=16, m=params.m, h=3, a=[7, 7, 7], c=[9, 9, 9])
    t, st = build_partitioned(same, keys, vals)
    assert st == B.BHT_ERR_BUILD_FAILED
    # the failed table rebuilds with proper constants
    B.bht_reseed(t.handle, B.make_params(params.a, params.c))
    assert t.build(dev(keys), dev(vals)) == B.BHT_OK
    check_table(t, params, keys, vals, n_queries=n)
    t.close()


@pytest.mark.parametrize("b,n,lf", [(16, 1 << 20, 0.9), (16, 300007, 0.98), (8, 200003, 0.9),
                                    (1, 100000, 0.8)])
def test_eviction_count_equals_first_bucket_overflow(b, n, lf):
    """A pair evicts on chip exactly when its first bucket already holds b
    pairs, so the build's eviction count equals the first-bucket overflow
    sum over buckets of max(0, X_j - b), X_j = pairs whose H_0 is bucket j,
    computed here from the oracle's hash.  Every evicted pair then reads at
    least one more bucket."""
    B = bht()
    scheme = "cht1" if b == 1 else "bcht"
    keys, vals = workload(n, 31)
    for s in range(6):
        params = oracle.params_for(scheme, n, lf, 950 + s, b=b)
        t, st = build_partitioned(params, keys, vals)
        if st == B.BHT_OK:
            break
        t.close()
    else:
        pytest.fail("no partitioned build succeeded")
    h0 = oracle.hash32_many(params.a[0], params.c[0], keys, params.m)
    counts = np.bincount(h0.astype(np.int64), minlength=params.m)
    expected = int(np.maximum(counts - b, 0).sum())
    part, evicted, probes = B.bht_build_stats(t.handle)
    assert part and evicted == expected
    assert probes >= evicted
    t.close()
    # a concurrent build reports no partitioned statistics
    t, st = build_partitioned(params, keys, vals, mode="concurrent")
    assert st == B.BHT_OK
    assert B.bht_build_stats(t.handle) == (False, 0, 0)
    assert B.bht_build_padding(t.handle) == (0, 0)
    t.close()


def test_build_with_caller_workspace():
    """bht_build_async_in takes the partitioned path with caller-owned
    workspace (here on a table in caller-owned memory too): the layout is
    valid, lookups equal brute force, a too-small workspace is refused, and
    schemes without that path report a size of 0 and build normally."""
    import torch
    B = bht()
    n = 300007
    keys, vals = workload(n, 41)
    params = oracle.params_for("bcht", n, 0.9, 1100)
    pb = B.make_params(params.a, params.c, rng_seed=params.rng_seed)
    nbytes = B.bht_table_bytes(params.m * 16, 16, "bcht", pb)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    t = B.Table(params.m * 16, 16, "bcht", params.a, params.c, rng_seed=params.rng_seed, buffer=buf)
    need = B.bht_build_workspace_bytes(t.handle, n)
    assert need > 8 * n
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    dk, dv = dev(keys), dev(vals)
    with pytest.raises(B.BhtError) as e:
        B.bht_build_async_in(t.handle, dk, dv, ws[:need - 256])
    assert e.value.status == B.BHT_ERR_INVALID_ARG
    B.bht_build_async_in(t.handle, dk, dv, ws)
    assert B.bht_build_wait(t.handle) == B.BHT_OK
    assert B.bht_build_stats(t.handle)[0]
    check_table(t, params, keys, vals)
    t.close()
    p2 = oracle.params_for("bp2ht", n, 0.6, 1101)        # well below the scheme's limit
    t = B.Table(p2.m * 16, 16, "bp2ht", p2.a, p2.c)
    assert B.bht_build_workspace_bytes(t.handle, n) == 0
    B.bht_build_async_in(t.handle, dk, dv, ws)
    assert B.bht_build_wait(t.handle) == B.BHT_OK
    assert oracle.check32(p2, t.download(), keys, vals)[0] == 0
    t.close()


@pytest.mark.parametrize("scheme,b,n,cap", [
    ("bcht", 16, 1, 16), ("bcht", 16, 17, 32), ("bcht", 16, 500, 600), ("bcht", 4, 1000, 1200),
    ("bcht", 32, 5000, 6000), ("bcht", 8, 1 << 18, 300000), ("cht1", 1, 700, 1000),
    ("bcht", 16, (1 << 18) - 1, 300000), ("bcht", 16, 1 << 18, 300000),
])
def test_partitioned_build_edge_sizes(scheme, b, n, cap):
    """Tiny tables (one bucket, fewer buckets than a minimum bin), sizes at
    the default threshold, every bucket size: layouts valid, lookups exact,
    and both build modes answer alike."""
    import torch
    B = bht()
    keys, vals = workload(n, 71)
    h = 3
    for s in range(10):
        a, c = datagen.hash_constants(7100 + s, h)
        params = oracle.Params(scheme=scheme, b=b, m=-(-cap // b), h=h, a=a, c=c,
                               rng_seed=datagen.rng_seed(7100 + s))
        t, st = build_partitioned(params, keys, vals)
        if st == B.BHT_OK:
            break
        t.close()
    else:
        pytest.fail("no partitioned build succeeded")
    check_table(t, params, keys, vals, n_queries=max(2 * n, 64))
    t.close()
    t, st = build_partitioned(params, keys, vals, mode="auto")
    if st == B.BHT_OK:
        check_table(t, params, keys, vals, n_queries=max(2 * n, 64))
    t.close()
