"""Seeded input generators: distinct keys, no sentinel, disjoint negatives."""
import numpy as np

import datagen


def test_keys_unique_no_sentinel_and_seeded():
    k = datagen.unique_keys(1 << 18, 5)
    assert k.dtype == np.uint32 and len(np.unique(k)) == len(k)
    assert not np.any(k == np.uint32(0xFFFFFFFF))
    np.testing.assert_array_equal(k, datagen.unique_keys(1 << 18, 5))
    assert not np.array_equal(k[:100], datagen.unique_keys(100, 6))
    # prefix property: the first n keys do not depend on the total count
    np.testing.assert_array_equal(k[:1000], datagen.unique_keys(1000, 5))


def test_permutation_is_a_bijection():
    for n in (1, 2, 3, 1000, 65536, 100003):
        p = datagen.permutation(n, 4)
        np.testing.assert_array_equal(np.sort(p), np.arange(n))
    assert not np.array_equal(datagen.permutation(1000, 4), np.arange(1000))


def test_native_splitmix_matches_published_recurrence():
    seed = 1234567
    ref = datagen.splitmix64(seed, 100)          # numpy statement of the recurrence
    np.testing.assert_array_equal(datagen.splitmix64_native(seed, 100), ref)
    np.testing.assert_array_equal(datagen.splitmix64_native(seed, 10, start=90), ref[90:])
    # published first output of splitmix64 seeded with 0
    assert int(datagen.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF


def test_negatives_disjoint_and_mixed_fraction():
    n = 1 << 16
    keys = datagen.unique_keys(n, 9)
    neg = datagen.negative_keys(n, n, 9)
    assert len(np.intersect1d(keys, neg)) == 0
    assert not np.any(neg == np.uint32(0xFFFFFFFF))
    for frac in (0.0, 0.5, 1.0):
        q = datagen.mixed_queries(n, n, frac, 9)
        assert len(q) == n
        assert int(np.isin(q, keys).sum()) == int(frac * n)
    q = datagen.positive_queries(n, 9)
    np.testing.assert_array_equal(np.sort(q), np.sort(keys))


def test_hash_constants_in_range():
    a, c = datagen.hash_constants(1, 4)
    assert all(1 <= x < datagen.P32 for x in a) and all(0 <= x < datagen.P32 for x in c)
    a, c = datagen.hash_constants64(1, 3)
    assert all(1 <= x < datagen.P61 for x in a) and all(0 <= x < datagen.P61 for x in c)


def test_capacity_and_sizes():
    assert datagen.capacity_for(1 << 20, 0.9) == 1165085
    assert -(-datagen.capacity_for(1 << 28, 0.9) // 16) == 18641352
    s = datagen.log_uniform_sizes(4096, 10, 22, 1)
    assert s.min() >= 1 << 10 and s.max() < 1 << 22


def test_keys64():
    k = datagen.unique_keys64(1 << 16, 3)
    assert len(np.unique(k)) == len(k) and not np.any(k == np.uint64(2**64 - 1))
    neg = datagen.negative_keys64(1000, 1 << 16, 3)
    assert len(np.intersect1d(k, neg)) == 0


def test_queries_follow_the_key_stream():
    n = 5000
    keys = datagen.unique_keys(n, 3)
    pos = datagen.positive_queries(n, 3)
    np.testing.assert_array_equal(np.sort(pos), np.sort(keys))
    for count, frac in [(n, 0.5), (3 * n, 0.7), (100, 0.0), (2 * n, 1.0)]:
        q = datagen.mixed_queries(n, count, frac, 3)
        member = np.isin(q, keys)
        assert int(member.sum()) == int(frac * count)
        assert len(np.unique(q[~member])) == int((~member).sum())   # distinct negatives
    q64 = datagen.mixed_queries(n, n, 0.5, 3, wide=True)
    assert int(np.isin(q64, datagen.unique_keys64(n, 3)).sum()) == n // 2


def test_query_sources_name_each_query_key():
    """query_sources gives, for every query, its position in the key stream:
    the query equals that key, positions below n are inserted keys and the
    rest absent ones, for the positive batch and mixed batches alike."""
    n = 3000
    stream = datagen.unique_keys(n + 5000, 21)
    for frac, count, shuffle_seed in ((None, n, None), (0.0, 2500, None), (0.5, 4000, 9),
                                      (1.0, 4500, None), (0.7, 1234, 77)):
        if frac is None:
            q = datagen.positive_queries(n, 21)
        else:
            q = datagen.mixed_queries(n, count, frac, 21, shuffle_seed=shuffle_seed)
        src = datagen.query_sources(n, len(q), frac, 21, shuffle_seed=shuffle_seed)
        np.testing.assert_array_equal(stream[src], q)
        npos = n if frac is None else int(np.floor(frac * count))
        assert int((src < n).sum()) == npos


def test_serve_workload_positives_are_table_keys():
    from datagen import workloads
    specs = workloads.initial_tables(6, 5, (8, 12))
    sizes = [s["n"] for s in specs]
    stream = workloads.request_stream(sizes, 300, 1000.0, 99, build_fraction=0.1,
                                      lookup_log2=(4, 9), table_log2=(8, 10), tables_seed=5)
    all_sizes = workloads.table_sizes_after(sizes, stream)
    assert len(all_sizes) == len(sizes) + sum(r["kind"] == "build" for r in stream)
    arrivals = [r["arrival"] for r in stream]
    assert arrivals == sorted(arrivals) and arrivals[0] == 0.0
    hits = total = 0
    for r in stream:
        if r["kind"] != "lookup":
            continue
        spec = workloads.table_spec(5, r["table"], all_sizes[r["table"]])
        keys, _ = workloads.table_data(spec)
        hits += int(np.isin(r["queries"], keys).sum())
        total += len(r["queries"])
    assert abs(hits / total - 0.7) < 0.01
