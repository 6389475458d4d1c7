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


def test_feistel_is_a_bijection_on_a_sample():
    x = np.arange(0, 1 << 20, dtype=np.uint32)
    y = datagen.feistel32(x, [1, 2, 3, 4])
    assert len(np.unique(y)) == len(x)


def test_negatives_disjoint_and_mixed_fraction():
    n = 1 << 16
    keys = datagen.unique_keys(n, 9)
    neg = datagen.negative_keys(n, n, 9)
    assert len(np.intersect1d(keys, neg)) == 0
    assert not np.any(neg == np.uint32(0xFFFFFFFF))
    for frac in (0.0, 0.5, 1.0):
        q = datagen.mixed_queries(keys, n, frac, 9)
        assert len(q) == n
        assert int(np.isin(q, keys).sum()) == int(frac * n)
    q = datagen.positive_queries(keys, 9)
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
