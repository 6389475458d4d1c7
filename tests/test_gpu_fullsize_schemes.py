"""Parity at the scheme comparison's full size (2^27 keys) for the tables
whose default build at that size is a partitioned one besides the 2^28
BCHT: the 64-bit BCHT (8 16-byte slots per bucket, LF 0.9), the two-level
iceberg table (16-slot primaries, 8-slot secondaries of 1/8 the primary
slots, t = 16, LF 0.85) and the one-slot cuckoo table (h = 3, LF 0.8),
built and queried as the benchmark does.

Also the power-of-two-choice table (h = 2, 16-slot buckets, LF 0.82, the
highest load it reaches reliably) and the paper's one-level iceberg table
(t = 13 of 16 slots, LF 0.82), whose builds are the concurrent kernels.

The whole GPU layout goes through the oracle's invariant checker, and every
(found, value) result of the three query batches (100, 0 and 50% positive)
is compared with the plain lookup definition (the oracle's sort-merge join
of the input pairs with the queries)."""
import numpy as np
import pytest

import datagen
import oracle
from tests._util import dev, host_u32, host_u64, host_u8
from tests.test_gpu_schemes import iceberg_params

pytestmark = pytest.mark.gpu

N = 1 << 27


def check_batches(t, keys, vals, wide, seed):
    import torch
    join = oracle.join_find64 if wide else oracle.join_find32
    for frac in (1.0, 0.0, 0.5):
        q = datagen.mixed_queries(N, N, frac, seed, wide=wide)
        v, f = t.find(dev(q))
        torch.cuda.synchronize()
        hv = host_u64(v) if wide else host_u32(v)
        hf = host_u8(f)
        del v, f
        ev, ef = join(keys, vals, q)
        assert int(ef.sum()) == int(frac * N), frac
        np.testing.assert_array_equal(hf, ef)
        np.testing.assert_array_equal(hv, ev)
        print("  batch %.1f positive: all %d results equal" % (frac, N), flush=True)


def test_full_size_64bit():
    import paper_2108_07232_amd as bht
    print("full-size parity: 64-bit BCHT, 2^27 keys, LF 0.9", flush=True)
    keys, vals = datagen.unique_keys64(N, 1), datagen.values64(N, 1)
    for s in range(4):
        p = oracle.params_for("bcht", N, 0.9, 1 + s, b=8, wide=True)
        t = bht.Table(p.m * 8, 8, "bcht", p.a, p.c, key_bits=64, rng_seed=p.rng_seed)
        st = t.build(dev(keys), dev(vals))
        if st == bht.BHT_OK:
            break
        assert st == bht.BHT_ERR_BUILD_FAILED
        t.close()
    assert st == bht.BHT_OK
    assert bht.bht_build_stats(t.handle)[0]            # the partitioned path
    code, msg = oracle.check64(p, t.download(), keys, vals)
    assert code == 0, msg
    print("  layout checked", flush=True)
    check_batches(t, keys, vals, True, 1)
    t.close()


def test_full_size_iceberg_two_level():
    import paper_2108_07232_amd as bht
    print("full-size parity: two-level iceberg, 2^27 keys, LF 0.85", flush=True)
    keys, vals = datagen.unique_keys(N, 2), datagen.values(N, 2)
    for s in range(4):
        p = iceberg_params(N, 0.85, 20 + s, b=16, b2=8, threshold=16)
        t = bht.Table(p.m * p.b, p.b, p.scheme, p.a, p.c, rng_seed=p.rng_seed,
                      iht_threshold=p.threshold, iht_secondary_b=p.b2, iht_secondary_m=p.m2)
        st = t.build(dev(keys), dev(vals))
        if st == bht.BHT_OK:
            break
        assert st == bht.BHT_ERR_BUILD_FAILED
        t.close()
    assert st == bht.BHT_OK
    assert bht.bht_build_stats(t.handle)[0]            # the partitioned path
    code, msg = oracle.check32(p, t.download(), keys, vals)
    assert code == 0, msg
    print("  layout checked", flush=True)
    check_batches(t, keys, vals, False, 2)
    t.close()


def test_full_size_one_slot_cuckoo():
    import paper_2108_07232_amd as bht
    print("full-size parity: 1CHT (b = 1, h = 3), 2^27 keys, LF 0.8", flush=True)
    keys, vals = datagen.unique_keys(N, 3), datagen.values(N, 3)
    for s in range(4):
        p = oracle.params_for("cht1", N, 0.8, 30 + s, b=1)
        t = bht.Table(p.m, 1, "cht1", p.a, p.c, rng_seed=p.rng_seed)
        st = t.build(dev(keys), dev(vals))
        if st == bht.BHT_OK:
            break
        assert st == bht.BHT_ERR_BUILD_FAILED
        t.close()
    assert st == bht.BHT_OK
    assert bht.bht_build_stats(t.handle)[0]            # the partitioned path
    code, msg = oracle.check32(p, t.download(), keys, vals)
    assert code == 0, msg
    print("  layout checked", flush=True)
    check_batches(t, keys, vals, False, 3)
    t.close()


def test_full_size_power_of_two():
    import paper_2108_07232_amd as bht
    print("full-size parity: BP2HT (b = 16, h = 2), 2^27 keys, LF 0.82", flush=True)
    keys, vals = datagen.unique_keys(N, 4), datagen.values(N, 4)
    for s in range(4):
        p = oracle.params_for("bp2ht", N, 0.82, 40 + s, b=16)
        t = bht.Table(p.m * 16, 16, "bp2ht", p.a, p.c, rng_seed=p.rng_seed)
        st = t.build(dev(keys), dev(vals))
        if st == bht.BHT_OK:
            break
        assert st == bht.BHT_ERR_BUILD_FAILED
        t.close()
    assert st == bht.BHT_OK
    code, msg = oracle.check32(p, t.download(), keys, vals)
    assert code == 0, msg
    print("  layout checked", flush=True)
    check_batches(t, keys, vals, False, 4)
    t.close()


def test_full_size_iceberg_one_level():
    import paper_2108_07232_amd as bht
    print("full-size parity: one-level iceberg (b = 16, t = 13), 2^27 keys, LF 0.82", flush=True)
    keys, vals = datagen.unique_keys(N, 5), datagen.values(N, 5)
    for s in range(4):
        p = iceberg_params(N, 0.82, 50 + s, b=16, threshold=13)
        t = bht.Table(p.m * p.b, p.b, p.scheme, p.a, p.c, rng_seed=p.rng_seed,
                      iht_threshold=p.threshold)
        st = t.build(dev(keys), dev(vals))
        if st == bht.BHT_OK:
            break
        assert st == bht.BHT_ERR_BUILD_FAILED
        t.close()
    assert st == bht.BHT_OK
    code, msg = oracle.check32(p, t.download(), keys, vals)
    assert code == 0, msg
    print("  layout checked", flush=True)
    check_batches(t, keys, vals, False, 5)
    t.close()
