"""Seeded random sweep over schemes, bucket sizes, sizes (ragged, tiny, at
and around the partitioned threshold), load factors and build modes: every
successful build passes the oracle's invariant checker and every lookup
equals brute force.  Builds that fail near a scheme's load limit are
reported, not errors."""
import numpy as np
import pytest

import datagen
import oracle
from tests._util import dev, host_u32, host_u64, host_u8
from tests.test_gpu_schemes import iceberg_params

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 63, 64, 65, 1000, 4097, 30000, 100003, 262143, 262144, 300007]


def make_case(rng):
    kind = str(rng.choice(["bcht", "bcht", "cht1", "iht1", "iht2", "bp2ht", "lb", "wide"]))
    n = int(rng.choice(SIZES))
    mode = str(rng.choice(["auto", "concurrent", "partitioned"]))
    seed = int(rng.integers(1, 1 << 30))
    if kind == "wide":
        return kind, n, mode, seed, oracle.params_for("bcht", n, float(rng.uniform(0.3, 0.93)),
                                                      seed, b=8, wide=True)
    if kind in ("iht1", "iht2"):
        b = int(rng.choice([16, 32]))
        b2 = 8 if kind == "iht2" else 0
        thr = int(rng.integers(1, b + 1)) if b2 == 0 else b
        return kind, n, mode, seed, iceberg_params(n, float(rng.uniform(0.3, 0.8)), seed, b=b,
                                                   b2=b2, threshold=thr)
    if kind == "bp2ht":
        return kind, n, mode, seed, oracle.params_for(
            "bp2ht", n, float(rng.uniform(0.3, 0.6)), seed, b=int(rng.choice([8, 16, 32])))
    if kind == "lb":
        return kind, n, mode, seed, oracle.params_for(
            "bcht_lb", n, float(rng.uniform(0.3, 0.9)), seed, b=int(rng.choice([8, 16, 32])))
    if kind == "cht1":
        return kind, n, mode, seed, oracle.params_for("cht1", n, float(rng.uniform(0.3, 0.8)),
                                                      seed, b=1)
    return kind, n, mode, seed, oracle.params_for(
        "bcht", n, float(rng.uniform(0.3, 0.93)), seed, b=int(rng.choice([4, 8, 16, 32])))


@pytest.mark.parametrize("block", range(4))
def test_random_configurations(block):
    import torch
    import paper_2108_07232_amd as B
    rng = np.random.default_rng(1000 + block)
    built = 0
    for c in range(30):
        kind, n, mode, seed, p = make_case(rng)
        print("sweep %d.%d %s n=%d mode=%s seed=%d" % (block, c, kind, n, mode, seed), flush=True)
        wide = kind == "wide"
        if wide:
            keys, vals = datagen.unique_keys64(n, seed % 1000), datagen.values64(n, seed % 1000)
            t = B.Table(p.m * 8, 8, "bcht", p.a, p.c, key_bits=64, rng_seed=p.rng_seed,
                        build_mode=mode)
        else:
            keys, vals = datagen.unique_keys(n, seed % 1000), datagen.values(n, seed % 1000)
            t = B.Table(p.m * p.b, p.b, p.scheme, p.a, p.c, rng_seed=p.rng_seed,
                        max_chain=p.max_chain, iht_threshold=p.threshold, iht_secondary_b=p.b2,
                        iht_secondary_m=p.m2, build_mode=mode)
        st = t.build(dev(keys), dev(vals))
        if st != B.BHT_OK:
            assert st == B.BHT_ERR_BUILD_FAILED, B.bht_status_string(st)
            t.close()
            continue
        built += 1
        layout = t.download()
        q = datagen.mixed_queries(n, max(2 * n, 64), 0.5, seed % 997, wide=wide)
        v, f = t.find(dev(q))
        torch.cuda.synchronize()
        if wide:
            code, msg = oracle.check64(p, layout, keys, vals)
            bv, bf = oracle.brute_find64(keys, vals, q)
            np.testing.assert_array_equal(host_u64(v), bv)
        else:
            code, msg = oracle.check32(p, layout, keys, vals)
            bv, bf = oracle.brute_find32(keys, vals, q)
            np.testing.assert_array_equal(host_u32(v), bv)
        assert code == 0, msg
        np.testing.assert_array_equal(host_u8(f), bf)
        t.close()
    assert built >= 25
