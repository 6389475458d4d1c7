"""Parity at the benchmark's full size (2^28 keys, LF 0.9, 16-slot buckets),
in the launch configuration the benchmark times.

The whole GPU layout is checked with the oracle's invariant checker, and
every one of the 3 x 2^28 (found, value) results is compared with the plain
lookup definition (the oracle's sort-merge join of the input pairs with the
queries, Sections I and III: a stored key returns its value, any other
query is reported missing)."""
import numpy as np
import pytest

import datagen
import oracle
from tests._util import dev, host_u32, host_u8

pytestmark = pytest.mark.gpu

N = 1 << 28


def test_full_size_build_and_find():
    import torch
    import paper_2108_07232_amd as bht
    print("full-size parity: 2^28 keys, LF 0.9", flush=True)
    keys, vals = datagen.unique_keys(N, 1), datagen.values(N, 1)
    params = oracle.params_for("bcht", N, 0.9, 1)
    t = bht.Table(params.m * params.b, 16, "bcht", params.a, params.c, rng_seed=params.rng_seed)
    dk, dv = dev(keys), dev(vals)
    st = t.build(dk, dv)
    assert st == bht.BHT_OK, bht.bht_status_string(st)
    del dk, dv
    layout = t.download()
    code, msg = oracle.check32(params, layout, keys, vals)
    assert code == 0, msg
    del layout
    print("  layout checked", flush=True)
    for frac in (1.0, 0.0, 0.5):
        q = datagen.mixed_queries(N, N, frac, 1) if frac < 1 else datagen.positive_queries(N, 1)
        v, f = t.find(dev(q))
        torch.cuda.synchronize()
        hv, hf = host_u32(v), host_u8(f)
        del v, f
        ev, ef = oracle.join_find32(keys, vals, q)
        assert int(ef.sum()) == int(frac * N), frac
        np.testing.assert_array_equal(hf, ef)
        np.testing.assert_array_equal(hv, ev)
        print("  batch %.1f positive: all %d results equal" % (frac, N), flush=True)
    t.close()
