"""Parity at the benchmark's full size (2^28 keys, LF 0.9, 16-slot buckets),
in the launch configuration the benchmark times.

Every query is checked against properties that hold at any size (each
positive query is found, no negative query is found, a half-positive batch
finds exactly half); a sample of each batch is checked value for value
against the oracle's brute-force lookup; the whole GPU layout is checked
with the oracle's invariant checker."""
import numpy as np
import pytest

import datagen
import oracle
from tests._util import dev, host_u32, host_u8

pytestmark = pytest.mark.gpu

N = 1 << 28
SAMPLE = 1 << 20


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
    rng = np.random.default_rng(0)
    samples = []
    for frac in (1.0, 0.0, 0.5):
        q = datagen.mixed_queries(N, N, frac, 1) if frac < 1 else datagen.positive_queries(N, 1)
        v, f = t.find(dev(q))
        torch.cuda.synchronize()
        hf = host_u8(f)
        assert int(hf.sum()) == int(frac * N), frac
        idx = rng.choice(N, SAMPLE, replace=False)
        samples.append((q[idx], host_u32(v)[idx], hf[idx]))
        del v, f
    q = np.concatenate([s[0] for s in samples])
    ev, ef = oracle.brute_find32(keys, vals, q)
    np.testing.assert_array_equal(np.concatenate([s[2] for s in samples]), ef)
    np.testing.assert_array_equal(np.concatenate([s[1] for s in samples]), ev)
    t.close()
