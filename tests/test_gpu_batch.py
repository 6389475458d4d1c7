"""Batched mode: many tables of uneven sizes built and queried by the
persistent kernels, captured in a HIP graph and replayed.  Every table's
results must equal brute force and the per-table (plain) calls, on every
replay."""
import numpy as np
import pytest

import datagen
import oracle
from tests._util import dev, host_u32, host_u8

pytestmark = pytest.mark.gpu


def make_tables(count, lo, hi, seed, b=16, tile=8, lf=0.9, unroll=0, sizes=None):
    import torch
    import paper_2108_07232_amd as bht
    if sizes is None:
        sizes = datagen.log_uniform_sizes(count, lo, hi, seed)
    else:
        sizes = np.asarray(sizes, dtype=np.int64)
    tabs = []
    for i, n in enumerate(sizes.tolist()):
        s = seed * 100000 + i
        keys, vals = datagen.unique_keys(n, s), datagen.values(n, s)
        q = datagen.mixed_queries(n, n, 0.5, s)
        p = oracle.params_for("bcht", n, lf, s, b=b)
        t = bht.Table(p.m * p.b, b, "bcht", p.a, p.c, rng_seed=p.rng_seed, tile=tile,
                      query_unroll=unroll)
        tabs.append(dict(n=n, keys=keys, vals=vals, q=q, params=p, table=t,
                         dk=dev(keys), dv=dev(vals), dq=dev(q),
                         ov=torch.full((n,), 7, dtype=torch.int32, device="cuda"),
                         of=torch.full((n,), 9, dtype=torch.uint8, device="cuda")))
    return tabs


def check_outputs(tabs, statuses):
    import paper_2108_07232_amd as bht
    for d, st in zip(tabs, statuses):
        if st != bht.BHT_OK:
            continue
        bv, bf = oracle.join_find32(d["keys"], d["vals"], d["q"])
        np.testing.assert_array_equal(host_u8(d["of"]), bf)
        np.testing.assert_array_equal(host_u32(d["ov"]), bv)


@pytest.mark.parametrize("b,tile,unroll", [(16, 8, 1), (8, 8, 1), (32, 16, 1), (16, 4, 1),
                                           (16, 8, 2), (32, 16, 2)])
def test_batch_matches_bruteforce_and_replays(b, tile, unroll):
    import torch
    import paper_2108_07232_amd as bht
    tabs = make_tables(150, 6, 15, 3 + b, b=b, tile=tile, unroll=unroll)
    entries = [(d["table"].handle, d["dk"], d["dv"], d["dq"], d["ov"], d["of"]) for d in tabs]
    batch = bht.bht_batch_create(entries, item_size=1024)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    for replay in range(3):
        with torch.cuda.stream(side):
            bht.bht_batch_run(batch, stream=side)
            rc, sts = bht.bht_batch_wait(batch, len(tabs), stream=side)
        assert sts.count(bht.BHT_OK) >= len(tabs) - 2, sts
        check_outputs(tabs, sts)
        for d, st in zip(tabs[:20], sts[:20]):
            if st == bht.BHT_OK:
                code, msg = oracle.check32(d["params"], d["table"].download(), d["keys"], d["vals"])
                assert code == 0, msg
        # eager work between replays: scribble over the outputs
        for d in tabs:
            d["ov"].fill_(123)
            d["of"].fill_(5)
        torch.cuda.synchronize()
    bht.bht_batch_destroy(batch)
    for d in tabs:
        d["table"].close()


def test_batch_equals_plain_calls_and_reports_failures():
    import torch
    import paper_2108_07232_amd as bht
    tabs = make_tables(40, 8, 14, 11)
    # one table that must fail: eviction cap 0 on a full table
    bad = tabs[7]
    p = bad["params"]
    bad["table"].close()
    n = bad["n"]
    bad["table"] = bht.Table(n, 16, "bcht", p.a, p.c, tile=8, max_chain=0)
    entries = [(d["table"].handle, d["dk"], d["dv"], d["dq"], d["ov"], d["of"]) for d in tabs]
    batch = bht.bht_batch_create(entries)
    bht.bht_batch_run(batch)              # null stream: direct launches
    rc, sts = bht.bht_batch_wait(batch, len(tabs))
    assert rc == bht.BHT_ERR_BUILD_FAILED and sts[7] == bht.BHT_ERR_BUILD_FAILED
    assert all(s == bht.BHT_OK for i, s in enumerate(sts) if i != 7)
    check_outputs(tabs, sts)
    with pytest.raises(bht.BhtError):
        bad["table"].find(bad["dq"])       # a failed table is not built
    batched = [(host_u32(d["ov"]).copy(), host_u8(d["of"]).copy()) for d in tabs]
    for i, d in enumerate(tabs):
        if i == 7:
            continue
        assert d["table"].build(d["dk"], d["dv"]) == bht.BHT_OK
        v, f = d["table"].find(d["dq"])
        np.testing.assert_array_equal(host_u32(v), batched[i][0])
        np.testing.assert_array_equal(host_u8(f), batched[i][1])
    bht.bht_batch_destroy(batch)
    for d in tabs:
        d["table"].close()


def test_batch_rejects_mixed_query_unroll():
    import paper_2108_07232_amd as bht
    tabs = make_tables(4, 8, 10, 21, unroll=2)
    bht.bht_set_tuning(tabs[2]["table"].handle, 8, 0, 0, 0, False, 1)
    entries = [(d["table"].handle, d["dk"], d["dv"], d["dq"], d["ov"], d["of"]) for d in tabs]
    with pytest.raises(bht.BhtError) as e:
        bht.bht_batch_create(entries)
    assert e.value.status == bht.BHT_ERR_INVALID_ARG
    for d in tabs:
        d["table"].close()


def test_batch_build_paths_agree():
    """The partitioned batched build (default) and the persistent concurrent
    build (chosen when any table asks for the concurrent build) both give
    valid layouts and identical query results, table by table."""
    import torch
    import paper_2108_07232_amd as bht
    outs = []
    for concurrent in (False, True):
        tabs = make_tables(60, 6, 17, 31)
        if concurrent:
            bht.bht_set_tuning(tabs[0]["table"].handle, 8, 0, 0, "concurrent")
        entries = [(d["table"].handle, d["dk"], d["dv"], d["dq"], d["ov"], d["of"]) for d in tabs]
        batch = bht.bht_batch_create(entries, item_size=2048)
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            for _ in range(2):                      # capture, then a replay
                bht.bht_batch_run(batch, stream=side)
                rc, sts = bht.bht_batch_wait(batch, len(tabs), stream=side)
        assert rc == bht.BHT_OK, sts
        check_outputs(tabs, sts)
        for d in tabs[::7]:
            code, msg = oracle.check32(d["params"], d["table"].download(), d["keys"], d["vals"])
            assert code == 0, msg
        outs.append([(host_u32(d["ov"]).copy(), host_u8(d["of"]).copy()) for d in tabs])
        bht.bht_batch_destroy(batch)
        for d in tabs:
            d["table"].close()
    for (v0, f0), (v1, f1) in zip(*outs):
        np.testing.assert_array_equal(v0, v1)
        np.testing.assert_array_equal(f0, f1)


def test_batch_large_tables():
    """Tables at the top of the batched workload's size range (2^21 to 2^22
    keys: bins of 512 buckets, several radix digits per table) next to small
    ones, on a capture and a replay; every result equals the plain lookup
    definition and every large layout passes the invariant checker."""
    import torch
    import paper_2108_07232_amd as bht
    sizes = [1 << 22, (1 << 21) + 12345, 3000000, 1 << 10, 777, (1 << 20) + 1, (1 << 22) - 5,
             2500000]
    tabs = make_tables(len(sizes), 0, 0, 41, sizes=sizes)
    entries = [(d["table"].handle, d["dk"], d["dv"], d["dq"], d["ov"], d["of"]) for d in tabs]
    batch = bht.bht_batch_create(entries, item_size=2048)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    for replay in range(2):
        print("  batch of %d tables up to 2^22 keys, run %d" % (len(sizes), replay), flush=True)
        with torch.cuda.stream(side):
            bht.bht_batch_run(batch, stream=side)
            rc, sts = bht.bht_batch_wait(batch, len(tabs), stream=side)
        assert rc == bht.BHT_OK, sts
        check_outputs(tabs, sts)
        for d in tabs:
            if d["n"] >= (1 << 21):
                code, msg = oracle.check32(d["params"], d["table"].download(), d["keys"],
                                           d["vals"])
                assert code == 0, msg
        for d in tabs:
            d["ov"].fill_(123)
            d["of"].fill_(5)
        torch.cuda.synchronize()
    bht.bht_batch_destroy(batch)
    for d in tabs:
        d["table"].close()


def test_batch_build_find_one_call():
    """The one-call batched entry point gives the same results as plain
    per-table calls and the plain lookup definition, and reports a failing
    table."""
    import paper_2108_07232_amd as bht
    tabs = make_tables(30, 6, 16, 51)
    bad = tabs[4]
    p = bad["params"]
    bad["table"].close()
    bad["table"] = bht.Table(bad["n"], 16, "bcht", p.a, p.c, tile=8, max_chain=0)
    entries = [(d["table"].handle, d["dk"], d["dv"], d["dq"], d["ov"], d["of"]) for d in tabs]
    rc, sts = bht.bht_batch_build_find(entries, item_size=1024)
    assert rc == bht.BHT_ERR_BUILD_FAILED and sts[4] == bht.BHT_ERR_BUILD_FAILED
    assert all(s == bht.BHT_OK for i, s in enumerate(sts) if i != 4)
    check_outputs(tabs, sts)
    for d in tabs[::6]:
        if d is bad:
            continue
        code, msg = oracle.check32(d["params"], d["table"].download(), d["keys"], d["vals"])
        assert code == 0, msg
    for d in tabs:
        d["table"].close()
