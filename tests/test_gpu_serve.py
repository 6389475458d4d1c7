"""Serving loop: requests that arrive while others run are admitted and
coalesced into shared launches; every lookup's result must be the same as
the same lookup run alone, and equal brute force, bit for bit."""
import numpy as np
import pytest

import datagen
import oracle
from datagen import workloads
from tests._util import host_u32, host_u8

pytestmark = pytest.mark.gpu


def table_data(seed, tid, n):
    return workloads.table_data(workloads.table_spec(seed, tid, n))


def reseed(spec, attempt):
    return datagen.hash_constants(spec["seed"] + 7919 * attempt, 3)


def run_case(budget, count=400, rate=2e5, seed=7, headroom=None):
    import torch

    from paper_2108_07232_amd import serve
    specs = workloads.initial_tables(12, seed, log2_range=(8, 14))
    tables = serve.build_resident_tables(torch, specs, workloads.table_data, reseed=reseed)
    sizes = [s["n"] for s in specs]
    stream = workloads.request_stream(sizes, count, rate, seed, build_fraction=0.1,
                                      lookup_log2=(4, 12), table_log2=(8, 14))
    reqs = serve.make_requests(torch, stream, workloads.table_data)
    if headroom is not None:      # budget = the resident set plus a little room
        budget = sum(t.info[3] for t in tables) + headroom
    srv = serve.Server(torch, budget, streams=3, max_batch=64, item_size=512)
    for tid, t in enumerate(tables):
        srv.add_table(tid, t)
    srv.run(reqs, time_limit=60)
    return srv, tables, sizes, reqs


def all_sizes(sizes, reqs):
    out = list(sizes)
    for r in reqs:
        if r.kind == "build":
            out.append(r.keys.numel())
    return out


def test_mixed_results_equal_alone_and_bruteforce():
    import torch
    import paper_2108_07232_amd as bht
    srv, tables, sizes, reqs = run_case(budget=1 << 40)
    assert srv.evicted == 0
    lookups = [r for r in reqs if r.kind == "lookup"]
    assert all(r.status == bht.BHT_OK for r in reqs), [r.status for r in reqs if r.status != 0]
    # coalescing happened: fewer launches than requests
    assert srv.launches < len(reqs)
    assert max(np.bincount([r.launch for r in lookups])) > 1
    sz = all_sizes(sizes, reqs)
    for r in lookups:
        t = srv.tables[r.table]
        v_alone, f_alone = t.find(r.queries)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host_u32(r.out_v), host_u32(v_alone))
        np.testing.assert_array_equal(host_u8(r.out_f), host_u8(f_alone))
        keys, vals = table_data(7, r.table, sz[r.table])
        q = host_u32(r.queries)
        bv, bf = oracle.brute_find32(keys, vals, q)
        np.testing.assert_array_equal(host_u8(r.out_f), bf)
        np.testing.assert_array_equal(host_u32(r.out_v), bv)
    srv.close()


def test_budget_evicts_least_recently_used_never_in_use():
    import paper_2108_07232_amd as bht
    srv, tables, sizes, reqs = run_case(budget=0, seed=8, headroom=200 << 10)
    assert srv.evicted > 0
    assert srv.bytes <= srv.budget
    sz = all_sizes(sizes, reqs)
    ok = [r for r in reqs if r.kind == "lookup" and r.status == bht.BHT_OK]
    assert len(ok) > 0
    for r in ok:
        keys, vals = table_data(8, r.table, sz[r.table])
        bv, bf = oracle.brute_find32(keys, vals, host_u32(r.queries))
        np.testing.assert_array_equal(host_u8(r.out_f), bf)
        np.testing.assert_array_equal(host_u32(r.out_v), bv)
    # a lookup only fails when its table was gone before the lookup arrived
    for r in reqs:
        if r.kind == "lookup" and r.status != bht.BHT_OK:
            assert r.status == bht.BHT_ERR_NOT_BUILT
    srv.close()
