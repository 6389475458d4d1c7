"""Autotuner for batched mode: picks bucket size, tile width, work-item size
and query unroll (queries per lane per chunk) for a batch of tables by
timing each candidate on the device.

It only orchestrates calls of the C ABI (tables are created per candidate,
because the bucket size changes their geometry); every build and query runs
in the library's kernels.  Results never depend on the choice: lookups are
exact for every bucket size, so the tuner compares speed only.
"""
from __future__ import annotations

import itertools
import time

BUCKETS = (8, 16, 32)
TILES = (4, 8, 16)
ITEMS = (2048, 8192)
UNROLLS = (1, 2)


def candidates(buckets=BUCKETS, tiles=TILES, items=ITEMS, unrolls=UNROLLS):
    """(bucket size, tile width, item size, query unroll) the library has
    kernels for."""
    supported = {(8, 4), (8, 8), (16, 4), (16, 8), (16, 16), (32, 8), (32, 16)}
    return [(b, w, it, u) for b, w, it, u in itertools.product(buckets, tiles, items, unrolls)
            if (b, w) in supported]


def time_batch(bht, torch, specs, b, w, item, unroll=1, reps=3, stream=None, all_times=None):
    """Median seconds of one batched build + query pass over the tables in
    `specs` (dicts with capacity, hash constants, device inputs and outputs),
    built with bucket size b, tile width w and query unroll.  Returns
    (seconds, statuses); every run's seconds are appended to all_times if
    it is a list."""
    tables = []
    try:
        for s in specs:
            t = bht.Table(s["capacity"], b, "bcht", s["a"], s["c"], rng_seed=s["rng_seed"], tile=w,
                          query_unroll=unroll)
            tables.append(t)
        entries = [(t.handle, s["keys"], s["vals"], s["queries"], s["out_v"], s["out_f"])
                   for t, s in zip(tables, specs)]
        batch = bht.bht_batch_create(entries, item_size=item)
        stream = stream or torch.cuda.Stream()
        times, sts = [], None
        try:
            with torch.cuda.stream(stream):
                bht.bht_batch_run(batch, stream=stream)        # capture + first run
                bht.bht_batch_wait(batch, len(tables), stream=stream)
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    bht.bht_batch_run(batch, stream=stream)
                    _, sts = bht.bht_batch_wait(batch, len(tables), stream=stream)
                    times.append(time.perf_counter() - t0)
        finally:
            bht.bht_batch_destroy(batch)
        if all_times is not None:
            all_times.extend(times)
        times.sort()
        return times[len(times) // 2], sts
    finally:
        for t in tables:
            t.close()


def tune(bht, torch, specs, cands=None, reps=3, log=None):
    """Times every candidate on `specs`; returns (best candidate, table of
    {candidate: seconds})."""
    cands = cands or candidates()
    results = {}
    for b, w, item, unroll in cands:
        sec, sts = time_batch(bht, torch, specs, b, w, item, unroll=unroll, reps=reps)
        if sts is not None and any(s != bht.BHT_OK for s in sts):
            sec = float("inf")       # a configuration that cannot build every table loses
        results[(b, w, item, unroll)] = sec
        if log:
            log("autotune b=%d tile=%d item=%d unroll=%d: %.3f ms" % (b, w, item, unroll, sec * 1e3))
    best = min(results, key=results.get)
    return best, results
