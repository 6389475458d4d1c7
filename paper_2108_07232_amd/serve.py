"""Serving loop with continuous batching over many resident tables.

Requests arrive over time (an open-loop arrival schedule): a *build*
creates a new table from caller-supplied device keys and values, a *lookup*
answers a query batch against a resident table.  The loop admits requests
as they arrive, keeps tables resident in HBM under a byte budget that
covers the tables and the per-stream build workspaces (least recently used
tables are evicted when a build needs room; a table with lookups waiting or
in flight is never evicted; request keys, queries and outputs are the
caller's and outside the budget), and launches every lookup
that is ready, from any number of tables, as one coalesced query launch on
a free stream, so new work is admitted while earlier launches still run.
Completion is observed with events; a request's latency runs from its
arrival to the end of the launch that answered it.

Host-side orchestration only: building and querying run in the library's
kernels (bht_build_async_in with a per-stream workspace, bht_multi_find).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import paper_2108_07232_amd as bht


@dataclass
class Request:
    kind: str                      # "build" or "lookup"
    arrival: float                 # seconds from the start of the run
    table: int                     # table id (new id for a build)
    queries: object = None         # lookup: device tensor (int32 bits)
    out_v: object = None           # lookup: device output tensors
    out_f: object = None
    keys: object = None            # build: device tensors
    vals: object = None
    capacity: int = 0              # build: slots
    a: tuple = ()                  # build: hash constants
    c: tuple = ()
    rng_seed: int = 0
    # filled by the server
    done: float = -1.0
    status: int = -1
    launch: int = -1               # index of the launch that answered it


@dataclass
class _Slot:
    stream: object
    ctx: object
    event: object = None            # set while a launch is in flight
    requests: list = field(default_factory=list)
    kind: str = ""
    done_event: object = None       # reused for every launch of this slot
    workspace: object = None        # build slots: device workspace of the partitioned build


class Server:
    """Continuous-batching server (see module docstring)."""

    def __init__(self, torch, budget_bytes: int, streams: int = 4, build_streams: int = 2,
                 max_batch: int = 1024, max_items: int = 1 << 16, item_size: int = 4096,
                 bucket: int = 16, workspace_bytes: int = 0):
        self.torch = torch
        self.budget = budget_bytes
        self.bucket = bucket
        self.max_batch = max_batch
        self.item_size = item_size
        self.tables = collections.OrderedDict()      # id -> bht.Table, LRU order
        self.ready = set()                           # ids of built tables
        self.bytes = 0
        self.evicted = 0
        self.launches = 0
        self.pins = collections.Counter()            # lookups waiting/in flight per table
        self.lookup_slots = [_Slot(torch.cuda.Stream(), bht.bht_find_ctx_create(max_batch, max_items))
                             for _ in range(streams)]
        self.build_slots = [_Slot(torch.cuda.Stream(), None) for _ in range(build_streams)]
        for slot in self.lookup_slots + self.build_slots:
            slot.done_event = torch.cuda.Event()
        # one build workspace per build stream (reused: a slot runs one build
        # at a time), so builds never allocate in the loop; grown on demand
        self.ws_bytes = 0                            # build workspaces, inside the budget
        for slot in self.build_slots:
            if workspace_bytes:
                slot.workspace = torch.empty(workspace_bytes, dtype=torch.uint8, device="cuda")
                self.ws_bytes += workspace_bytes
        self.building = set()                        # ids with a build waiting or running

    def close(self):
        self.torch.cuda.synchronize()
        for s in self.lookup_slots:
            bht.bht_find_ctx_destroy(s.ctx)
        for t in self.tables.values():
            t.close()
        self.tables.clear()

    def warmup(self, keys, vals):
        """Runs one build and one coalesced lookup on every stream so that
        kernel code objects and allocator pools are loaded before timing.
        keys / vals: a few device key-value pairs (int32 bits)."""
        torch = self.torch
        for slot in self.build_slots:
            with torch.cuda.stream(slot.stream):
                params = bht.make_params([3, 5, 7], [11, 13, 17])
                nbytes = bht.bht_table_bytes(4 * keys.numel(), self.bucket, "bcht", params)
                buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
                t = bht.Table(4 * keys.numel(), self.bucket, "bcht", [3, 5, 7], [11, 13, 17],
                              buffer=buf)
                self._build(slot, t, keys, vals)
                bht.bht_build_wait(t.handle, stream=slot.stream)
                for ls in self.lookup_slots:
                    ov = torch.empty(keys.numel(), dtype=torch.int32, device="cuda")
                    of = torch.empty(keys.numel(), dtype=torch.uint8, device="cuda")
                    bht.bht_multi_find(ls.ctx, [(t.handle, keys, ov, of)], self.item_size,
                                       stream=ls.stream)
                    ls.stream.synchronize()
                t.close()
        torch.cuda.synchronize()

    def _build(self, slot, table, keys, vals):
        """Enqueues a build on the slot's stream, through the partitioned
        path with the slot's workspace when the table takes it."""
        need = bht.bht_build_workspace_bytes(table.handle, keys.numel())
        if need == 0:
            bht.bht_build_async(table.handle, keys, vals, stream=slot.stream)
            return
        if slot.workspace is None or slot.workspace.numel() < need:
            # a grown workspace counts against the budget like a table
            old = 0 if slot.workspace is None else slot.workspace.numel()
            slot.workspace = None
            self.ws_bytes -= old
            self._make_room(need)
            slot.workspace = self.torch.empty(need, dtype=self.torch.uint8, device="cuda")
            self.ws_bytes += need
        bht.bht_build_async_in(table.handle, keys, vals, slot.workspace, stream=slot.stream)

    # ------------------------------------------------------------- tables

    def add_table(self, tid: int, table) -> None:
        """Registers an already built table (the initial resident set)."""
        self.tables[tid] = table
        self.ready.add(tid)
        self.bytes += table.info[3]

    def _make_room(self, need: int) -> bool:
        while self.bytes + self.ws_bytes + need > self.budget:
            victim = next((tid for tid in self.tables if self.pins[tid] == 0 and tid in self.ready),
                          None)
            if victim is None:
                return False
            t = self.tables.pop(victim)
            self.ready.discard(victim)
            self.bytes -= t.info[3]
            t.close()
            self.evicted += 1
        return True

    # --------------------------------------------------------------- loop

    def _poll(self, now_fn) -> int:
        """Retires finished launches; returns the number of requests completed."""
        completed = 0
        for slot in self.lookup_slots + self.build_slots:
            if slot.event is not None and slot.event.query():
                now = now_fn()
                if slot.kind == "build":
                    req = slot.requests[0]
                    st = bht.bht_build_wait(self.tables[req.table].handle, stream=slot.stream)
                    req.status = st
                    self.building.discard(req.table)
                    if st == bht.BHT_OK:
                        self.ready.add(req.table)
                    else:
                        t = self.tables.pop(req.table)
                        self.bytes -= t.info[3]
                        t.close()
                    req.done = now
                    completed += 1
                else:
                    for req in slot.requests:
                        req.done = now
                        req.status = bht.BHT_OK
                        self.pins[req.table] -= 1
                    completed += len(slot.requests)
                slot.event, slot.requests, slot.kind = None, [], ""
        return completed

    def run(self, requests, time_limit: float = 120.0):
        """Serves `requests` (sorted by arrival); returns them with done,
        status and launch filled in."""
        torch = self.torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        pending_builds = collections.deque()
        pending_lookups = collections.deque()
        nxt, completed = 0, 0
        while completed < len(requests):
            t = now()
            if t > time_limit:
                raise RuntimeError("serving run exceeded %.0f s" % time_limit)
            while nxt < len(requests) and requests[nxt].arrival <= t:
                r = requests[nxt]
                if r.kind == "build":
                    pending_builds.append(r)
                    self.building.add(r.table)
                else:
                    self.pins[r.table] += 1
                    pending_lookups.append(r)
                nxt += 1
            # builds: one per free build stream
            for slot in self.build_slots:
                if slot.event is None and pending_builds:
                    r = pending_builds[0]
                    m = -(-r.capacity // self.bucket)
                    if not self._make_room(m * self.bucket * 8):
                        break
                    pending_builds.popleft()
                    params = bht.make_params(r.a, r.c, rng_seed=r.rng_seed)
                    nbytes = bht.bht_table_bytes(r.capacity, self.bucket, "bcht", params)
                    with torch.cuda.stream(slot.stream):
                        # table memory from the framework's caching allocator
                        buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
                        table = bht.Table(r.capacity, self.bucket, "bcht", r.a, r.c,
                                          rng_seed=r.rng_seed, buffer=buf)
                        self.tables[r.table] = table
                        self.bytes += table.info[3]
                        self._build(slot, table, r.keys, r.vals)
                        slot.done_event.record(slot.stream)
                    slot.event, slot.requests, slot.kind = slot.done_event, [r], "build"
                    r.launch = self.launches
                    self.launches += 1
            # lookups: every ready one, coalesced, on a free stream
            if pending_lookups:
                slot = next((s for s in self.lookup_slots if s.event is None), None)
                if slot is not None:
                    building = self.building
                    batch, keep = [], collections.deque()
                    while pending_lookups:
                        r = pending_lookups.popleft()
                        if r.table in self.ready and len(batch) < self.max_batch:
                            batch.append(r)
                        elif r.table in self.tables or r.table in building:
                            keep.append(r)          # its table is still being built
                        else:                       # evicted, failed or unknown table
                            r.status, r.done = bht.BHT_ERR_NOT_BUILT, now()
                            self.pins[r.table] -= 1
                            completed += 1
                    pending_lookups = keep
                    if batch:
                        reqs = []
                        for r in batch:
                            self.tables.move_to_end(r.table)
                            reqs.append((self.tables[r.table].handle, r.queries, r.out_v, r.out_f))
                            r.launch = self.launches
                        bht.bht_multi_find(slot.ctx, reqs, self.item_size, stream=slot.stream)
                        slot.done_event.record(slot.stream)
                        slot.event, slot.requests, slot.kind = slot.done_event, batch, "lookup"
                        self.launches += 1
            completed += self._poll(now)
        torch.cuda.synchronize()
        return requests


def serve_serial(torch, tables: dict, requests, bucket: int = 16, time_limit: float = 120.0):
    """Baseline: each request handled alone, in arrival order, with one
    plain call (bht_build, or bht_find) and a wait for it."""
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    for r in requests:
        t = time.perf_counter() - t0
        if t > time_limit:
            raise RuntimeError("serial run exceeded %.0f s" % time_limit)
        while time.perf_counter() - t0 < r.arrival:
            pass
        if r.kind == "build":
            table = bht.Table(r.capacity, bucket, "bcht", r.a, r.c, rng_seed=r.rng_seed)
            r.status = bht.bht_build(table.handle, r.keys, r.vals, stream=stream)
            tables[r.table] = table
        else:
            table = tables.get(r.table)
            if table is None:
                r.status = bht.BHT_ERR_NOT_BUILT
            else:
                bht.bht_find(table.handle, r.queries, r.out_v, r.out_f, stream=stream)
                stream.synchronize()
                r.status = bht.BHT_OK
        r.done = time.perf_counter() - t0
    return requests


def latency_stats(requests):
    """p50 / p99 / mean latency in milliseconds over completed requests."""
    import numpy as np
    lat = np.array([r.done - r.arrival for r in requests if r.status == bht.BHT_OK and r.done >= 0])
    if len(lat) == 0:
        return {}
    return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
            "mean_ms": round(float(lat.mean()) * 1e3, 4), "completed": int(len(lat))}


def make_requests(torch, specs, keys_of=None):
    """Request objects with device tensors from host request specifications
    (dictionaries with kind, arrival, table and either a `queries` uint32
    array or a `spec` of a new table).  keys_of(spec) returns the host keys
    and values of a build request's table."""
    import numpy as np
    dev = torch.device("cuda", torch.cuda.current_device())
    out = []
    for s in specs:
        if s["kind"] == "build":
            t = s["spec"]
            k, v = keys_of(t)
            out.append(Request("build", s["arrival"], s["table"],
                               keys=torch.from_numpy(np.ascontiguousarray(k).view(np.int32)).to(dev),
                               vals=torch.from_numpy(np.ascontiguousarray(v).view(np.int32)).to(dev),
                               capacity=t["capacity"], a=tuple(t["a"]), c=tuple(t["c"]),
                               rng_seed=t["rng_seed"]))
        else:
            q = np.ascontiguousarray(s["queries"]).view(np.int32)
            n = len(q)
            out.append(Request("lookup", s["arrival"], s["table"],
                               queries=torch.from_numpy(q).to(dev),
                               out_v=torch.empty(n, dtype=torch.int32, device=dev),
                               out_f=torch.empty(n, dtype=torch.uint8, device=dev)))
    return out


def build_resident_tables(torch, specs, keys_of, bucket: int = 16, reseed=None):
    """Tables for a list of table specifications (capacity, hash constants,
    generator seed), built together with one batched launch sequence.  A
    table whose build fails is rebuilt alone with the constants reseed(spec,
    attempt) returns.  Returns the tables in the order of `specs`."""
    import numpy as np
    dev = torch.device("cuda", torch.cuda.current_device())
    tables, entries, keep = [], [], []
    for s in specs:
        t = bht.Table(s["capacity"], bucket, "bcht", s["a"], s["c"], rng_seed=s["rng_seed"])
        k, v = keys_of(s)
        dk = torch.from_numpy(np.ascontiguousarray(k).view(np.int32)).to(dev)
        dv = torch.from_numpy(np.ascontiguousarray(v).view(np.int32)).to(dev)
        keep.append((dk, dv))
        tables.append(t)
        entries.append((t.handle, dk, dv, None, None, None))
    batch = bht.bht_batch_create(entries)
    bht.bht_batch_run(batch)
    _, sts = bht.bht_batch_wait(batch, len(specs))
    bht.bht_batch_destroy(batch)
    for i, st in enumerate(sts):
        attempt = 0
        while st != bht.BHT_OK:
            attempt += 1
            if reseed is None or attempt > 50:
                raise RuntimeError("table %d failed to build" % i)
            a, c = reseed(specs[i], attempt)
            bht.bht_reseed(tables[i].handle, bht.make_params(a, c))
            st = tables[i].build(*keep[i])
    del keep
    torch.cuda.synchronize()
    return tables
