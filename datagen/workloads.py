"""Seeded request streams and table sets for the batched and serving
workloads, as host data (numpy arrays and plain dictionaries).

Like the rest of this package it holds none of the hash-table arithmetic;
turning the specifications into device tensors and tables is the caller's
business (``paper_2108_07232_amd.serve.make_requests`` and
``build_resident_tables``).

- table sizes: log-uniform floor(2^(lo + (hi - lo) u));
- arrivals: a Poisson process (exponential gaps) at the offered rate;
- a request is a build of a new table with probability ``build_fraction``,
  else a lookup batch (size log-uniform) with a given positive fraction
  against a uniformly chosen table among the initial ones and those whose
  builds were requested earlier.
"""
from __future__ import annotations

import numpy as np

from . import (TAG_ARRIVALS, TAG_SIZES, capacity_for, hash_constants, log_uniform_sizes,
               mixed_queries, rng_seed, uniform01, unique_keys, values)


def table_seed(seed: int, tid: int) -> int:
    """Generator seed of table `tid` of a serving run."""
    return seed * 1000003 + 17 * tid + 5


def table_spec(seed: int, tid: int, n: int, load_factor: float = 0.9) -> dict:
    """Geometry, hash constants and generator seed of one table (no arrays)."""
    ts = table_seed(seed, tid)
    a, c = hash_constants(ts, 3)
    return dict(tid=tid, n=int(n), seed=ts, capacity=capacity_for(int(n), load_factor),
                a=tuple(int(x) for x in a), c=tuple(int(x) for x in c), rng_seed=rng_seed(ts))


def table_data(spec: dict):
    """The keys and values of a table spec (host arrays)."""
    return unique_keys(spec["n"], spec["seed"]), values(spec["n"], spec["seed"])


def initial_tables(count: int, seed: int, log2_range=(12, 24)) -> list:
    """The resident set: `count` table specs, sizes log-uniform in 2^log2_range."""
    sizes = log_uniform_sizes(count, log2_range[0], log2_range[1], seed).tolist()
    return [table_spec(seed, tid, n) for tid, n in enumerate(sizes)]


def request_stream(initial_sizes, count: int, rate: float, seed: int,
                   build_fraction: float = 0.05, lookup_log2=(8, 20), table_log2=(12, 24),
                   positive: float = 0.7, tables_seed: int | None = None) -> list:
    """`count` request specs in arrival order.  A build spec carries a table
    spec (its keys come from `table_data`); a lookup spec carries its query
    array (host uint32).  `seed` draws the stream; `tables_seed` (default:
    `seed`) is the seed the resident tables were made with, so that a
    lookup's positive keys are its table's keys."""
    if tables_seed is None:
        tables_seed = seed
    u = uniform01(3 * count, seed, TAG_ARRIVALS).reshape(count, 3)
    gaps = -np.log1p(-u[:, 0]) / rate
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes_b = log_uniform_sizes(count, table_log2[0], table_log2[1], seed, TAG_SIZES)
    sizes_l = log_uniform_sizes(count, lookup_log2[0], lookup_log2[1], seed, TAG_SIZES + 16)
    table_sizes = list(int(x) for x in initial_sizes)
    out = []
    for i in range(count):
        if u[i, 1] < build_fraction:
            tid = len(table_sizes)
            spec = table_spec(tables_seed, tid, int(sizes_b[i]))
            out.append(dict(kind="build", arrival=float(arrivals[i]), table=tid, spec=spec))
            table_sizes.append(spec["n"])
        else:
            tid = min(int(u[i, 2] * len(table_sizes)), len(table_sizes) - 1)
            q = mixed_queries(table_sizes[tid], int(sizes_l[i]), positive,
                              table_seed(tables_seed, tid),
                              shuffle_seed=seed * 7919 + i)
            out.append(dict(kind="lookup", arrival=float(arrivals[i]), table=tid, queries=q))
    return out


def table_sizes_after(initial_sizes, stream) -> list:
    """Key count of every table id the stream names (initial ones first)."""
    out = list(int(x) for x in initial_sizes)
    for r in stream:
        if r["kind"] == "build":
            out.append(r["spec"]["n"])
    return out
