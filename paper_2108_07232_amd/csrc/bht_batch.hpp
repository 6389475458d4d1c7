// Batched mode: many independent cuckoo tables of uneven sizes built and
// then queried by persistent kernels that pull (table, range) work items
// from device-side queues (one atomic counter per phase).  Each wave takes
// an item, runs the same per-lane insertion or query loop as the
// single-table kernels on that table's range, and takes the next item, so
// thousands of small tables cost a few launches instead of thousands, and
// large tables still spread over the whole device.
//
// Phases are separate kernels (reset -> build -> find): on gfx950 each XCD
// has its own L2, and the kernel boundary is what makes one table's
// inserts, performed by atomics, visible to plain bucket loads of queries
// running on any XCD.
#pragma once
#include "bht_kernels.hpp"

namespace bht {

struct BatchTable {
  uint64_t* slots;
  uint64_t words;
  const uint32_t* keys;
  const uint32_t* vals;
  uint64_t n_keys;
  const uint32_t* queries;
  uint32_t* out_v;
  uint8_t* out_f;
  uint64_t n_queries;
  Hash32 H;
  uint32_t max_chain;
  uint32_t rng_seed;
};

struct BatchItem {
  uint32_t table;
  uint32_t pad;
  uint64_t start;
  uint64_t count;
};

// Clears the queue heads and every table's status word (no memset nodes, so
// the sequence can be captured in a graph and replayed).
__global__ void batch_reset_kernel(unsigned int* __restrict__ heads,
                                   uint32_t* __restrict__ status, uint32_t n_tables) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 4) heads[i] = 0;
  for (uint32_t t = i; t < n_tables; t += gridDim.x * blockDim.x) status[t] = 0;
}

// Section III: every bucket of every table starts empty.  Item = a range of
// 64-bit words of one table's slot array.
__global__ __launch_bounds__(kBlock) void batch_fill_kernel(const BatchTable* __restrict__ tables,
                                                           const BatchItem* __restrict__ items,
                                                           uint64_t n_items) {
  for (uint64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const BatchItem item = items[it];
    uint64_t* const p = tables[item.table].slots;
    for (uint64_t w = item.start + threadIdx.x; w < item.start + item.count; w += blockDim.x)
      p[w] = kEmptyPair;
  }
}

__device__ __forceinline__ uint64_t next_item(unsigned int* head) {
  unsigned int v = 0;
  if (__lane_id() == 0) v = atomicAdd(head, 1u);
  return (uint64_t)__builtin_amdgcn_readfirstlane(v);
}

template <int B, int W>
__global__ __launch_bounds__(kBlock) void batch_build_kernel(const BatchTable* __restrict__ tables,
                                                            const BatchItem* __restrict__ items,
                                                            uint64_t n_items,
                                                            unsigned int* __restrict__ head,
                                                            uint32_t* __restrict__ status) {
  const uint32_t salt = lane_salt();
  for (;;) {
    const uint64_t it = next_item(head);
    if (it >= n_items) break;
    const BatchItem item = items[it];
    const BatchTable& T = tables[item.table];
    BuildArgs32 g;
    g.slots = T.slots;
    g.keys = T.keys;
    g.vals = T.vals;
    g.n = T.n_keys;
    g.status = status + item.table;
    g.probe_total = nullptr;
    g.H = T.H;
    g.max_chain = T.max_chain;
    g.rng_seed = T.rng_seed;
    Range r;
    r.cursor = item.start;
    r.end = item.start + item.count;
    uint32_t probes = 0;
    const uint32_t flags =
        cuckoo_build_range<B, W, false>(g, r, g.rng_seed ^ salt ^ (uint32_t)(it * 0x85EBCA6Bu),
                                        &probes);
    if (flags) atomicOr(g.status, flags);
  }
}

template <int B, int W, int Q = 1>
__global__ __launch_bounds__(kBlock) void batch_find_kernel(const BatchTable* __restrict__ tables,
                                                           const BatchItem* __restrict__ items,
                                                           uint64_t n_items,
                                                           unsigned int* __restrict__ head) {
  for (;;) {
    const uint64_t it = next_item(head);
    if (it >= n_items) break;
    const BatchItem item = items[it];
    const BatchTable& T = tables[item.table];
    FindArgs32 g;
    g.slots = T.slots;
    g.queries = T.queries;
    g.n = T.n_queries;
    g.out_v = T.out_v;
    g.out_f = T.out_f;
    g.probes = nullptr;
    g.H = T.H;
    Range r;
    r.cursor = item.start;
    r.end = item.start + item.count;
    cuckoo_find_chunk_range<B, W, false, Q>(g, r);
  }
}

// Small coalesced query launches pass their request descriptors as kernel
// arguments (no staging copy, no queue reset): a launch is then as cheap as
// a single-table query.  Work items are implicit: request r owns items
// [first_item[r], first_item[r+1]), each item_size queries long, and waves
// take items round-robin.
struct FindTable {
  const uint64_t* slots;
  const uint32_t* queries;
  uint32_t* out_v;
  uint8_t* out_f;
  uint64_t n;
  Hash32 H;
};

constexpr int kInlineRequests = 24;

struct InlineFind {
  FindTable t[kInlineRequests];
  uint32_t first_item[kInlineRequests + 1];
  uint32_t count;
  uint32_t item_size;
};

template <int B, int W>
__global__ __launch_bounds__(kBlock) void inline_find_kernel(InlineFind a) {
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint32_t total = a.first_item[a.count];
  for (uint64_t it = wave; it < total; it += nwaves) {
    uint32_t r = 0;
    while (r + 1 < a.count && a.first_item[r + 1] <= it) ++r;
    const FindTable& T = a.t[r];
    FindArgs32 g;
    g.slots = T.slots;
    g.queries = T.queries;
    g.n = T.n;
    g.out_v = T.out_v;
    g.out_f = T.out_f;
    g.probes = nullptr;
    g.H = T.H;
    Range rg;
    rg.cursor = (uint64_t)(it - a.first_item[r]) * a.item_size;
    rg.end = rg.cursor + a.item_size < T.n ? rg.cursor + a.item_size : T.n;
    cuckoo_find_chunk_range<B, W, false>(g, rg);
  }
}

}  // namespace bht
