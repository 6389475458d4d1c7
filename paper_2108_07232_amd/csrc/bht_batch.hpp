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
#include "bht_partition.hpp"

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

// ---------------------------------------------- partitioned batched build
//
// The partitioned build of bht_partition.hpp for all tables of a batch at
// once, with one radix pass per table: a table's pairs are grouped by the
// bin (8,192 slots) of their first bucket within that table, so pairs of
// different tables never mix and every table needs at most 1,024 bins.
// Bins of all tables are numbered globally (table t owns bins
// [bin_off_t, bin_off_t + nbins_t)); placement and overflow insertion run
// over the global bins.  Work items of the counting and scatter kernels are
// (table, chunk of at most 65,536 pairs); the partitioned pairs live in a
// workspace where table t's pairs start at key_off_t.

struct BatchPart {
  unsigned long long key_off;    // first workspace position of the table's pairs
  unsigned long long hist_off;   // first counter of the table's chunk histograms
  uint32_t bin_off;              // first global bin of the table
  uint32_t nbins;                // bins of the table (at most kMaxFan)
};

struct BatchChunk {
  uint32_t table;
  uint32_t local;                // chunk index within the table
  unsigned long long start;      // first pair of the chunk, within the table's input
  unsigned long long count;
};

struct BatchPartArgs {
  const BatchTable* tables;
  const BatchPart* parts;
  const BatchChunk* chunks;
  const uint32_t* bin_table;     // global bin -> table
  uint32_t n_chunks;
  uint32_t count;                // tables
  uint32_t nbins;                // global bins
  uint32_t bin_shift;            // bins of 2^bin_shift buckets
  uint32_t* hist;
  unsigned long long* total;     // per global bin
  unsigned long long* cursor;
  unsigned long long* bin_start;
  unsigned long long* bin_len;
  uint32_t* ovf_len;
  uint32_t* keys;                // workspace
  uint32_t* vals;
  unsigned int* head;            // overflow queue
  uint32_t* status;              // per table
};

__global__ void batch_part_clear_kernel(BatchPartArgs a) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t j = i; j < a.nbins; j += gridDim.x * blockDim.x) a.total[j] = 0;
  if (i == 0) *a.head = 0;
}

__global__ __launch_bounds__(kPassBlock) void batch_part_hist_kernel(BatchPartArgs a) {
  const BatchChunk c = a.chunks[blockIdx.x];
  const BatchTable& T = a.tables[c.table];
  const BatchPart P = a.parts[c.table];
  const Hash32 H = T.H;
  const uint32_t shift = a.bin_shift;
  const bool sentinel =
      hist_range(T.keys, c.start, c.start + c.count, P.nbins,
                 [&](uint32_t k) { return hash32(H, 0, k) >> shift; },
                 a.hist + P.hist_off + (uint64_t)c.local * P.nbins, a.total + P.bin_off);
  if (sentinel) atomicOr(a.status + c.table, kFlagSentinel);
}

// One block per table: the table's bin totals become workspace ranges.
__global__ __launch_bounds__(kPartBlock) void batch_part_scan_kernel(BatchPartArgs a) {
  __shared__ unsigned long long wt[kPartBlock / 64];
  __shared__ unsigned long long base[kMaxFan];
  const BatchPart P = a.parts[blockIdx.x];
  const unsigned long long* tot = a.total + P.bin_off;
  block_exclusive_scan<kPartBlock, unsigned long long>(tot, base, P.nbins, wt);
  for (uint32_t d = threadIdx.x; d < P.nbins; d += kPartBlock) {
    const uint64_t g = (uint64_t)P.bin_off + d;
    a.cursor[g] = P.key_off + base[d];
    a.bin_start[g] = P.key_off + base[d];
    a.bin_len[g] = tot[d];
  }
}

__global__ __launch_bounds__(kPassBlock, kScatterBlocksPerCU) void batch_part_scatter_kernel(BatchPartArgs a) {
  const BatchChunk c = a.chunks[blockIdx.x];
  const BatchTable& T = a.tables[c.table];
  const BatchPart P = a.parts[c.table];
  const Hash32 H = T.H;
  const uint32_t shift = a.bin_shift;
  scatter_range(T.keys, T.vals, c.start, c.start + c.count, P.nbins,
                [&](uint32_t k) { return hash32(H, 0, k) >> shift; },
                a.hist + P.hist_off + (uint64_t)c.local * P.nbins, a.cursor + P.bin_off, a.keys,
                a.vals);
}

// One block per global bin.
template <int B>
__global__ __launch_bounds__(kBinBlock) void batch_place_kernel(BatchPartArgs a) {
  const uint32_t g = blockIdx.x;
  const uint32_t t = a.bin_table[g];
  const BatchTable& T = a.tables[t];
  const uint32_t R = 1u << a.bin_shift;
  const uint64_t first = (uint64_t)(g - a.parts[t].bin_off) * R;
  const uint32_t nb = (uint64_t)T.H.m - first < (uint64_t)R ? (uint32_t)(T.H.m - first) : R;
  const uint32_t ovf = place_bin<B>(T.slots, a.keys, a.vals, T.H, R, first, nb, a.bin_start[g],
                                    a.bin_len[g], T.max_chain, T.rng_seed, g, (uint32_t)B,
                                    a.status + t);
  if (threadIdx.x == 0) a.ovf_len[g] = ovf;
}

// Pairs evicted during placement continue at their next bucket (cuckoo
// insertion, Section III-A); waves take global bins from a queue.
template <int B, int W>
__global__ __launch_bounds__(kBlock) void batch_overflow_kernel(BatchPartArgs a) {
  const uint32_t salt = lane_salt();
  for (;;) {
    const uint32_t g = part_queue_pop(a.head);
    if (g >= a.nbins) break;
    const uint32_t len = a.ovf_len[g];
    if (len == 0) continue;
    const uint32_t t = a.bin_table[g];
    const BatchTable& T = a.tables[t];
    BuildArgs32 b;
    b.slots = T.slots;
    b.keys = a.keys;
    b.vals = a.vals;
    b.n = 0;
    b.status = a.status + t;
    b.probe_total = nullptr;
    b.H = T.H;
    b.max_chain = T.max_chain;
    b.rng_seed = T.rng_seed;
    Range r;
    r.cursor = a.bin_start[g];
    r.end = r.cursor + len;
    uint32_t probes = 0;
    const uint32_t flags = cuckoo_build_range<B, W, false, true>(
        b, r, T.rng_seed ^ salt ^ (g * 0x85EBCA6Bu), &probes);
    if (flags) atomicOr(a.status + t, flags);
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
