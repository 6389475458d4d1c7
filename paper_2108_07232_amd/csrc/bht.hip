// C ABI of libbht: table objects, argument checking, launch geometry and
// dispatch to the gfx950 kernels.  Declared in include/bht.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

#include "bht.h"
#include "bht_diag.hpp"
#include "bht_kernels.hpp"
#include "bht_schemes.hpp"
#include "bht_wide.hpp"
#include "bht_batch.hpp"
#include "bht_partition.hpp"
#include "bht_wide_partition.hpp"
#include "bht_iceberg_partition.hpp"

using namespace bht;

struct bht_table {
  bht_scheme scheme;
  uint32_t b;           // slots per (primary) bucket
  uint64_t m;           // (primary) buckets
  uint32_t key_bits;
  bht_params params;
  uint32_t tile;        // lanes per tile reading one bucket
  uint32_t find_schedule;
  uint32_t grid_blocks; // 0 = resident capacity
  uint64_t* d_slots;
  uint64_t words;       // uint64 words in the slot array
  uint64_t slots;       // pair capacity (both levels)
  uint32_t* d_status;   // [0] flags; lives after the slot array
  uint32_t h_status[8]; // host copy
  bool owns_memory;     // slot array allocated by the library
  uint64_t n_stored;
  uint64_t pending_n;
  bool built;
  bool pending;
  int device;
  bool timing;             // record events around the main kernels
  hipEvent_t ev[4];        // build start/stop, find start/stop
  bool build_timed, find_timed;
  uint32_t build_mode;     // bht_build_mode
  uint32_t iht_early_exit; // iceberg finds stop after a primary below the threshold
  uint32_t unroll;         // chunk-schedule queries per lane per chunk (1 or 2)
  void* d_part;            // partitioned build workspace (library-owned)
  uint64_t part_bytes;
  bool pending_partitioned;
  bool last_partitioned;   // the last successful build took the partitioned path
  uint64_t last_evicted;   // ... and evicted this many pairs on chip
  uint64_t last_probes;    // ... and read this many buckets inserting them
  uint64_t last_pad1;      // ... and its radix passes wrote this much padding
  uint64_t last_pad2;
  uint64_t counted_build_probes;  // bucket reads of the last build, if it was counted
  uint64_t find_probe_base;       // find-probe counter value at the last stats read
};

struct bht_batch {
  uint32_t count;
  std::vector<bht_table*> tables;
  std::vector<uint64_t> n_keys;
  uint32_t b, tile;
  bht::BatchTable* d_tables;
  bht::BatchItem* d_items;      // fill items, then build items, then find items
  uint64_t n_fill, n_build, n_find;
  unsigned int* d_heads;
  uint32_t* d_status;
  uint32_t* h_status;
  const void* build_kernel;
  const void* find_kernel;
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipStream_t graph_stream;
  // partitioned build of all tables (when every table fits one radix pass)
  bool partitioned;
  void* d_ws;                   // workspace: pairs, counters, descriptors
  bht::BatchPartArgs pa;
  const void* place_kernel;
  const void* overflow_kernel;
};

struct bht_find_ctx {
  uint32_t max_requests;
  uint64_t max_items;
  bht::BatchTable* d_tables;
  bht::BatchItem* d_items;
  unsigned int* d_heads;
  bht::BatchTable* h_tables;    // pinned staging
  bht::BatchItem* h_items;
  hipEvent_t staged;             // the last call's copies are done with the staging
  bool used;
};

namespace {

thread_local std::string g_last_error;

bht_status fail(bht_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

bht_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return BHT_ERR_HIP;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return hip_fail(_e, #expr);   \
  } while (0)

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Pairs per lane (at least) of the builds whose placements compare bucket
// loads, which bounds the placements in flight.
#ifndef BHT_LB_PAIRS_PER_LANE
#define BHT_LB_PAIRS_PER_LANE 32
#endif
constexpr uint64_t kLbPairsPerLane = BHT_LB_PAIRS_PER_LANE;

// Secondary buckets per lane of the partitioned iceberg build's overflow
// phase (bounds its secondary choices in flight; 1 = the whole device).
#ifndef BHT_ICEBERG_OVF_SPREAD
#define BHT_ICEBERG_OVF_SPREAD 1
#endif
constexpr uint64_t kIcebergOverflowSpread = BHT_ICEBERG_OVF_SPREAD;

// Blocks of `block` threads of `kernel` the current device keeps resident.
int resident_blocks(const void* kernel, int block) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> known;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  auto it = known.find({kernel, dev});
  if (it != known.end()) return it->second;
  int cus = 0, per_cu = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0);
  const int cap = std::max(1, cus) * std::max(1, per_cu);
  known.emplace(std::make_pair(kernel, dev), cap);
  return cap;
}

// Blocks to launch: enough to give every lane an item, capped at what the
// device keeps resident at once (the kernels loop over their share).
// items_per_lane > 0 asks for at least ceil(items / (256 * items_per_lane))
// blocks even beyond the resident count: short per-wave ranges let the
// dispatcher balance waves that finish at different times.
int grid_for(const void* kernel, uint64_t items, uint32_t fixed = 0, uint64_t items_per_lane = 0) {
  if (fixed) return (int)fixed;
  static std::mutex mu;
  static std::unordered_map<const void*, int> resident;
  int cap;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = resident.find(kernel);
    if (it == resident.end()) {
      int dev = 0, cus = 0, per_cu = 0;
      (void)hipGetDevice(&dev);
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0);
      cap = std::max(1, cus) * std::max(1, per_cu);
      resident.emplace(kernel, cap);
    } else {
      cap = it->second;
    }
  }
  uint64_t want = (items + kBlock - 1) / kBlock;
  uint64_t grid = std::min<uint64_t>(want, (uint64_t)cap);
  if (items_per_lane)
    grid = std::max<uint64_t>(grid, std::min<uint64_t>(
        (items + kBlock * items_per_lane - 1) / (kBlock * items_per_lane), 1u << 20));
  return (int)std::max<uint64_t>(1, grid);
}

Hash64 make_hash64(const bht_params& p, uint64_t m, uint32_t h) {
  Hash64 H;
  for (int i = 0; i < 4; ++i) {
    H.a[i] = p.a[i];
    H.c[i] = p.b[i];
  }
  H.m = m;
  H.M = UINT64_MAX / m;
  H.h = h;
  return H;
}

Hash32 make_hash32(const bht_params& p, uint64_t m, uint32_t h) {
  Hash32 H;
  for (int i = 0; i < 4; ++i) {
    H.a[i] = (uint32_t)p.a[i];
    H.c[i] = (uint32_t)p.b[i];
  }
  H.m = (uint32_t)m;
  H.M = fastmod32_constant((uint32_t)m);
  H.h = h;
  return H;
}

// splitmix64 (Steele, Lea, Flood; "Fast splittable pseudorandom number
// generators", 2014): the stream from which seeded hash constants are drawn.
uint64_t splitmix64_next(uint64_t* state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Section VII draws the hash constants at random: a_i uniform in [1, p-1] and
// b_i uniform in [0, p-1], by rejection from the seed's stream (32-bit draws
// for p = 2^32 - 5, 61-bit draws for p = 2^61 - 1); the eviction generator
// seed is the next nonzero 32-bit draw.  All four hash slots are filled.
void draw_constants(uint64_t seed, uint32_t key_bits, uint64_t a[4], uint64_t b[4],
                    uint32_t* rng_seed) {
  uint64_t st = seed ^ 0x5EEDC0457A27ull;
  const uint64_t prime = key_bits == 64 ? kP61 : kP32;
  const int shift = key_bits == 64 ? 3 : 32;
  for (int i = 0; i < 4; ++i) {
    uint64_t x;
    do x = splitmix64_next(&st) >> shift; while (x == 0 || x >= prime);
    a[i] = x;
    do x = splitmix64_next(&st) >> shift; while (x >= prime);
    b[i] = x;
  }
  uint32_t r;
  do r = (uint32_t)(splitmix64_next(&st) >> 32); while (r == 0);
  *rng_seed = r;
}

bool valid_params(const bht_params& p, bht_scheme scheme, uint32_t b, std::string* why) {
  if (p.key_bits != 32 && p.key_bits != 64) return *why = "key_bits must be 32 or 64", false;
  const uint64_t prime = p.key_bits == 32 ? kP32 : kP61;
  if (p.num_hashes < 1 || p.num_hashes > 4) return *why = "num_hashes must be 1..4", false;
  for (uint32_t i = 0; i < p.num_hashes; ++i) {
    if (p.a[i] < 1 || p.a[i] >= prime || p.b[i] >= prime)
      return *why = "hash constants must satisfy 1 <= a < p and 0 <= b < p", false;
  }
  switch (scheme) {
    case BHT_BCHT:
      if (p.key_bits == 64 ? b != 8 : (b != 4 && b != 8 && b != 16 && b != 32))
        return *why = "BCHT bucket size must be 4, 8, 16 or 32 (8 for 64-bit keys)", false;
      break;
    case BHT_CHT1:
      if (b != 1 || p.key_bits != 32) return *why = "CHT1 needs bucket_size 1, 32-bit keys", false;
      break;
    case BHT_BP2HT:
      if (p.key_bits != 32 || p.num_hashes != 2 || (b != 8 && b != 16 && b != 32))
        return *why = "BP2HT needs 32-bit keys, 2 hashes and bucket size 8, 16 or 32", false;
      break;
    case BHT_BCHT_LB:
      if (p.key_bits != 32 || p.num_hashes < 2 || (b != 8 && b != 16 && b != 32))
        return *why = "BCHT_LB needs 32-bit keys, 2..4 hashes and bucket size 8, 16 or 32", false;
      break;
    case BHT_IHT:
      if (p.key_bits != 32 || p.num_hashes != 3 || (b != 16 && b != 32))
        return *why = "IHT needs 32-bit keys, 3 hashes and bucket size 16 or 32", false;
      if (p.iht_secondary_b != 0 && p.iht_secondary_b != 8)
        return *why = "IHT secondary buckets hold 8 slots (or 0 for one level)", false;
      if (p.iht_secondary_b && (p.iht_secondary_m == 0 || p.iht_secondary_m > 0xFFFFFFFFull))
        return *why = "IHT secondary bucket count must be 1 .. 2^32 - 1", false;
      if (p.iht_threshold > b) return *why = "IHT threshold exceeds the bucket size", false;
      break;
    default:
      return *why = "unknown scheme", false;
  }
  return true;
}

// Lanes per bucket read.  Every lane owns one operation whatever the width;
// the width only splits each bucket read among a tile's lanes.  A cuckoo
// table of 16-slot buckets takes 4 lanes of 32 bytes (two 16-byte loads per
// bucket per lane): its query and overflow kernels need 70 registers per
// lane instead of 82 and keep 7 waves per SIMD instead of 5, measured 0.3%
// faster in the queries and 2.5% in the overflow insertion (2 lanes: queries
// 1.5% slower; 1 lane: 9% slower).  The other schemes keep one 16-byte load
// per lane.
// Queries per lane per chunk of the chunk schedule.  Cuckoo tables of
// 16-slot buckets (4-lane tiles) take 2: measured 0.7% faster queries.
uint32_t default_unroll(bht_scheme scheme, uint32_t b) {
  return (scheme == BHT_BCHT || scheme == BHT_CHT1) && b == 16 ? 2 : 1;
}

uint32_t default_tile(bht_scheme scheme, uint32_t b) {
  switch (b) {
    case 1: return 1;
    case 4: return 4;
    case 8: return 8;
    case 16: return (scheme == BHT_BCHT || scheme == BHT_CHT1) ? 4 : 8;
    default: return 16;
  }
}

// --------------------------------------------------------------- dispatch

enum class Kind { Cuckoo, P2, Iceberg, LoadBalanced };

// The kernels of one table configuration (bucket size, secondary bucket
// size, tile width, probe counting, query schedule).
struct KernelSet {
  Kind kind;
  const void* build;
  const void* find;
  bool chunk;  // the query kernel uses the chunk schedule
};

constexpr uint32_t kDefaultSchedule = BHT_FIND_CHUNK;

template <int B, int W, bool C>
KernelSet cuckoo_set(uint32_t schedule, uint32_t unroll) {
  const bool chunk = schedule == BHT_FIND_CHUNK || schedule == BHT_FIND_PARALLEL;
  const void* chunk_kernel = unroll == 2 ? (const void*)cuckoo_find_chunk_kernel<B, W, C, 2>
                                         : (const void*)cuckoo_find_chunk_kernel<B, W, C, 1>;
  return {Kind::Cuckoo, (const void*)cuckoo_build_kernel<B, W, C>,
          schedule == BHT_FIND_PARALLEL ? (const void*)cuckoo_find_parallel_kernel<B, W, C>
          : chunk                       ? chunk_kernel
                                        : (const void*)cuckoo_find_kernel<B, W, C>,
          chunk};
}

template <int B, int W, bool C>
KernelSet p2_set() {
  return {Kind::P2, (const void*)p2_build_kernel<B, W, C>,
          (const void*)stable_find_chunk_kernel<B, 0, W, C>, true};
}

template <int B, int W, bool C>
KernelSet lb_set() {
  return {Kind::LoadBalanced, (const void*)lb_build_kernel<B, W, C>,
          (const void*)stable_find_chunk_kernel<B, 0, W, C>, true};
}

template <int B, int B2, int W, bool C>
KernelSet iceberg_set() {
  return {Kind::Iceberg, (const void*)iceberg_build_kernel<B, B2, W, C>,
          (const void*)stable_find_chunk_kernel<B, B2, W, C>, true};
}

template <bool C>
bool pick_t(bht_scheme scheme, uint32_t b, uint32_t b2, uint32_t w, uint32_t schedule,
            uint32_t unroll, KernelSet* ks) {
  if (scheme == BHT_BCHT || scheme == BHT_CHT1) {
#define BHT_CASE(B_, W_) \
  if (b == B_ && w == W_) return *ks = cuckoo_set<B_, W_, C>(schedule, unroll), true;
    BHT_CASE(1, 1)
    BHT_CASE(4, 4)
    BHT_CASE(8, 4)
    BHT_CASE(8, 8)
    BHT_CASE(16, 4)
    BHT_CASE(16, 8)
    BHT_CASE(16, 16)
    BHT_CASE(32, 8)
    BHT_CASE(32, 16)
#undef BHT_CASE
  } else if (schedule == BHT_FIND_PARALLEL) {
    return false;                    // parallel probing: cuckoo tables only
  } else if (scheme == BHT_BCHT_LB) {
    if (b == 8 && w == 8) return *ks = lb_set<8, 8, C>(), true;
    if (b == 16 && w == 8) return *ks = lb_set<16, 8, C>(), true;
    if (b == 32 && w == 16) return *ks = lb_set<32, 16, C>(), true;
  } else if (scheme == BHT_BP2HT) {
    if (b == 8 && w == 8) return *ks = p2_set<8, 8, C>(), true;
    if (b == 16 && w == 8) return *ks = p2_set<16, 8, C>(), true;
    if (b == 32 && w == 16) return *ks = p2_set<32, 16, C>(), true;
  } else if (scheme == BHT_IHT) {
    if (b == 16 && b2 == 0 && w == 8) return *ks = iceberg_set<16, 0, 8, C>(), true;
    if (b == 16 && b2 == 8 && w == 8) return *ks = iceberg_set<16, 8, 8, C>(), true;
    if (b == 32 && b2 == 0 && w == 16) return *ks = iceberg_set<32, 0, 16, C>(), true;
    if (b == 32 && b2 == 8 && w == 16) return *ks = iceberg_set<32, 8, 16, C>(), true;
  }
  return false;
}

bool pick(const bht_table* t, uint32_t w, uint32_t schedule, bool count, KernelSet* ks) {
  if (schedule == BHT_FIND_DEFAULT) schedule = kDefaultSchedule;
  const uint32_t b2 = t->scheme == BHT_IHT ? t->params.iht_secondary_b : 0;
  return count ? pick_t<true>(t->scheme, t->b, b2, w, schedule, t->unroll, ks)
               : pick_t<false>(t->scheme, t->b, b2, w, schedule, t->unroll, ks);
}

// Running total of the bucket reads of instrumented finds: a 64-bit word in
// the status area after the slot array (words 16-17; the build uses 0-3).
unsigned long long* find_probe_counter(const bht_table* t) {
  return reinterpret_cast<unsigned long long*>(t->d_status + 16);
}

bht_status add_find_probes(const uint8_t* probes, uint64_t n, const bht_table* t, hipStream_t st) {
  const int grid = (int)std::min<uint64_t>((n + kBlock - 1) / kBlock, 1024);
  probe_sum_kernel<<<grid, kBlock, 0, st>>>(probes, n, find_probe_counter(t));
  HIP_TRY(hipGetLastError());
  return BHT_OK;
}

bht_status launch_fill(bht_table* t, hipStream_t st) {
  const uint64_t pairs = t->words / 2 + 1;
  const int grid = (int)std::min<uint64_t>((pairs + kBlock - 1) / kBlock, 8192);
  fill_empty_kernel<<<grid, kBlock, 0, st>>>(t->d_slots, t->words, t->d_status);
  HIP_TRY(hipGetLastError());
  return BHT_OK;
}

uint64_t* secondary_slots(const bht_table* t) {
  if (t->scheme != BHT_IHT || t->params.iht_secondary_b == 0) return nullptr;
  return t->d_slots + t->m * t->b;
}

Hash32 secondary_hash(const bht_table* t) {
  const uint64_t m2 = t->params.iht_secondary_b ? t->params.iht_secondary_m : t->m;
  return make_hash32(t->params, m2, t->params.num_hashes);
}

// ------------------------------------------------- partitioned build

// Smallest build that takes the partitioned path by default: below it the
// fixed cost of its eight launches outweighs the saved atomics.
constexpr uint64_t kPartMinKeys = 1ull << 18;
// The same for two-level iceberg tables (at LF 0.85 the partitioned build
// is 1.7-2.2x the concurrent one from 2^18 to 2^26 pairs, every build of
// 12 succeeding on both).  One-level iceberg tables take the partitioned
// path only when asked: near their load limit (t = 13, LF 0.85) it
// succeeded for 10, 8 and 3 of 12 constant sets at 2^20, 2^22 and 2^24
// pairs, where the concurrent build succeeded for all.
#ifndef BHT_ICEBERG_PART_MIN_LOG2
#define BHT_ICEBERG_PART_MIN_LOG2 18
#endif
constexpr uint64_t kIcebergPartMinKeys = 1ull << BHT_ICEBERG_PART_MIN_LOG2;

struct PartKernels {
  const void* place;
  const void* overflow;
  bool iceberg;          // placement without eviction, iceberg overflow insertion
};

// Placement and overflow kernels of a partitioned build of table t (tile
// width w); false when the table's scheme or geometry has none.
bool part_kernels(const bht_table* t, uint32_t w, PartKernels* k) {
  const uint32_t b = t->b;
  if (t->scheme == BHT_IHT) {
    const uint32_t b2 = t->params.iht_secondary_b;
#define BHT_ICASE(B_, B2_, W_)                                                     \
  if (b == B_ && b2 == B2_ && w == W_) {                                           \
    *k = {(const void*)bin_place_kernel<B_, false>,                                \
          (const void*)iceberg_overflow_kernel<B_, B2_, W_>, true};                \
    return true;                                                                   \
  }
    BHT_ICASE(16, 0, 8)
    BHT_ICASE(16, 8, 8)
    BHT_ICASE(32, 0, 16)
    BHT_ICASE(32, 8, 16)
#undef BHT_ICASE
    return false;
  }
  if (t->scheme != BHT_BCHT && t->scheme != BHT_CHT1) return false;
#define BHT_PCASE(B_, W_)                                                          \
  if (b == B_ && w == W_) {                                                        \
    *k = {(const void*)bin_place_kernel<B_>, (const void*)overflow_build_kernel<B_, W_>, false}; \
    return true;                                                                   \
  }
  BHT_PCASE(1, 1)
  BHT_PCASE(4, 4)
  BHT_PCASE(8, 4)
  BHT_PCASE(8, 8)
  BHT_PCASE(16, 4)
  BHT_PCASE(16, 8)
  BHT_PCASE(16, 16)
  BHT_PCASE(32, 8)
  BHT_PCASE(32, 16)
#undef BHT_PCASE
  return false;
}

// Padding pairs a line-writing pass over `chunks` chunks of `fan` digits
// adds to n pairs, at most: under a line (lw pairs) per non-empty (chunk,
// digit) range.
uint64_t line_pad_bound(uint64_t chunks, uint64_t fan, uint64_t n, uint64_t lw = kLineWords) {
  return std::min<uint64_t>(chunks * fan, n) * (lw - 1);
}

uint64_t round_to_line(uint64_t words) { return (words + kLineWords - 1) / kLineWords * kLineWords; }

uint32_t log2_exact(uint64_t x) {
  uint32_t r = 0;
  while ((1ull << r) < x) ++r;
  return r;
}

// Second-pass chunks the workspace provides for: the count of pieces of at
// most one chunk per first-pass range (`ceil_chunks`, a bound), plus a
// quarter more (at most 512) for the round-balanced cuts part_scan1_kernel
// may choose; each chunk adds up to kLinePadPerChunk2 words of padding room.
uint64_t second_pass_chunk_cap(uint64_t ceil_chunks) {
  return ceil_chunks + std::min<uint64_t>(ceil_chunks / 4, 512);
}

// Bins, passes, digit counts and chunk size for n pairs; false if the table
// has more bins than two passes can address.  Bins are as large as LDS
// allows, halved (down to 32 buckets) while a single pass still covers them,
// so small tables get enough bins to fill the device; chunks shrink for the
// same reason.
bool part_plan(const bht_table* t, uint64_t n, PartPlan* P) {
  const uint64_t S = t->key_bits == 64 ? kBin64Slots : t->b == 1 ? bin_slots<1>() : bin_slots<16>();
  uint64_t R = S / t->b;
  while (R > 32 && (t->m + R / 2 - 1) / (R / 2) <= kMaxFan) R /= 2;
  const uint64_t nbins = (t->m + R - 1) / R;
  const uint64_t per = (n + (uint64_t)kPartSub * 512 - 1) / ((uint64_t)kPartSub * 512);
  *P = PartPlan{};
  P->chunk = kPartSub * (uint32_t)std::min<uint64_t>(std::max<uint64_t>(per, 1), kPartChunkMax / kPartSub);
  if (t->key_bits == 64) P->H64 = make_hash64(t->params, t->m, t->params.num_hashes);
  else P->H = make_hash32(t->params, t->m, t->params.num_hashes);
  P->bin_shift = log2_exact(R);
  P->nbins = (uint32_t)nbins;
  if (nbins <= kMaxFan) {
    P->levels = 1;
    P->fan1 = (uint32_t)nbins;
  } else {
    P->levels = 2;
    const uint64_t fan1 = (nbins + kFan2 - 1) / kFan2;
    if (fan1 > kMaxFan) return false;
    P->fan1 = (uint32_t)fan1;
  }
  // Passes of at most 256 digits write whole lines, while the padding they
  // add is expected to stay under 8% of the pairs (half a line per (chunk,
  // digit) range; small tables have small chunks), the
  // positions, padding included, stay below 2^32, and (two passes) the
  // padded first-pass output still fits the slot array it is written to.
  // At 2^24 pairs a padded second pass (12% padding) is no faster than the
  // plain scatter; at 2^25 (6%) it is 8% faster.
  if (kScatterLines) {
    const uint64_t lw = t->key_bits == 64 ? line_words<uint64_t>() : line_words<uint32_t>();
    auto light = [n, lw](uint64_t chunks, uint64_t fan) {
      return line_pad_bound(chunks, fan, n, lw) <= n * 16 / 100;
    };
    const uint64_t chunks1 = (n + P->chunk - 1) / P->chunk;
    const uint64_t in2 = n + line_pad_bound(chunks1, P->fan1, n, lw);
    if (P->levels == 1) {
      P->lines1 = P->fan1 <= kLineMaxFan && light(chunks1, P->fan1) && in2 < (1ull << 32);
    } else {
      const uint64_t mid = round_to_line(in2);
      P->lines1 = P->fan1 <= kLineMaxFan && light(chunks1, P->fan1) && mid <= t->slots &&
                  mid < (1ull << 32);
      const uint64_t in = P->lines1 ? in2 : n;
      const uint64_t chunks2 = in / P->chunk + P->fan1;
      P->chunks2_cap = (uint32_t)second_pass_chunk_cap(chunks2);
      P->lines2 = light(chunks2, kFan2) &&
                  in + P->chunks2_cap * kLinePadPerChunk2 + kLineWords * (P->fan1 + 1) <
                      (1ull << 32);
    }
  }
  if (P->levels == 2 && !P->chunks2_cap)
    P->chunks2_cap = (uint32_t)second_pass_chunk_cap(n / P->chunk + P->fan1);
  return true;
}

// Workspace carve-up (256-byte aligned pieces) for n pairs under plan P.
// mid_words: words of each first-pass output array (of two passes; keys,
// then values, in the slot array); keys/vals hold out_words words each.
struct PartLayout {
  uint64_t hist1, hist2, total1, cursor1, seg_start, seg_len, chunk_first, chunk_seg, total2, cursor2,
      bin_start, bin_len, ovf_len, head, keys, vals, bytes;
  uint64_t chunks1, chunks2, mid_words, out_words;
};

PartLayout part_layout(const PartPlan& P, uint64_t n, uint32_t word_bytes = 4) {
  PartLayout L{};
  uint64_t off = 0;
  auto take = [&off](uint64_t bytes) {
    const uint64_t at = off;
    off += (bytes + 255) / 256 * 256;
    return at;
  };
  L.chunks1 = (n + P.chunk - 1) / P.chunk;
  // first-pass output words, padding included
  const uint64_t in2 =
      n + (P.lines1 ? line_pad_bound(L.chunks1, P.fan1, n, 128 / word_bytes) : 0);
  L.chunks2 = P.levels == 2 ? P.chunks2_cap : 0;
  L.mid_words = P.levels == 2 ? (P.lines1 ? round_to_line(in2) : n) : 0;
  L.out_words = in2 + (P.lines2 ? L.chunks2 * kLinePadPerChunk2 + kLineWords * (P.fan1 + 1) : 0);
  L.hist1 = take(L.chunks1 * P.fan1 * 4);
  L.hist2 = take(L.chunks2 * kFan2 * 4);
  L.total1 = take(P.fan1 * 8ull);
  L.cursor1 = take(P.fan1 * 8ull);
  L.seg_start = take(P.fan1 * 8ull);
  L.seg_len = take(P.fan1 * 8ull);
  L.chunk_first = take((P.fan1 + 1) * 4ull);
  L.chunk_seg = take(L.chunks2 * 4ull);
  L.total2 = take(P.levels == 2 ? P.fan1 * (uint64_t)kFan2 * 8 : 0);
  L.cursor2 = take(P.levels == 2 ? P.fan1 * (uint64_t)kFan2 * 8 : 0);
  L.bin_start = take(P.nbins * 8ull);
  L.bin_len = take(P.nbins * 8ull);
  L.ovf_len = take(P.nbins * 4ull);
  L.head = take(4);
  L.keys = take(L.out_words * word_bytes);
  L.vals = take(L.out_words * word_bytes);
  L.bytes = off;
  return L;
}

// Schemes with a partitioned build: the cuckoo tables, and iceberg tables
// whose primaries take at least one pair.
bool partition_scheme(const bht_table* t) {
  if (t->scheme == BHT_BCHT || t->scheme == BHT_CHT1) return true;
  return t->scheme == BHT_IHT && t->key_bits == 32 && t->params.iht_threshold > 0;
}

bool use_partitioned(const bht_table* t, uint64_t n, bool counting) {
  if (counting || n == 0 || n >= (1ull << 32)) return false;
  if (!partition_scheme(t)) return false;
  if (t->key_bits == 64 && t->b != 8) return false;
  if (t->build_mode == BHT_BUILD_CONCURRENT) return false;
  PartPlan P;
  if (!part_plan(t, n, &P)) return false;
  if (t->build_mode == BHT_BUILD_PARTITIONED) return true;
  if (!t->owns_memory) return false;
  if (t->scheme == BHT_IHT)
    return t->params.iht_secondary_b != 0 && n >= kIcebergPartMinKeys;
  return n >= kPartMinKeys;
}

// *w <- the workspace for layout L: the caller's ws (of ws_bytes), or, when
// ws is null, the table's own, allocated on first use and grown as needed.
bht_status part_workspace(bht_table* t, const PartLayout& L, hipStream_t st, void* ws,
                          uint64_t ws_bytes, char** w) {
  if (ws && (ws_bytes < L.bytes || (reinterpret_cast<uintptr_t>(ws) & 255)))
    return fail(BHT_ERR_INVALID_ARG, "workspace too small or not 256-byte aligned");
  if (!ws && t->part_bytes < L.bytes) {
    // grow the workspace; the stream's earlier work may still use the old one
    if (t->d_part) {
      HIP_TRY(hipStreamSynchronize(st));
      HIP_TRY(hipFree(t->d_part));
      t->d_part = nullptr;
      t->part_bytes = 0;
    }
    hipError_t e = hipMalloc(&t->d_part, L.bytes);
    if (e != hipSuccess) {
      t->d_part = nullptr;
      return fail(BHT_ERR_OOM, std::string("build workspace: ") + hipGetErrorString(e));
    }
    t->part_bytes = L.bytes;
  }
  *w = static_cast<char*>(ws ? ws : t->d_part);
  return BHT_OK;
}

PartMeta part_meta(const PartLayout& L, char* w) {
  PartMeta M;
  M.hist1 = reinterpret_cast<uint32_t*>(w + L.hist1);
  M.hist2 = reinterpret_cast<uint32_t*>(w + L.hist2);
  M.total1 = reinterpret_cast<unsigned long long*>(w + L.total1);
  M.cursor1 = reinterpret_cast<unsigned long long*>(w + L.cursor1);
  M.seg_start = reinterpret_cast<unsigned long long*>(w + L.seg_start);
  M.seg_len = reinterpret_cast<unsigned long long*>(w + L.seg_len);
  M.chunk_first = reinterpret_cast<uint32_t*>(w + L.chunk_first);
  M.chunk_seg = reinterpret_cast<uint32_t*>(w + L.chunk_seg);
  M.total2 = reinterpret_cast<unsigned long long*>(w + L.total2);
  M.cursor2 = reinterpret_cast<unsigned long long*>(w + L.cursor2);
  M.bin_start = reinterpret_cast<unsigned long long*>(w + L.bin_start);
  M.bin_len = reinterpret_cast<unsigned long long*>(w + L.bin_len);
  M.ovf_len = reinterpret_cast<uint32_t*>(w + L.ovf_len);
  M.head = reinterpret_cast<unsigned int*>(w + L.head);
  return M;
}

// Radix passes of a partitioned build: groups the n pairs (keys, vals) by
// bin into (keys2, vals2), through (mid_k, mid_v) when two passes are
// planned.  T = key and value word (uint32_t or uint64_t).
template <typename T>
void launch_radix(const PartPlan& P, const PartMeta& M, const PartLayout& L, const T* keys,
                  const T* vals, uint64_t n, T* mid_k, T* mid_v, T* keys2, T* vals2,
                  uint32_t* status, hipStream_t st) {
  void (*hist)(PartPassT<T>);
  void (*scatter)(PartPassT<T>);
  void (*scatter_lines)(PartPassT<T>) = nullptr;
  if constexpr (sizeof(T) == 4) {
    hist = part_hist_kernel<uint32_t>;
    scatter = part_scatter_kernel<uint32_t>;
    scatter_lines = part_scatter_lines_kernel<uint32_t>;
  } else {
    hist = part_hist64_kernel;
    scatter = part_scatter64_kernel;
    scatter_lines = part_scatter_lines_kernel<uint64_t>;
  }
  // The second pass's chunks are cut for its scatter's rounds of resident
  // blocks.
  PartPlan Q = P;
  Q.resident2 = P.levels == 2
                    ? (uint32_t)resident_blocks((const void*)(P.lines2 ? scatter_lines : scatter),
                                                kPassBlock)
                    : 0u;
  part_clear_kernel<<<64, kPartBlock, 0, st>>>(M, P.fan1, P.levels, status);
  PartPassT<T> p1;
  p1.in_k = keys;
  p1.in_v = vals;
  p1.out_k = P.levels == 1 ? keys2 : mid_k;
  p1.out_v = P.levels == 1 ? vals2 : mid_v;
  p1.n = n;
  p1.level = 1;
  p1.fan = P.fan1;
  p1.lines = P.lines1;
  p1.padded = 0;
  p1.status = status;
  p1.P = Q;
  p1.M = M;
  hist<<<(unsigned)L.chunks1, kPassBlock, 0, st>>>(p1);
  part_scan1_kernel<<<1, kPartBlock, 0, st>>>(Q, M, status);
  (P.lines1 ? scatter_lines : scatter)<<<(unsigned)L.chunks1, kPassBlock, 0, st>>>(p1);
  if (P.levels == 2) {
    PartPassT<T> p2 = p1;
    p2.in_k = mid_k;
    p2.in_v = mid_v;
    p2.out_k = keys2;
    p2.out_v = vals2;
    p2.level = 2;
    p2.fan = kFan2;
    p2.lines = P.lines2;
    p2.padded = P.lines1;
    hist<<<(unsigned)L.chunks2, kPassBlock, 0, st>>>(p2);
    part_scan2_kernel<<<P.fan1, kPartBlock, 0, st>>>(Q, M, status);
    (P.lines2 ? scatter_lines : scatter)<<<(unsigned)L.chunks2, kPassBlock, 0, st>>>(p2);
  }
}

// Partitioned build of a 64-bit table (8-slot buckets); library-owned
// workspace.
bht_status build64_partitioned(bht_table* t, const uint64_t* keys, const uint64_t* vals,
                               uint64_t n, hipStream_t st) {
  PartPlan P;
  if (!part_plan(t, n, &P)) return fail(BHT_ERR_UNSUPPORTED, "table too large to partition");
  const PartLayout L = part_layout(P, n, 8);
  char* w = nullptr;
  bht_status ws_status = part_workspace(t, L, st, nullptr, 0, &w);
  if (ws_status != BHT_OK) return ws_status;
  const PartMeta M = part_meta(L, w);
  uint64_t* keys2 = reinterpret_cast<uint64_t*>(w + L.keys);
  uint64_t* vals2 = reinterpret_cast<uint64_t*>(w + L.vals);
  // the first of two passes writes into the slot array (2 words per slot,
  // at least mid_words pairs: the plan checks it when the pass pads)
  uint64_t* mid_k = t->d_slots;
  uint64_t* mid_v = mid_k + L.mid_words;

  if (t->timing) HIP_TRY(hipEventRecord(t->ev[0], st));
  launch_radix<uint64_t>(P, M, L, keys, vals, n, mid_k, mid_v, keys2, vals2, t->d_status, st);
  BinArgs64 ba;
  ba.slots = t->d_slots;
  ba.keys = keys2;
  ba.vals = vals2;
  ba.status = t->d_status;
  ba.max_chain = t->params.max_chain;
  ba.rng_seed = (uint32_t)t->params.rng_seed;
  ba.P = P;
  ba.M = M;
  bin_place64_kernel<<<P.nbins, kBinBlock, 0, st>>>(ba);
  WideOverflowArgs oa;
  oa.g.slots = t->d_slots;
  oa.g.keys = keys2;
  oa.g.vals = vals2;
  oa.g.n = n;
  oa.g.status = t->d_status;
  oa.g.H = P.H64;
  oa.g.max_chain = t->params.max_chain;
  oa.g.rng_seed = (uint32_t)t->params.rng_seed;
  oa.M = M;
  oa.nbins = P.nbins;
  const int og = grid_for((const void*)wide_overflow_kernel<8>, (uint64_t)P.nbins * 64,
                          t->grid_blocks);
  wide_overflow_kernel<8><<<og, kBlock, 0, st>>>(oa);
  HIP_TRY(hipGetLastError());
  if (t->timing) HIP_TRY(hipEventRecord(t->ev[1], st));
  t->build_timed = t->timing;
  t->pending = true;
  t->pending_n = n;
  t->pending_partitioned = true;
  return BHT_OK;
}

// ws: caller-owned workspace of ws_bytes, or null for the table's own.
bht_status build32_partitioned(bht_table* t, const uint32_t* keys, const uint32_t* vals,
                               uint64_t n, hipStream_t st, void* ws = nullptr,
                               uint64_t ws_bytes = 0) {
  PartPlan P;
  if (!part_plan(t, n, &P)) return fail(BHT_ERR_UNSUPPORTED, "table too large to partition");
  PartKernels K;
  if (!part_kernels(t, t->tile, &K))
    return fail(BHT_ERR_UNSUPPORTED, "no kernel for this bucket size and tile width");
  const PartLayout L = part_layout(P, n);
  char* w = nullptr;
  bht_status ws_status = part_workspace(t, L, st, ws, ws_bytes, &w);
  if (ws_status != BHT_OK) return ws_status;
  const PartMeta M = part_meta(L, w);
  uint32_t* keys2 = reinterpret_cast<uint32_t*>(w + L.keys);
  uint32_t* vals2 = reinterpret_cast<uint32_t*>(w + L.vals);
  // With two passes the first pass writes into the table's slot array,
  // which holds at least mid_words pairs (the plan checks it when the pass
  // pads) and is rewritten whole by the placement (and a two-level iceberg
  // table's secondary array by the reset below).
  uint32_t* mid_k = reinterpret_cast<uint32_t*>(t->d_slots);
  uint32_t* mid_v = mid_k + L.mid_words;

  if (t->timing) HIP_TRY(hipEventRecord(t->ev[0], st));
  launch_radix<uint32_t>(P, M, L, keys, vals, n, mid_k, mid_v, keys2, vals2, t->d_status, st);
  if (uint64_t* sec = secondary_slots(t)) {
    const uint64_t words = t->params.iht_secondary_m * t->params.iht_secondary_b;
    const int grid = (int)std::min<uint64_t>((words / 2 + kBlock) / kBlock, 8192);
    fill_empty_kernel<<<grid, kBlock, 0, st>>>(sec, words, nullptr);
  }
  BinArgs ba;
  ba.slots = t->d_slots;
  ba.keys = keys2;
  ba.vals = vals2;
  ba.status = t->d_status;
  ba.max_chain = t->params.max_chain;
  ba.rng_seed = t->params.rng_seed;
  ba.cap = K.iceberg ? std::min(t->params.iht_threshold, t->b) : t->b;
  ba.P = P;
  ba.M = M;
  reinterpret_cast<void (*)(BinArgs)>(const_cast<void*>(K.place))
      <<<P.nbins, kBinBlock, 0, st>>>(ba);
  if (K.iceberg) {
    IcebergOverflowArgs ia;
    ia.g.slots = t->d_slots;
    ia.g.slots2 = secondary_slots(t);
    ia.g.keys = keys2;
    ia.g.vals = vals2;
    ia.g.n = n;
    ia.g.status = t->d_status;
    ia.g.probe_total = nullptr;
    ia.g.H = P.H;
    ia.g.H2 = secondary_hash(t);
    ia.g.threshold = t->params.iht_threshold;
    ia.M = M;
    ia.nbins = P.nbins;
    // Secondary choices are made on device-scope reads and made again when
    // a concurrent placement takes the chosen slot, so they follow current
    // loads with the whole device in flight (at 2^27 pairs the highest load
    // factor reached is 0.86 at any spread from 1 to 32 secondary buckets
    // per lane; with reads that could be stale a full device failed 5 of 6
    // builds at 0.86 and needed a spread of 32).
    const uint64_t sec_buckets = t->params.iht_secondary_b ? t->params.iht_secondary_m : t->m;
    const uint64_t lanes = std::max<uint64_t>(sec_buckets / kIcebergOverflowSpread, 64);
    const int ig = grid_for(K.overflow, lanes, t->grid_blocks);
    reinterpret_cast<void (*)(IcebergOverflowArgs)>(const_cast<void*>(K.overflow))
        <<<ig, kBlock, 0, st>>>(ia);
  } else {
    OverflowArgs oa;
    oa.g.slots = t->d_slots;
    oa.g.keys = keys2;
    oa.g.vals = vals2;
    oa.g.n = n;
    oa.g.status = t->d_status;
    oa.g.probe_total = nullptr;
    oa.g.H = P.H;
    oa.g.max_chain = t->params.max_chain;
    oa.g.rng_seed = t->params.rng_seed;
    oa.M = M;
    oa.nbins = P.nbins;
    const int og = grid_for(K.overflow, (uint64_t)P.nbins * 64, t->grid_blocks);
    reinterpret_cast<void (*)(OverflowArgs)>(const_cast<void*>(K.overflow))
        <<<og, kBlock, 0, st>>>(oa);
  }
  HIP_TRY(hipGetLastError());
  if (t->timing) HIP_TRY(hipEventRecord(t->ev[1], st));
  t->build_timed = t->timing;
  t->pending = true;
  t->pending_n = n;
  t->pending_partitioned = true;
  return BHT_OK;
}

bht_status build32_enqueue(bht_table* t, const uint32_t* keys, const uint32_t* vals, uint64_t n,
                           unsigned long long* probe_total, void* stream) {
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (t->key_bits != 32) return fail(BHT_ERR_INVALID_ARG, "table holds 64-bit keys");
  if (n > t->slots) return fail(BHT_ERR_CAPACITY, "more pairs than slots");
  if (n && (!keys || !vals)) return fail(BHT_ERR_INVALID_ARG, "null key or value pointer");
  KernelSet ks;
  if (!pick(t, t->tile, t->find_schedule, probe_total != nullptr, &ks))
    return fail(BHT_ERR_UNSUPPORTED, "no kernel for this bucket size and tile width");
  hipStream_t st = as_stream(stream);
  t->built = false;
  t->pending_partitioned = false;
  t->counted_build_probes = 0;
  if (use_partitioned(t, n, probe_total != nullptr)) return build32_partitioned(t, keys, vals, n, st);
  bht_status s = launch_fill(t, st);
  if (s != BHT_OK) return s;
  if (n) {
    // Load-balanced placements (power of two, iceberg) decide from bucket
    // loads read before the lane's CAS; with every pair of a small table in
    // flight at once those loads would all be stale.  Giving each lane at
    // least 32 pairs keeps the pairs in flight under ~3% of the table, so
    // placement matches the serial rule; large tables still fill the device.
    const uint64_t grid_items =
        ks.kind == Kind::Cuckoo ? n : (n + kLbPairsPerLane - 1) / kLbPairsPerLane;
    const int grid = grid_for(ks.build, grid_items, t->grid_blocks);
    if (t->timing) HIP_TRY(hipEventRecord(t->ev[0], st));
    if (ks.kind == Kind::Cuckoo || ks.kind == Kind::LoadBalanced) {
      BuildArgs32 g;
      g.slots = t->d_slots;
      g.keys = keys;
      g.vals = vals;
      g.n = n;
      g.status = t->d_status;
      g.probe_total = probe_total;
      g.H = make_hash32(t->params, t->m, t->params.num_hashes);
      g.max_chain = t->params.max_chain;
      g.rng_seed = t->params.rng_seed;
      reinterpret_cast<void (*)(BuildArgs32)>(const_cast<void*>(ks.build))
          <<<grid, kBlock, 0, st>>>(g);
    } else {
      SchemeArgs32 g;
      g.slots = t->d_slots;
      g.slots2 = secondary_slots(t);
      g.keys = keys;
      g.vals = vals;
      g.n = n;
      g.status = t->d_status;
      g.probe_total = probe_total;
      g.H = make_hash32(t->params, t->m, t->params.num_hashes);
      g.H2 = secondary_hash(t);
      g.threshold = t->params.iht_threshold;
      reinterpret_cast<void (*)(SchemeArgs32)>(const_cast<void*>(ks.build))
          <<<grid, kBlock, 0, st>>>(g);
    }
    HIP_TRY(hipGetLastError());
    if (t->timing) HIP_TRY(hipEventRecord(t->ev[1], st));
    t->build_timed = t->timing;
  }
  t->pending = true;
  t->pending_n = n;
  return BHT_OK;
}

bht_status find32_enqueue(const bht_table* t, const uint32_t* q, uint64_t n, uint32_t* out_v,
                          uint8_t* out_f, uint8_t* probes, void* stream) {
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (t->key_bits != 32) return fail(BHT_ERR_INVALID_ARG, "table holds 64-bit keys");
  if (!t->built) return fail(BHT_ERR_NOT_BUILT, "find before a successful build");
  if (n == 0) return BHT_OK;
  if (!q || !out_v || !out_f) return fail(BHT_ERR_INVALID_ARG, "null query or output pointer");
  KernelSet ks;
  if (!pick(t, t->tile, t->find_schedule, probes != nullptr, &ks))
    return fail(BHT_ERR_UNSUPPORTED, "no kernel for this bucket size and tile width");
  hipStream_t st = as_stream(stream);
  const int grid = grid_for(ks.find, n, t->grid_blocks, ks.chunk ? 16 : 0);
  bht_table* mt = const_cast<bht_table*>(t);
  if (t->timing) HIP_TRY(hipEventRecord(t->ev[2], st));
  if (ks.kind == Kind::Cuckoo) {
    FindArgs32 g;
    g.slots = t->d_slots;
    g.queries = q;
    g.n = n;
    g.out_v = out_v;
    g.out_f = out_f;
    g.probes = probes;
    g.H = make_hash32(t->params, t->m, t->params.num_hashes);
    reinterpret_cast<void (*)(FindArgs32)>(const_cast<void*>(ks.find)) <<<grid, kBlock, 0, st>>>(g);
  } else {
    SchemeFindArgs32 g;
    g.slots = t->d_slots;
    g.slots2 = secondary_slots(t);
    g.queries = q;
    g.n = n;
    g.out_v = out_v;
    g.out_f = out_f;
    g.probes = probes;
    g.H = make_hash32(t->params, t->m, t->params.num_hashes);
    g.H2 = secondary_hash(t);
    g.rounds = t->params.num_hashes;
    g.early_below = t->scheme == BHT_IHT && t->iht_early_exit ? t->params.iht_threshold : 0;
    reinterpret_cast<void (*)(SchemeFindArgs32)>(const_cast<void*>(ks.find))
        <<<grid, kBlock, 0, st>>>(g);
  }
  HIP_TRY(hipGetLastError());
  if (t->timing) HIP_TRY(hipEventRecord(t->ev[3], st));
  mt->find_timed = t->timing;
  if (probes) return add_find_probes(probes, n, t, st);
  return BHT_OK;
}

}  // namespace

extern "C" {

const char* bht_status_string(bht_status s) {
  switch (s) {
    case BHT_OK: return "ok";
    case BHT_ERR_INVALID_ARG: return "invalid argument";
    case BHT_ERR_CAPACITY: return "more pairs than slots";
    case BHT_ERR_SENTINEL_KEY: return "input key equals the reserved empty key";
    case BHT_ERR_BUILD_FAILED: return "build failed (reseed and rebuild)";
    case BHT_ERR_NOT_BUILT: return "table not built";
    case BHT_ERR_OOM: return "device allocation failed";
    case BHT_ERR_HIP: return "HIP runtime error";
    case BHT_ERR_UNSUPPORTED: return "unsupported parameters";
  }
  return "unknown status";
}

const char* bht_last_error(void) { return g_last_error.c_str(); }

uint64_t bht_hash32(uint64_t a, uint64_t b, uint32_t k, uint64_t m) {
  if (m == 0 || m > 0xFFFFFFFFull) return ~0ull;
  return hash32((uint32_t)a, (uint32_t)b, k, fastmod32_constant((uint32_t)m), (uint32_t)m);
}

uint64_t bht_hash64(uint64_t a, uint64_t b, uint64_t k, uint64_t m) {
  if (m == 0) return ~0ull;
  return hash64(a, b, k, UINT64_MAX / m, m);
}

}  // extern "C"

namespace {

// Geometry of a table; returns false (with *why) for invalid parameters.
struct Geometry {
  uint64_t m, slots, words, slot_bytes, total_bytes;
};

bool geometry(uint64_t capacity_slots, uint32_t bucket_size, bht_scheme scheme,
              const bht_params* params, Geometry* g, bht_status* err) {
  if (!params) return *err = fail(BHT_ERR_INVALID_ARG, "null argument"), false;
  if (bucket_size == 0 || capacity_slots == 0)
    return *err = fail(BHT_ERR_INVALID_ARG, "zero size"), false;
  std::string why;
  if (!valid_params(*params, scheme, bucket_size, &why))
    return *err = fail(BHT_ERR_INVALID_ARG, why), false;
  g->m = (capacity_slots + bucket_size - 1) / bucket_size;
  if (g->m > 0xFFFFFFFFull) return *err = fail(BHT_ERR_INVALID_ARG, "more than 2^32 - 1 buckets"), false;
  g->slots = g->m * bucket_size;
  if (scheme == BHT_IHT && params->iht_secondary_b)
    g->slots += params->iht_secondary_m * params->iht_secondary_b;
  g->words = g->slots * (params->key_bits == 64 ? 2 : 1);
  g->slot_bytes = (g->words * sizeof(uint64_t) + 255) / 256 * 256;
  g->total_bytes = g->slot_bytes + 256;          // + the build status words
  return true;
}

bht_status create_common(uint64_t capacity_slots, uint32_t bucket_size, bht_scheme scheme,
                         const bht_params* params, void* buffer, uint64_t buffer_bytes,
                         bht_table** out) {
  if (!out) return fail(BHT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  Geometry g;
  bht_status err = BHT_OK;
  if (!geometry(capacity_slots, bucket_size, scheme, params, &g, &err)) return err;
  bht_table* t = new bht_table();
  t->scheme = scheme;
  t->b = bucket_size;
  t->m = g.m;
  t->key_bits = params->key_bits;
  t->params = *params;
  t->tile = default_tile(scheme, bucket_size);
  t->unroll = default_unroll(scheme, bucket_size);
  t->slots = g.slots;
  t->words = g.words;
  hipError_t e = hipGetDevice(&t->device);
  if (e != hipSuccess) {
    delete t;
    return hip_fail(e, "hipGetDevice");
  }
  char* base = static_cast<char*>(buffer);
  if (!buffer) {
    e = hipMalloc(&base, g.total_bytes);
    if (e != hipSuccess) {
      delete t;
      return fail(BHT_ERR_OOM, std::string("slot array: ") + hipGetErrorString(e));
    }
    t->owns_memory = true;
  } else if (buffer_bytes < g.total_bytes || (reinterpret_cast<uintptr_t>(buffer) & 255)) {
    delete t;
    return fail(BHT_ERR_INVALID_ARG, "buffer too small or not 256-byte aligned");
  }
  t->d_slots = reinterpret_cast<uint64_t*>(base);
  t->d_status = reinterpret_cast<uint32_t*>(base + g.slot_bytes);
  // the find-probe counter starts from whatever the memory holds
  e = hipMemcpy(&t->find_probe_base, find_probe_counter(t), 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    if (t->owns_memory) (void)hipFree(base);
    delete t;
    return hip_fail(e, "reading the status area");
  }
  *out = t;
  return BHT_OK;
}

}  // namespace

extern "C" {

uint64_t bht_table_bytes(uint64_t capacity_slots, uint32_t bucket_size, bht_scheme scheme,
                         const bht_params* params) {
  Geometry g;
  bht_status err;
  return geometry(capacity_slots, bucket_size, scheme, params, &g, &err) ? g.total_bytes : 0;
}

bht_status bht_create(uint64_t capacity_slots, uint32_t bucket_size, bht_scheme scheme,
                      const bht_params* params, bht_table** out) {
  return create_common(capacity_slots, bucket_size, scheme, params, nullptr, 0, out);
}

bht_status bht_create_in(uint64_t capacity_slots, uint32_t bucket_size, bht_scheme scheme,
                         const bht_params* params, void* d_buffer, uint64_t buffer_bytes,
                         bht_table** out) {
  if (!d_buffer) return fail(BHT_ERR_INVALID_ARG, "null buffer");
  return create_common(capacity_slots, bucket_size, scheme, params, d_buffer, buffer_bytes, out);
}

void bht_destroy(bht_table* t) {
  if (!t) return;
  if (t->timing)
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(t->ev[i]);
  if (t->owns_memory) (void)hipFree(t->d_slots);
  if (t->d_part) (void)hipFree(t->d_part);
  delete t;
}

bht_status bht_reseed(bht_table* t, const bht_params* params) {
  if (!t || !params) return fail(BHT_ERR_INVALID_ARG, "null argument");
  std::string why;
  if (params->key_bits != t->key_bits || !valid_params(*params, t->scheme, t->b, &why))
    return fail(BHT_ERR_INVALID_ARG, why.empty() ? "key width differs" : why);
  t->params = *params;
  t->built = false;
  return BHT_OK;
}

bht_status bht_build_async(bht_table* t, const uint32_t* d_keys, const uint32_t* d_values,
                           uint64_t n, void* stream) {
  return build32_enqueue(t, d_keys, d_values, n, nullptr, stream);
}

uint64_t bht_build_workspace_bytes(const bht_table* t, uint64_t n) {
  if (!t || t->key_bits != 32 || n == 0 || n >= (1ull << 32) || n > t->slots) return 0;
  if (t->scheme != BHT_BCHT && t->scheme != BHT_CHT1) return 0;
  PartPlan P;
  if (!part_plan(t, n, &P)) return 0;
  return part_layout(P, n).bytes;
}

bht_status bht_build_async_in(bht_table* t, const uint32_t* d_keys, const uint32_t* d_values,
                              uint64_t n, void* d_workspace, uint64_t workspace_bytes,
                              void* stream) {
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (t->key_bits != 32) return fail(BHT_ERR_INVALID_ARG, "table holds 64-bit keys");
  if (n > t->slots) return fail(BHT_ERR_CAPACITY, "more pairs than slots");
  if (n && (!d_keys || !d_values)) return fail(BHT_ERR_INVALID_ARG, "null key or value pointer");
  if (!d_workspace) return fail(BHT_ERR_INVALID_ARG, "null workspace");
  if (bht_build_workspace_bytes(t, n) == 0 || t->build_mode == BHT_BUILD_CONCURRENT)
    return build32_enqueue(t, d_keys, d_values, n, nullptr, stream);    // workspace unused
  KernelSet ks;
  if (!pick(t, t->tile, t->find_schedule, false, &ks))
    return fail(BHT_ERR_UNSUPPORTED, "no kernel for this bucket size and tile width");
  t->built = false;
  t->pending_partitioned = false;
  return build32_partitioned(t, d_keys, d_values, n, as_stream(stream), d_workspace,
                             workspace_bytes);
}

}  // extern "C"

// Workspace of the no-allocation build: device memory of the library's code
// object, one copy per GPU, held until the process ends.  In host code the
// array's name stands for a host-side shadow, never for device memory: its
// device address comes from hipGetSymbolAddress, once per device.
constexpr uint64_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// *out <- this device's copy of the scratch array; dev must be current.
bht_status scratch_for(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(BHT_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(BHT_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BHT_OK;
}

}  // namespace

extern "C" {

uint64_t bht_build_noalloc_max_bytes(void) { return kScratchBytes; }

bht_status bht_build_async_noalloc(bht_table* t, const uint32_t* d_keys,
                                   const uint32_t* d_values, uint64_t n, void* stream) {
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (t->key_bits != 32) return fail(BHT_ERR_INVALID_ARG, "table holds 64-bit keys");
  if (n > t->slots) return fail(BHT_ERR_CAPACITY, "more pairs than slots");
  if (n && (!d_keys || !d_values)) return fail(BHT_ERR_INVALID_ARG, "null key or value pointer");
  // the concurrent path has no workspace and allocates nothing
  if (!use_partitioned(t, n, false)) return build32_enqueue(t, d_keys, d_values, n, nullptr, stream);
  PartPlan P;
  if (!part_plan(t, n, &P)) return fail(BHT_ERR_UNSUPPORTED, "table too large to partition");
  const uint64_t need = part_layout(P, n).bytes;
  if (need > kScratchBytes)
    return fail(BHT_ERR_CAPACITY, "build needs " + std::to_string(need) +
                                      " bytes of workspace; the no-allocation scratch holds " +
                                      std::to_string(kScratchBytes));
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != t->device) return fail(BHT_ERR_INVALID_ARG, "the table's device is not current");
  void* ws = nullptr;
  const bht_status s = scratch_for(dev, &ws);
  if (s != BHT_OK) return s;
  KernelSet ks;
  if (!pick(t, t->tile, t->find_schedule, false, &ks))
    return fail(BHT_ERR_UNSUPPORTED, "no kernel for this bucket size and tile width");
  t->built = false;
  t->pending_partitioned = false;
  return build32_partitioned(t, d_keys, d_values, n, as_stream(stream), ws, kScratchBytes);
}

bht_status bht_build_wait(bht_table* t, void* stream) {
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (!t->pending) return t->built ? BHT_OK : fail(BHT_ERR_NOT_BUILT, "no build pending");
  hipStream_t st = as_stream(stream);
  HIP_TRY(hipMemcpyAsync(t->h_status, t->d_status, sizeof(t->h_status), hipMemcpyDeviceToHost,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  t->pending = false;
  const uint32_t flags = t->h_status[0];
  if (flags & kFlagSentinel)
    return fail(BHT_ERR_SENTINEL_KEY, t->key_bits == 64 ? "input holds a reserved 64-bit key"
                                                        : "input holds key 0xFFFFFFFF");
  if (flags & kFlagFailed) return fail(BHT_ERR_BUILD_FAILED, "eviction cap reached");
  t->built = true;
  t->n_stored = t->pending_n;
  t->last_partitioned = t->pending_partitioned;
  t->last_evicted = t->pending_partitioned ? t->h_status[1] : 0;
  t->last_probes = t->pending_partitioned
                       ? ((uint64_t)t->h_status[3] << 32 | t->h_status[2])
                       : 0;
  // words each radix pass wrote (0 when it did not run), less the pairs
  auto pad = [t](int w) {
    const uint64_t words = (uint64_t)t->h_status[w + 1] << 32 | t->h_status[w];
    return t->pending_partitioned && words > t->n_stored ? words - t->n_stored : 0;
  };
  t->last_pad1 = pad(kStatusPass1Words);
  t->last_pad2 = pad(kStatusPass2Words);
  return BHT_OK;
}

bht_status bht_build_padding(const bht_table* t, uint64_t* pass1_words, uint64_t* pass2_words) {
  if (!t || !pass1_words || !pass2_words) return fail(BHT_ERR_INVALID_ARG, "null argument");
  if (!t->built) return fail(BHT_ERR_NOT_BUILT, "no successful build");
  *pass1_words = t->last_pad1;
  *pass2_words = t->last_pad2;
  return BHT_OK;
}

bht_status bht_build_stats(const bht_table* t, uint32_t* partitioned, uint64_t* evicted,
                           uint64_t* overflow_probes) {
  if (!t || !partitioned || !evicted || !overflow_probes)
    return fail(BHT_ERR_INVALID_ARG, "null argument");
  if (!t->built) return fail(BHT_ERR_NOT_BUILT, "no successful build");
  *partitioned = t->last_partitioned ? 1u : 0u;
  *evicted = t->last_evicted;
  *overflow_probes = t->last_probes;
  return BHT_OK;
}

bht_status bht_build(bht_table* t, const uint32_t* d_keys, const uint32_t* d_values, uint64_t n,
                     void* stream) {
  bht_status s = build32_enqueue(t, d_keys, d_values, n, nullptr, stream);
  if (s != BHT_OK) return s;
  return bht_build_wait(t, stream);
}

bht_status bht_params_from_seed(uint64_t seed, bht_scheme scheme, uint32_t key_bits,
                                bht_params* out) {
  if (!out) return fail(BHT_ERR_INVALID_ARG, "null argument");
  if (key_bits != 32 && key_bits != 64) return fail(BHT_ERR_INVALID_ARG, "key_bits must be 32 or 64");
  bht_params p{};
  switch (scheme) {
    case BHT_BP2HT: p.num_hashes = 2; break;
    case BHT_BCHT: case BHT_IHT: case BHT_CHT1: case BHT_BCHT_LB: p.num_hashes = 3; break;
    default: return fail(BHT_ERR_INVALID_ARG, "unknown scheme");
  }
  p.key_bits = key_bits;
  p.max_chain = 128;
  draw_constants(seed, key_bits, p.a, p.b, &p.rng_seed);
  *out = p;
  return BHT_OK;
}

bht_status bht_build_retry(bht_table* t, const void* d_keys, const void* d_values, uint64_t n,
                           uint64_t seed, uint32_t max_attempts, uint32_t* attempts_out,
                           void* stream) {
  if (attempts_out) *attempts_out = 0;
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (max_attempts == 0) return fail(BHT_ERR_INVALID_ARG, "max_attempts must be at least 1");
  bht_status s = BHT_ERR_BUILD_FAILED;
  for (uint32_t attempt = 0; attempt < max_attempts; ++attempt) {
    if (attempt > 0) {
      // new constants for every retry; everything else stays as configured
      bht_params p = t->params;
      draw_constants(seed + attempt - 1, t->key_bits, p.a, p.b, &p.rng_seed);
      t->params = p;
      t->built = false;
    }
    s = t->key_bits == 64
            ? bht_build64(t, static_cast<const uint64_t*>(d_keys),
                          static_cast<const uint64_t*>(d_values), n, stream)
            : bht_build(t, static_cast<const uint32_t*>(d_keys),
                        static_cast<const uint32_t*>(d_values), n, stream);
    if (attempts_out) *attempts_out = attempt + 1;
    if (s != BHT_ERR_BUILD_FAILED) return s;
  }
  return s;
}

bht_status bht_build_counted(bht_table* t, const uint32_t* d_keys, const uint32_t* d_values,
                             uint64_t n, uint64_t* d_probe_total, void* stream) {
  if (!d_probe_total) return fail(BHT_ERR_INVALID_ARG, "null probe counter");
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  hipStream_t st = as_stream(stream);
  uint64_t before = 0, after = 0;
  HIP_TRY(hipMemcpyAsync(&before, d_probe_total, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  bht_status s = build32_enqueue(t, d_keys, d_values, n,
                                 reinterpret_cast<unsigned long long*>(d_probe_total), stream);
  if (s != BHT_OK) return s;
  s = bht_build_wait(t, stream);
  HIP_TRY(hipMemcpyAsync(&after, d_probe_total, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  t->counted_build_probes = after - before;
  return s;
}

bht_status bht_get_probe_stats(const bht_table* t, uint64_t* build_probes, uint64_t* find_probes) {
  if (!t || !build_probes || !find_probes) return fail(BHT_ERR_INVALID_ARG, "null argument");
  HIP_TRY(hipDeviceSynchronize());
  uint64_t now = 0;
  HIP_TRY(hipMemcpy(&now, find_probe_counter(t), 8, hipMemcpyDeviceToHost));
  bht_table* mt = const_cast<bht_table*>(t);
  *build_probes = t->counted_build_probes;
  *find_probes = now - t->find_probe_base;
  mt->find_probe_base = now;
  return BHT_OK;
}

bht_status bht_find(const bht_table* t, const uint32_t* d_queries, uint64_t n,
                    uint32_t* d_out_values, uint8_t* d_out_found, void* stream) {
  return find32_enqueue(t, d_queries, n, d_out_values, d_out_found, nullptr, stream);
}

bht_status bht_find_counted(const bht_table* t, const uint32_t* d_queries, uint64_t n,
                            uint32_t* d_out_values, uint8_t* d_out_found, uint8_t* d_probes,
                            void* stream) {
  if (!d_probes) return fail(BHT_ERR_INVALID_ARG, "null probe array");
  return find32_enqueue(t, d_queries, n, d_out_values, d_out_found, d_probes, stream);
}

bht_status bht_build64(bht_table* t, const uint64_t* d_keys, const uint64_t* d_values,
                       uint64_t n, void* stream) {
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (t->key_bits != 64) return fail(BHT_ERR_INVALID_ARG, "table holds 32-bit keys");
  if (n > t->slots) return fail(BHT_ERR_CAPACITY, "more pairs than slots");
  if (n && (!d_keys || !d_values)) return fail(BHT_ERR_INVALID_ARG, "null key or value pointer");
  if (t->b != 8) return fail(BHT_ERR_UNSUPPORTED, "64-bit tables use 8-slot buckets");
  hipStream_t st = as_stream(stream);
  t->built = false;
  t->pending_partitioned = false;
  t->counted_build_probes = 0;
  if (use_partitioned(t, n, false)) {
    bht_status s = build64_partitioned(t, d_keys, d_values, n, st);
    if (s != BHT_OK) return s;
    return bht_build_wait(t, stream);
  }
  bht_status s = launch_fill(t, st);
  if (s != BHT_OK) return s;
  if (n) {
    WideBuildArgs g;
    g.slots = t->d_slots;
    g.keys = d_keys;
    g.vals = d_values;
    g.n = n;
    g.status = t->d_status;
    g.H = make_hash64(t->params, t->m, t->params.num_hashes);
    g.max_chain = t->params.max_chain;
    g.rng_seed = t->params.rng_seed;
    const int grid = grid_for((const void*)wide_build_kernel<8>, n, t->grid_blocks);
    if (t->timing) HIP_TRY(hipEventRecord(t->ev[0], st));
    wide_build_kernel<8><<<grid, kBlock, 0, st>>>(g);
    HIP_TRY(hipGetLastError());
    if (t->timing) HIP_TRY(hipEventRecord(t->ev[1], st));
    t->build_timed = t->timing;
  }
  t->pending = true;
  t->pending_n = n;
  return bht_build_wait(t, stream);
}

}  // extern "C"

namespace {

bht_status find64_enqueue(const bht_table* t, const uint64_t* q, uint64_t n, uint64_t* out_v,
                          uint8_t* out_f, uint8_t* probes, void* stream) {
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (t->key_bits != 64) return fail(BHT_ERR_INVALID_ARG, "table holds 32-bit keys");
  if (!t->built) return fail(BHT_ERR_NOT_BUILT, "find before a successful build");
  if (n == 0) return BHT_OK;
  if (!q || !out_v || !out_f) return fail(BHT_ERR_INVALID_ARG, "null query or output pointer");
  WideFindArgs g;
  g.slots = t->d_slots;
  g.queries = q;
  g.n = n;
  g.out_v = out_v;
  g.out_f = out_f;
  g.probes = probes;
  g.H = make_hash64(t->params, t->m, t->params.num_hashes);
  hipStream_t st = as_stream(stream);
  const void* kernel = probes ? (const void*)wide_find_chunk_kernel<8, true>
                              : (const void*)wide_find_chunk_kernel<8, false>;
  const int grid = grid_for(kernel, n, t->grid_blocks, 16);
  bht_table* mt = const_cast<bht_table*>(t);
  if (t->timing) HIP_TRY(hipEventRecord(t->ev[2], st));
  reinterpret_cast<void (*)(WideFindArgs)>(const_cast<void*>(kernel)) <<<grid, kBlock, 0, st>>>(g);
  HIP_TRY(hipGetLastError());
  if (t->timing) HIP_TRY(hipEventRecord(t->ev[3], st));
  mt->find_timed = t->timing;
  if (probes) return add_find_probes(probes, n, t, st);
  return BHT_OK;
}

}  // namespace

extern "C" {

bht_status bht_find64(const bht_table* t, const uint64_t* d_queries, uint64_t n,
                      uint64_t* d_out_values, uint8_t* d_out_found, void* stream) {
  return find64_enqueue(t, d_queries, n, d_out_values, d_out_found, nullptr, stream);
}

bht_status bht_find64_counted(const bht_table* t, const uint64_t* d_queries, uint64_t n,
                              uint64_t* d_out_values, uint8_t* d_out_found, uint8_t* d_probes,
                              void* stream) {
  if (!d_probes) return fail(BHT_ERR_INVALID_ARG, "null probe array");
  return find64_enqueue(t, d_queries, n, d_out_values, d_out_found, d_probes, stream);
}

bht_status bht_set_tuning(bht_table* t, const bht_tuning* tuning) {
  if (!t || !tuning) return fail(BHT_ERR_INVALID_ARG, "null argument");
  const uint32_t w = tuning->tile_width ? tuning->tile_width : t->tile;
  if (tuning->find_schedule > BHT_FIND_PARALLEL) return fail(BHT_ERR_INVALID_ARG, "bad schedule");
  if (tuning->build_mode > BHT_BUILD_PARTITIONED) return fail(BHT_ERR_INVALID_ARG, "bad build mode");
  if (tuning->iht_early_exit > 1) return fail(BHT_ERR_INVALID_ARG, "iht_early_exit must be 0 or 1");
  if (tuning->query_unroll > 2) return fail(BHT_ERR_INVALID_ARG, "query_unroll must be 0, 1 or 2");
  if (tuning->iht_early_exit && t->scheme != BHT_IHT)
    return fail(BHT_ERR_UNSUPPORTED, "early exit after the primary applies to iceberg tables");
  if (t->key_bits == 64) {
    if (w != 8) return fail(BHT_ERR_UNSUPPORTED, "64-bit tables read buckets with 8 lanes");
    t->grid_blocks = tuning->grid_blocks;
    t->build_mode = tuning->build_mode;
    return BHT_OK;
  }
  KernelSet ks;
  if (!pick(t, w, tuning->find_schedule, false, &ks))
    return fail(BHT_ERR_UNSUPPORTED, "no kernel for this bucket size and tile width");
  t->tile = w;
  t->find_schedule = tuning->find_schedule;
  t->grid_blocks = tuning->grid_blocks;
  t->build_mode = tuning->build_mode;
  t->iht_early_exit = tuning->iht_early_exit;
  t->unroll = tuning->query_unroll ? tuning->query_unroll : default_unroll(t->scheme, t->b);
  return BHT_OK;
}

bht_status bht_get_tuning(const bht_table* t, bht_tuning* tuning) {
  if (!t || !tuning) return fail(BHT_ERR_INVALID_ARG, "null argument");
  tuning->tile_width = t->tile;
  tuning->find_schedule = t->find_schedule;
  tuning->grid_blocks = t->grid_blocks;
  tuning->build_mode = t->build_mode;
  tuning->iht_early_exit = t->iht_early_exit;
  tuning->query_unroll = t->unroll == 2 ? 2 : 1;
  return BHT_OK;
}

bht_status bht_enable_timing(bht_table* t, int on) {
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (on && !t->timing) {
    for (int i = 0; i < 4; ++i) HIP_TRY(hipEventCreate(&t->ev[i]));
    t->timing = true;
  }
  return BHT_OK;
}

bht_status bht_kernel_ms(const bht_table* t, float* build_ms, float* find_ms) {
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (!t->timing) return fail(BHT_ERR_INVALID_ARG, "timing not enabled");
  if (build_ms) {
    *build_ms = -1.0f;
    if (t->build_timed) {
      HIP_TRY(hipEventSynchronize(t->ev[1]));
      HIP_TRY(hipEventElapsedTime(build_ms, t->ev[0], t->ev[1]));
    }
  }
  if (find_ms) {
    *find_ms = -1.0f;
    if (t->find_timed) {
      HIP_TRY(hipEventSynchronize(t->ev[3]));
      HIP_TRY(hipEventElapsedTime(find_ms, t->ev[2], t->ev[3]));
    }
  }
  return BHT_OK;
}

bht_status bht_info(const bht_table* t, uint64_t* num_buckets, uint32_t* bucket_size,
                    uint64_t* n_stored, uint64_t* table_bytes) {
  if (!t) return fail(BHT_ERR_INVALID_ARG, "null table");
  if (num_buckets) *num_buckets = t->m;
  if (bucket_size) *bucket_size = t->b;
  if (n_stored) *n_stored = t->built ? t->n_stored : 0;
  if (table_bytes) *table_bytes = t->words * sizeof(uint64_t);
  return BHT_OK;
}

bht_status bht_download(const bht_table* t, void* host_slots) {
  if (!t || !host_slots) return fail(BHT_ERR_INVALID_ARG, "null argument");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(host_slots, t->d_slots, t->words * sizeof(uint64_t), hipMemcpyDeviceToHost));
  return BHT_OK;
}

bht_status bht_upload(bht_table* t, const void* host_slots, uint64_t n_stored) {
  if (!t || !host_slots) return fail(BHT_ERR_INVALID_ARG, "null argument");
  if (n_stored > t->slots) return fail(BHT_ERR_CAPACITY, "more pairs than slots");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(t->d_slots, host_slots, t->words * sizeof(uint64_t), hipMemcpyHostToDevice));
  t->built = true;
  t->pending = false;
  t->n_stored = n_stored;
  t->counted_build_probes = 0;
  return BHT_OK;
}

bht_status bht_device_slots(const bht_table* t, void** d_slots) {
  if (!t || !d_slots) return fail(BHT_ERR_INVALID_ARG, "null argument");
  *d_slots = t->d_slots;
  return BHT_OK;
}

bht_status bht_diag_gather(const void* d_buf, uint64_t bytes, uint64_t n_reads, uint32_t line_bytes,
                           uint64_t seed, uint64_t* d_sink, void* stream) {
  if (!d_buf || !d_sink) return fail(BHT_ERR_INVALID_ARG, "null pointer");
  if (line_bytes != 32 && line_bytes != 64 && line_bytes != 128 && line_bytes != 256)
    return fail(BHT_ERR_INVALID_ARG, "line_bytes must be 32, 64, 128 or 256");
  if (bytes < line_bytes) return fail(BHT_ERR_INVALID_ARG, "buffer smaller than one line");
  const uint64_t* buf = static_cast<const uint64_t*>(d_buf);
  auto sink = reinterpret_cast<unsigned long long*>(d_sink);
  hipStream_t st = as_stream(stream);
  const uint64_t units64 = bytes / line_bytes;
  const uint32_t units = (uint32_t)std::min<uint64_t>(units64, 0xFFFFFFFFull);
#define BHT_GATHER(LB)                                                              \
  if (line_bytes == LB) {                                                           \
    const int grid = grid_for((const void*)diag_gather_kernel<LB>, 1ull << 40);     \
    diag_gather_kernel<LB><<<grid, kBlock, 0, st>>>(buf, units, n_reads, seed, sink); \
  }
  BHT_GATHER(32)
  BHT_GATHER(64)
  BHT_GATHER(128)
  BHT_GATHER(256)
#undef BHT_GATHER
  HIP_TRY(hipGetLastError());
  return BHT_OK;
}

bht_status bht_diag_stream(const void* d_src, void* d_dst, uint64_t bytes, uint64_t* d_sink,
                           void* stream) {
  if (!d_src || !d_sink || bytes < 16) return fail(BHT_ERR_INVALID_ARG, "bad buffer");
  if ((reinterpret_cast<uintptr_t>(d_src) | reinterpret_cast<uintptr_t>(d_dst)) & 15)
    return fail(BHT_ERR_INVALID_ARG, "buffers must be 16-byte aligned");
  const uint64_t n16 = bytes / 16;
  const auto* src = static_cast<const u64x2*>(d_src);
  auto* dst = static_cast<u64x2*>(d_dst);
  auto sink = reinterpret_cast<unsigned long long*>(d_sink);
  hipStream_t st = as_stream(stream);
  const uint64_t blocks = (n16 + kStreamChunk - 1) / kStreamChunk;
  if (blocks > 0x7FFFFFFFull) return fail(BHT_ERR_INVALID_ARG, "buffer too large");
  if (dst)
    diag_stream_kernel<true><<<(unsigned)blocks, kBlock, 0, st>>>(src, dst, n16, sink);
  else
    diag_stream_kernel<false><<<(unsigned)blocks, kBlock, 0, st>>>(src, nullptr, n16, sink);
  HIP_TRY(hipGetLastError());
  return BHT_OK;
}

bht_status bht_diag_cas(void* d_buf, uint64_t bytes, uint64_t n_ops, uint64_t seed,
                        uint64_t* d_sink, void* stream) {
  if (!d_buf || !d_sink || bytes < 8) return fail(BHT_ERR_INVALID_ARG, "bad buffer");
  const int grid = grid_for((const void*)diag_cas_kernel, 1ull << 40);
  diag_cas_kernel<<<grid, kBlock, 0, as_stream(stream)>>>(
      static_cast<uint64_t*>(d_buf), (uint32_t)std::min<uint64_t>(bytes / 8, 0xFFFFFFFFull), n_ops,
      seed,
      reinterpret_cast<unsigned long long*>(d_sink));
  HIP_TRY(hipGetLastError());
  return BHT_OK;
}

bht_status bht_batch_create(const bht_batch_entry* entries, uint32_t count, uint32_t item_size,
                            bht_batch** out) {
  if (!out || (!entries && count)) return fail(BHT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (count == 0) return fail(BHT_ERR_INVALID_ARG, "empty batch");
  if (item_size == 0) item_size = 8192;
  if (item_size < 64) return fail(BHT_ERR_INVALID_ARG, "item_size must be at least 64");
  const bht_table* t0 = entries[0].table;
  if (!t0) return fail(BHT_ERR_INVALID_ARG, "null table");
  std::unordered_set<const bht_table*> seen;
  for (uint32_t i = 0; i < count; ++i) {
    const bht_batch_entry& e = entries[i];
    const bht_table* t = e.table;
    if (!t) return fail(BHT_ERR_INVALID_ARG, "null table in batch");
    if (!seen.insert(t).second) return fail(BHT_ERR_INVALID_ARG, "table appears twice in batch");
    if (t->scheme != BHT_BCHT || t->key_bits != 32)
      return fail(BHT_ERR_UNSUPPORTED, "batches hold 32-bit bucketed cuckoo tables");
    if (t->b != t0->b || t->tile != t0->tile || (t->unroll == 2) != (t0->unroll == 2))
      return fail(BHT_ERR_INVALID_ARG,
                  "tables of a batch share bucket size, tile width and query unroll");
    if (e.n_keys > t->slots) return fail(BHT_ERR_CAPACITY, "more pairs than slots");
    if ((e.n_keys && (!e.d_keys || !e.d_values)) ||
        (e.n_queries && (!e.d_queries || !e.d_out_values || !e.d_out_found)))
      return fail(BHT_ERR_INVALID_ARG, "null data pointer in batch");
  }
  const void* bk = nullptr;
  const void* fk = nullptr;
#define BHT_BATCH_CASE(B_, W_)                                             \
  if (t0->b == B_ && t0->tile == W_) {                                     \
    bk = (const void*)batch_build_kernel<B_, W_>;                          \
    fk = t0->unroll == 2 ? (const void*)batch_find_kernel<B_, W_, 2>       \
                         : (const void*)batch_find_kernel<B_, W_, 1>;      \
  }
  BHT_BATCH_CASE(8, 4)
  BHT_BATCH_CASE(8, 8)
  BHT_BATCH_CASE(16, 4)
  BHT_BATCH_CASE(16, 8)
  BHT_BATCH_CASE(16, 16)
  BHT_BATCH_CASE(32, 8)
  BHT_BATCH_CASE(32, 16)
#undef BHT_BATCH_CASE
  if (!bk) return fail(BHT_ERR_UNSUPPORTED, "no batched kernel for this bucket size and tile");
  const void* pk = nullptr;
  const void* ok = nullptr;
#define BHT_BATCH_PCASE(B_, W_)                                   \
  if (t0->b == B_ && t0->tile == W_) {                            \
    pk = (const void*)batch_place_kernel<B_>;                     \
    ok = (const void*)batch_overflow_kernel<B_, W_>;              \
  }
  BHT_BATCH_PCASE(8, 4)
  BHT_BATCH_PCASE(8, 8)
  BHT_BATCH_PCASE(16, 4)
  BHT_BATCH_PCASE(16, 8)
  BHT_BATCH_PCASE(16, 16)
  BHT_BATCH_PCASE(32, 8)
  BHT_BATCH_PCASE(32, 16)
#undef BHT_BATCH_PCASE

  std::vector<BatchTable> tables(count);
  std::vector<BatchItem> fill, build, find;
  const uint64_t fill_words = 1ull << 16;
  for (uint32_t i = 0; i < count; ++i) {
    const bht_batch_entry& e = entries[i];
    const bht_table* t = e.table;
    BatchTable& T = tables[i];
    T.slots = t->d_slots;
    T.words = t->words;
    T.keys = e.d_keys;
    T.vals = e.d_values;
    T.n_keys = e.n_keys;
    T.queries = e.d_queries;
    T.out_v = e.d_out_values;
    T.out_f = e.d_out_found;
    T.n_queries = e.n_queries;
    T.H = make_hash32(t->params, t->m, t->params.num_hashes);
    T.max_chain = t->params.max_chain;
    T.rng_seed = t->params.rng_seed;
    for (uint64_t s = 0; s < t->words; s += fill_words)
      fill.push_back({i, 0, s, std::min<uint64_t>(fill_words, t->words - s)});
    for (uint64_t s = 0; s < e.n_keys; s += item_size)
      build.push_back({i, 0, s, std::min<uint64_t>(item_size, e.n_keys - s)});
    for (uint64_t s = 0; s < e.n_queries; s += item_size)
      find.push_back({i, 0, s, std::min<uint64_t>(item_size, e.n_queries - s)});
  }
  bht_batch* b = new bht_batch();
  b->count = count;
  b->b = t0->b;
  b->tile = t0->tile;
  b->build_kernel = bk;
  b->find_kernel = fk;
  b->n_fill = fill.size();
  b->n_build = build.size();
  b->n_find = find.size();
  for (uint32_t i = 0; i < count; ++i) {
    b->tables.push_back(entries[i].table);
    b->n_keys.push_back(entries[i].n_keys);
  }
  std::vector<BatchItem> all(fill);
  all.insert(all.end(), build.begin(), build.end());
  all.insert(all.end(), find.begin(), find.end());
  hipError_t e = hipSuccess;
  {
    // Partitioned build: every table in one radix pass (at most kMaxFan bins
    // of bin_slots / b buckets each), fewer than 2^32 pairs in all, and no
    // table asks for the concurrent build.
    const uint64_t R = bin_slots<16>() / t0->b;
    uint64_t n_all = 0, bins = 0, counters = 0;
    bool part = pk != nullptr;
    for (uint32_t i = 0; i < count && part; ++i) {
      const bht_table* t = entries[i].table;
      const uint64_t nb = (t->m + R - 1) / R;
      if (nb > kMaxFan || t->build_mode == BHT_BUILD_CONCURRENT) part = false;
      n_all += entries[i].n_keys;
      bins += nb;
      counters += ((entries[i].n_keys + kBatchChunk - 1) / kBatchChunk) * nb;
    }
    if (n_all >= (1ull << 32) || bins >= (1ull << 32)) part = false;
    if (part) {
      std::vector<BatchPart> parts(count);
      std::vector<BatchChunk> chunks;
      std::vector<uint32_t> bin_table;
      bin_table.reserve(bins);
      uint64_t key_off = 0, hist_off = 0;
      for (uint32_t i = 0; i < count; ++i) {
        const bht_table* t = entries[i].table;
        const uint64_t n = entries[i].n_keys;
        const uint32_t nb = (uint32_t)((t->m + R - 1) / R);
        parts[i] = {key_off, hist_off, (uint32_t)bin_table.size(), nb};
        uint32_t local = 0;
        for (uint64_t s0 = 0; s0 < n; s0 += kBatchChunk, ++local)
          chunks.push_back({i, local, s0, std::min<uint64_t>(kBatchChunk, n - s0)});
        for (uint32_t j = 0; j < nb; ++j) bin_table.push_back(i);
        key_off += n;
        hist_off += (uint64_t)local * nb;
      }
      // workspace carve-up (256-byte aligned pieces)
      uint64_t off = 0;
      auto take = [&off](uint64_t bytes) {
        const uint64_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
      };
      const uint64_t o_keys = take(n_all * 4), o_vals = take(n_all * 4);
      const uint64_t o_hist = take(hist_off * 4);
      const uint64_t o_total = take(bins * 8), o_cursor = take(bins * 8);
      const uint64_t o_start = take(bins * 8), o_len = take(bins * 8);
      const uint64_t o_ovf = take(bins * 4), o_bt = take(bins * 4);
      const uint64_t o_parts = take(sizeof(BatchPart) * count);
      const uint64_t o_chunks = take(sizeof(BatchChunk) * std::max<size_t>(1, chunks.size()));
      const uint64_t o_head = take(16);
      e = hipMalloc(&b->d_ws, off);
      if (e == hipSuccess) {
        char* w = static_cast<char*>(b->d_ws);
        BatchPartArgs& pa = b->pa;
        pa.parts = reinterpret_cast<const BatchPart*>(w + o_parts);
        pa.chunks = reinterpret_cast<const BatchChunk*>(w + o_chunks);
        pa.bin_table = reinterpret_cast<const uint32_t*>(w + o_bt);
        pa.n_chunks = (uint32_t)chunks.size();
        pa.count = count;
        pa.nbins = (uint32_t)bins;
        pa.bin_shift = log2_exact(R);
        pa.hist = reinterpret_cast<uint32_t*>(w + o_hist);
        pa.total = reinterpret_cast<unsigned long long*>(w + o_total);
        pa.cursor = reinterpret_cast<unsigned long long*>(w + o_cursor);
        pa.bin_start = reinterpret_cast<unsigned long long*>(w + o_start);
        pa.bin_len = reinterpret_cast<unsigned long long*>(w + o_len);
        pa.ovf_len = reinterpret_cast<uint32_t*>(w + o_ovf);
        pa.keys = reinterpret_cast<uint32_t*>(w + o_keys);
        pa.vals = reinterpret_cast<uint32_t*>(w + o_vals);
        pa.head = reinterpret_cast<unsigned int*>(w + o_head);
        e = hipMemcpy(w + o_parts, parts.data(), sizeof(BatchPart) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess && !chunks.empty())
          e = hipMemcpy(w + o_chunks, chunks.data(), sizeof(BatchChunk) * chunks.size(),
                        hipMemcpyHostToDevice);
        if (e == hipSuccess)
          e = hipMemcpy(w + o_bt, bin_table.data(), 4 * bins, hipMemcpyHostToDevice);
        b->partitioned = e == hipSuccess;
        b->place_kernel = pk;
        b->overflow_kernel = ok;
      } else {
        b->d_ws = nullptr;          // not enough memory: the concurrent build serves
        e = hipSuccess;
        (void)hipGetLastError();
      }
    }
  }
  if (e == hipSuccess) e = hipMalloc(&b->d_tables, sizeof(BatchTable) * count);
  if (e == hipSuccess) e = hipMalloc(&b->d_items, sizeof(BatchItem) * std::max<size_t>(1, all.size()));
  if (e == hipSuccess) e = hipMalloc(&b->d_heads, 16);
  if (e == hipSuccess) e = hipMalloc(&b->d_status, sizeof(uint32_t) * count);
  if (e == hipSuccess) e = hipHostMalloc(&b->h_status, sizeof(uint32_t) * count, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_tables, tables.data(), sizeof(BatchTable) * count, hipMemcpyHostToDevice);
  if (e == hipSuccess && !all.empty())
    e = hipMemcpy(b->d_items, all.data(), sizeof(BatchItem) * all.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    bht_batch_destroy(b);
    return fail(BHT_ERR_OOM, std::string("batch arrays: ") + hipGetErrorString(e));
  }
  b->pa.tables = b->d_tables;
  b->pa.status = b->d_status;
  *out = b;
  return BHT_OK;
}

namespace {
bht_status batch_launch(bht_batch* b, hipStream_t st) {
  batch_reset_kernel<<<std::max<uint32_t>(1, std::min<uint32_t>((b->count + 255) / 256, 1024)),
                       256, 0, st>>>(b->d_heads, b->d_status, b->count);
  HIP_TRY(hipGetLastError());
  if (b->partitioned) {
    const BatchPartArgs& pa = b->pa;
    batch_part_clear_kernel<<<std::max<uint32_t>(1, std::min<uint32_t>((pa.nbins + 255) / 256, 1024)),
                              256, 0, st>>>(pa);
    if (pa.n_chunks) batch_part_hist_kernel<<<pa.n_chunks, kPassBlock, 0, st>>>(pa);
    batch_part_scan_kernel<<<pa.count, kPartBlock, 0, st>>>(pa);
    if (pa.n_chunks) batch_part_scatter_kernel<<<pa.n_chunks, kPassBlock, 0, st>>>(pa);
    reinterpret_cast<void (*)(BatchPartArgs)>(const_cast<void*>(b->place_kernel))
        <<<pa.nbins, kBinBlock, 0, st>>>(pa);
    const int og = grid_for(b->overflow_kernel, (uint64_t)pa.nbins * 64);
    reinterpret_cast<void (*)(BatchPartArgs)>(const_cast<void*>(b->overflow_kernel))
        <<<og, kBlock, 0, st>>>(pa);
    HIP_TRY(hipGetLastError());
  } else if (b->n_fill) {
    batch_fill_kernel<<<(int)std::min<uint64_t>(b->n_fill, 8192), kBlock, 0, st>>>(
        b->d_tables, b->d_items, b->n_fill);
    HIP_TRY(hipGetLastError());
  }
  if (b->n_build && !b->partitioned) {
    const int grid = grid_for(b->build_kernel, b->n_build * kBlock);
    reinterpret_cast<void (*)(const BatchTable*, const BatchItem*, uint64_t, unsigned int*,
                              uint32_t*)>(const_cast<void*>(b->build_kernel))
        <<<grid, kBlock, 0, st>>>(b->d_tables, b->d_items + b->n_fill, b->n_build, b->d_heads,
                                  b->d_status);
    HIP_TRY(hipGetLastError());
  }
  if (b->n_find) {
    const int grid = grid_for(b->find_kernel, b->n_find * kBlock);
    reinterpret_cast<void (*)(const BatchTable*, const BatchItem*, uint64_t, unsigned int*)>(
        const_cast<void*>(b->find_kernel))
        <<<grid, kBlock, 0, st>>>(b->d_tables, b->d_items + b->n_fill + b->n_build, b->n_find,
                                  b->d_heads + 1);
    HIP_TRY(hipGetLastError());
  }
  return BHT_OK;
}
}  // namespace

bht_status bht_batch_run(bht_batch* b, void* stream) {
  if (!b) return fail(BHT_ERR_INVALID_ARG, "null batch");
  hipStream_t st = as_stream(stream);
  for (bht_table* t : b->tables) {
    t->built = false;
    t->counted_build_probes = 0;
  }
  if (st == nullptr) return batch_launch(b, st);
  if (b->exec && b->graph_stream != st) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
  }
  if (!b->exec) {
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    bht_status s = batch_launch(b, st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != BHT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph = g;
    b->graph_stream = st;
  }
  HIP_TRY(hipGraphLaunch(b->exec, st));
  return BHT_OK;
}

bht_status bht_batch_wait(bht_batch* b, void* stream, bht_status* status_out) {
  if (!b) return fail(BHT_ERR_INVALID_ARG, "null batch");
  hipStream_t st = as_stream(stream);
  HIP_TRY(hipMemcpyAsync(b->h_status, b->d_status, sizeof(uint32_t) * b->count,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  bht_status worst = BHT_OK;
  for (uint32_t i = 0; i < b->count; ++i) {
    const uint32_t f = b->h_status[i];
    bht_status s = BHT_OK;
    if (f & kFlagSentinel) s = BHT_ERR_SENTINEL_KEY;
    else if (f & kFlagFailed) s = BHT_ERR_BUILD_FAILED;
    if (status_out) status_out[i] = s;
    bht_table* t = b->tables[i];
    t->built = s == BHT_OK;
    t->pending = false;
    t->n_stored = s == BHT_OK ? b->n_keys[i] : 0;
    if (s != BHT_OK && worst == BHT_OK) worst = s;
  }
  if (worst != BHT_OK) g_last_error = "some tables of the batch failed to build";
  return worst;
}

void bht_batch_destroy(bht_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_tables) (void)hipFree(b->d_tables);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_heads) (void)hipFree(b->d_heads);
  if (b->d_status) (void)hipFree(b->d_status);
  if (b->h_status) (void)hipHostFree(b->h_status);
  if (b->d_ws) (void)hipFree(b->d_ws);
  delete b;
}

bht_status bht_batch_build_find(const bht_batch_entry* entries, uint32_t count, uint32_t item_size,
                                bht_status* status_out, void* stream) {
  bht_batch* b = nullptr;
  bht_status s = bht_batch_create(entries, count, item_size, &b);
  if (s != BHT_OK) return s;
  for (bht_table* t : b->tables) {
    t->built = false;
    t->counted_build_probes = 0;
  }
  // one pass: the kernels go straight onto the stream, no graph is captured
  s = batch_launch(b, as_stream(stream));
  if (s == BHT_OK) s = bht_batch_wait(b, stream, status_out);
  else (void)hipStreamSynchronize(as_stream(stream));
  bht_batch_destroy(b);
  return s;
}

bht_status bht_find_ctx_create(uint32_t max_requests, uint64_t max_items, bht_find_ctx** out) {
  if (!out || max_requests == 0 || max_items == 0) return fail(BHT_ERR_INVALID_ARG, "bad argument");
  *out = nullptr;
  bht_find_ctx* c = new bht_find_ctx();
  c->max_requests = max_requests;
  c->max_items = max_items;
  hipError_t e = hipMalloc(&c->d_tables, sizeof(BatchTable) * max_requests);
  if (e == hipSuccess) e = hipMalloc(&c->d_items, sizeof(BatchItem) * max_items);
  if (e == hipSuccess) e = hipMalloc(&c->d_heads, 16);
  if (e == hipSuccess)
    e = hipHostMalloc(&c->h_tables, sizeof(BatchTable) * max_requests, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(&c->h_items, sizeof(BatchItem) * max_items, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming);
  if (e != hipSuccess) {
    bht_find_ctx_destroy(c);
    return fail(BHT_ERR_OOM, std::string("find context: ") + hipGetErrorString(e));
  }
  *out = c;
  return BHT_OK;
}

bht_status bht_multi_find(bht_find_ctx* c, const bht_find_request* reqs, uint32_t count,
                          uint32_t item_size, void* stream) {
  if (!c || (!reqs && count)) return fail(BHT_ERR_INVALID_ARG, "null argument");
  if (count == 0) return BHT_OK;
  if (count > c->max_requests) return fail(BHT_ERR_CAPACITY, "more requests than the context holds");
  if (item_size == 0) item_size = 8192;
  if (item_size < 64) return fail(BHT_ERR_INVALID_ARG, "item_size must be at least 64");
  const bht_table* t0 = reqs[0].table;
  if (!t0) return fail(BHT_ERR_INVALID_ARG, "null table");
  uint64_t items = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const bht_find_request& r = reqs[i];
    const bht_table* t = r.table;
    if (!t) return fail(BHT_ERR_INVALID_ARG, "null table in request");
    if (!t->built) return fail(BHT_ERR_NOT_BUILT, "request on a table that is not built");
    if (t->scheme != BHT_BCHT || t->key_bits != 32 || t->b != t0->b || t->tile != t0->tile)
      return fail(BHT_ERR_UNSUPPORTED, "requests of one call share a 32-bit BCHT configuration");
    if (r.n && (!r.d_queries || !r.d_out_values || !r.d_out_found))
      return fail(BHT_ERR_INVALID_ARG, "null data pointer in request");
    items += (r.n + item_size - 1) / item_size;
  }
  if (items > c->max_items) return fail(BHT_ERR_CAPACITY, "more work items than the context holds");
  const void* fk = nullptr;
  const void* ik = nullptr;
#define BHT_MF_CASE(B_, W_)                              \
  if (t0->b == B_ && t0->tile == W_) {                   \
    fk = (const void*)batch_find_kernel<B_, W_>;         \
    ik = (const void*)inline_find_kernel<B_, W_>;        \
  }
  BHT_MF_CASE(8, 4)
  BHT_MF_CASE(8, 8)
  BHT_MF_CASE(16, 4)
  BHT_MF_CASE(16, 8)
  BHT_MF_CASE(16, 16)
  BHT_MF_CASE(32, 8)
  BHT_MF_CASE(32, 16)
#undef BHT_MF_CASE
  if (!fk) return fail(BHT_ERR_UNSUPPORTED, "no query kernel for this bucket size and tile");
  if (count <= (uint32_t)kInlineRequests && items <= 0xFFFFFFFFull) {
    // Spread a small launch over the resident waves: shrink the item (down
    // to one 64-query chunk) until every wave has about one item.
    uint64_t total_q = 0;
    for (uint32_t i = 0; i < count; ++i) total_q += reqs[i].n;
    const uint64_t waves = (uint64_t)grid_for(ik, 1ull << 40) * (kBlock / 64);
    const uint64_t even = ((total_q + waves - 1) / waves + 63) / 64 * 64;
    item_size = (uint32_t)std::max<uint64_t>(64, std::min<uint64_t>(item_size, even));
    InlineFind arg;
    memset(&arg, 0, sizeof(arg));
    uint32_t first = 0;
    for (uint32_t i = 0; i < count; ++i) {
      const bht_find_request& r = reqs[i];
      FindTable& T = arg.t[i];
      T.slots = r.table->d_slots;
      T.queries = r.d_queries;
      T.out_v = r.d_out_values;
      T.out_f = r.d_out_found;
      T.n = r.n;
      T.H = make_hash32(r.table->params, r.table->m, r.table->params.num_hashes);
      arg.first_item[i] = first;
      first += (uint32_t)((r.n + item_size - 1) / item_size);
    }
    arg.first_item[count] = first;
    arg.count = count;
    arg.item_size = item_size;
    if (first == 0) return BHT_OK;
    const int grid = grid_for(ik, (uint64_t)first * kBlock);
    reinterpret_cast<void (*)(InlineFind)>(const_cast<void*>(ik))
        <<<grid, kBlock, 0, as_stream(stream)>>>(arg);
    HIP_TRY(hipGetLastError());
    return BHT_OK;
  }
  hipStream_t st = as_stream(stream);
  // the previous call's copies out of the staging buffers must be finished
  if (c->used) HIP_TRY(hipEventSynchronize(c->staged));
  uint64_t k = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const bht_find_request& r = reqs[i];
    BatchTable& T = c->h_tables[i];
    memset(&T, 0, sizeof(T));
    T.slots = r.table->d_slots;
    T.words = r.table->words;
    T.queries = r.d_queries;
    T.out_v = r.d_out_values;
    T.out_f = r.d_out_found;
    T.n_queries = r.n;
    T.H = make_hash32(r.table->params, r.table->m, r.table->params.num_hashes);
    for (uint64_t s = 0; s < r.n; s += item_size)
      c->h_items[k++] = {i, 0, s, std::min<uint64_t>(item_size, r.n - s)};
  }
  HIP_TRY(hipMemcpyAsync(c->d_tables, c->h_tables, sizeof(BatchTable) * count,
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(c->d_items, c->h_items, sizeof(BatchItem) * k, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(c->staged, st));
  c->used = true;
  batch_reset_kernel<<<1, 64, 0, st>>>(c->d_heads, nullptr, 0);
  HIP_TRY(hipGetLastError());
  const int grid = grid_for(fk, k * kBlock);
  reinterpret_cast<void (*)(const BatchTable*, const BatchItem*, uint64_t, unsigned int*)>(
      const_cast<void*>(fk))<<<grid, kBlock, 0, st>>>(c->d_tables, c->d_items, k, c->d_heads);
  HIP_TRY(hipGetLastError());
  return BHT_OK;
}

void bht_find_ctx_destroy(bht_find_ctx* c) {
  if (!c) return;
  if (c->used) (void)hipEventSynchronize(c->staged);
  if (c->staged) (void)hipEventDestroy(c->staged);
  if (c->d_tables) (void)hipFree(c->d_tables);
  if (c->d_items) (void)hipFree(c->d_items);
  if (c->d_heads) (void)hipFree(c->d_heads);
  if (c->h_tables) (void)hipHostFree(c->h_tables);
  if (c->h_items) (void)hipHostFree(c->h_items);
  delete c;
}

}  // extern "C"
