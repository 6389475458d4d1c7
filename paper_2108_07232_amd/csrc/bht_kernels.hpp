// Device kernels for static bucketed hash tables on gfx950 (wave64).
//
// Execution model.  Every lane of a wave owns one operation (an insertion
// or a query) at a time and keeps its state in registers.  The wave is cut
// into tiles of W lanes; a tile reads the buckets its lanes need
// cooperatively, lane t of the tile loading slots [t*S, (t+1)*S) of the
// bucket (S = B / W), so that one 128-byte bucket is one coalesced request
// (Section V-A: a bucket no larger than a cache line costs one memory
// transaction).  The tile inspects the loaded buckets of all its lanes in
// turn with ballots (Listing 2: load = population count of non-empty slots,
// a match = first lane whose key equals the query), and then each lane
// issues its own atomic.  A lane that finishes takes the next item of the
// wave's contiguous input range, so every loop iteration keeps up to 64
// independent bucket reads in flight per wave; this replaces the paper's
// per-tile serial work queue (Listing 1) whose single operation in flight
// per tile leaves HBM latency exposed.
//
// Insertion is driven by atomic return values only.  Bucket reads are
// ordinary loads that may return a stale copy of a line another XCD's L2
// has since changed; a stale copy can only under-report occupancy, because
// slots are never emptied during a build.  A lane therefore CASes at slot =
// load and, when that CAS fails (the slot is taken), at the next slot,
// without re-reading: occupied slots stay a prefix of the bucket (each
// successful CAS is at the first empty slot), and reaching the end of the
// bucket proves it full.  A full bucket is handled with an unconditional
// atomic exchange at a random slot (Section V-B), whose returned pair is the
// evicted one.  No step waits on another lane, so a build always terminates:
// at most b CAS attempts per bucket visit and max_chain evictions per key.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bht_hash.hpp"

namespace bht {

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
constexpr uint64_t kEmptyPair = ~0ull;
constexpr uint64_t kEmpty64 = ~0ull;
enum : uint32_t { kFlagFailed = 1u, kFlagSentinel = 2u };
constexpr int kBlock = 256;

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Value of v in lane src (any lane of the wave), via the LDS crossbar.
__device__ __forceinline__ uint32_t shfl32(uint32_t v, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)v);
}

__device__ __forceinline__ uint32_t xorshift32(uint32_t x) {
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}

__device__ __forceinline__ uint64_t cas64(uint64_t* p, uint64_t expected, uint64_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return expected;
}

__device__ __forceinline__ uint64_t xchg64(uint64_t* p, uint64_t v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T sel4(const T* a, uint32_t i) {
  return i == 0 ? a[0] : i == 1 ? a[1] : i == 2 ? a[2] : a[3];
}

// Bucket index of hash i (i varies per lane) without dynamic indexing.
__device__ __forceinline__ uint32_t hash32_dyn(const Hash32& H, uint32_t i, uint32_t k) {
  return hash32(sel4(H.a, i), sel4(H.c, i), k, H.M, H.m);
}

// Cuckoo rule (Section III-A footnote): the evicted key continues with the
// hash after the lowest-index hash that names the bucket it left.
__device__ __forceinline__ uint32_t next_bucket(const Hash32& H, uint32_t key, uint32_t left) {
  uint32_t hv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) hv[i] = (i < (int)H.h) ? hash32(H, i, key) : 0u;
  uint32_t nxt = hv[0];
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    if (i < (int)H.h && hv[i] == left) nxt = (i + 1 < (int)H.h) ? hv[i + 1] : hv[0];
  }
  return nxt;
}

// ---------------------------------------------------------- bucket slices

template <int S>
struct Part {
  uint64_t s[S];
};

// The same words read with device-scope atomic loads, which skip copies of
// the line that this XCD's caches may hold from before another XCD's
// update (load-balanced placements decide on these values).
template <int S>
__device__ __forceinline__ Part<S> load_part_fresh(const uint64_t* p) {
  Part<S> r;
#pragma unroll
  for (int i = 0; i < S; ++i) r.s[i] = __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return r;
}

template <int S>
__device__ __forceinline__ Part<S> load_part(const uint64_t* p) {
  Part<S> r;
  if constexpr (S == 1) {
    r.s[0] = *p;
  } else {
#pragma unroll
    for (int i = 0; i < S / 2; ++i) {
      u64x2 v = reinterpret_cast<const u64x2*>(p)[i];
      r.s[2 * i] = v.x;
      r.s[2 * i + 1] = v.y;
    }
  }
  return r;
}

template <int S>
__device__ __forceinline__ Part<S> empty_part() {
  Part<S> r;
#pragma unroll
  for (int i = 0; i < S; ++i) r.s[i] = kEmptyPair;
  return r;
}

template <int W>
__device__ __forceinline__ uint64_t tile_bits(uint64_t mask, uint32_t tile_base) {
  if constexpr (W == 64) return mask;
  else return (mask >> tile_base) & ((1ull << W) - 1);
}

// Wave-contiguous share of n items: wave w gets [w*per, (w+1)*per).
struct Range {
  uint64_t cursor, end;
};

__device__ __forceinline__ Range wave_range(uint64_t n) {
  const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t wave = gtid >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t per = (n + nwaves - 1) / nwaves;
  Range r;
  r.cursor = wave * per < n ? wave * per : n;
  r.end = r.cursor + per < n ? r.cursor + per : n;
  return r;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ------------------------------------------------------------------ fill

// Section III: every bucket starts empty.  Also clears the build status.
__global__ void fill_empty_kernel(uint64_t* __restrict__ slots, uint64_t words,
                                  uint32_t* __restrict__ status) {
  const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  if (gtid < 4 && status) status[gtid] = 0;
  const u64x2 e = {kEmptyPair, kEmptyPair};
  u64x2* p2 = reinterpret_cast<u64x2*>(slots);
  for (uint64_t i = gtid; i < words / 2; i += stride) p2[i] = e;
  if ((words & 1) && gtid == 0) slots[words - 1] = kEmptyPair;
}

// Adds the per-query probe counts of an instrumented find to a 64-bit total
// (one block-wide sum, then one atomic per block).
__global__ void probe_sum_kernel(const uint8_t* __restrict__ probes, uint64_t n,
                                 unsigned long long* __restrict__ total) {
  __shared__ unsigned long long part[kBlock / 64];
  unsigned long long sum = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    sum += probes[i];
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
    if (t) atomicAdd(total, t);
  }
}

// ----------------------------------------------------------- input feed

// A wave consumes its range in order.  Lane i holds item base+i of chunk A
// and item base+64+i of chunk B in registers; lanes that need work take the
// next items by rank (one crossbar read each) and, once chunk A is used up,
// chunk B becomes A and the following chunk is loaded.  That load is needed
// one chunk later, so refilling a lane never waits on memory.
template <typename T>
struct Feed {
  const T* src;
  uint64_t base, cursor, end;
  T a, b;

  __device__ __forceinline__ void init(const T* s, Range r, T fill) {
    const uint32_t lane = __lane_id();
    src = s;
    base = cursor = r.cursor;
    end = r.end;
    a = (base + lane < end) ? src[base + lane] : fill;
    b = (base + 64 + lane < end) ? src[base + 64 + lane] : fill;
  }

  // Offset of this lane's new item within the two chunks, or -1 if none.
  __device__ __forceinline__ int64_t claim(bool need, uint64_t* idx) {
    const uint64_t nm = ballot(need);
    const uint64_t take = cursor + lanes_below(nm);
    *idx = take;
    const uint64_t taken = (uint64_t)__popcll(nm);
    const int64_t off = (need && take < end) ? (int64_t)(take - base) : -1;
    last_reads_b = cursor + taken > base + 64;
    cursor = cursor + taken < end ? cursor + taken : end;
    return off;
  }

  __device__ __forceinline__ T value_at(int64_t off) const {
    const uint32_t src_lane = (uint32_t)off & 63u;
    T x = (T)shfl32((uint32_t)a, src_lane);
    if (last_reads_b) {  // wave-uniform: some lane reads chunk B
      const T y = (T)shfl32((uint32_t)b, src_lane);
      if (off >= 64) x = y;
    }
    return x;
  }

  // After every value_at of this round: retire chunk A once it is used up.
  __device__ __forceinline__ void advance(T fill) {
    if (cursor >= base + 64) {
      const uint32_t lane = __lane_id();
      base += 64;
      a = b;
      b = (base + 64 + lane < end) ? src[base + 64 + lane] : fill;
    }
  }

  bool last_reads_b = false;
};

// Tile-cooperative read of the buckets of the lanes in `mask`: slice j holds
// this lane's part (slots [lt*S, lt*S+S)) of the bucket of tile lane j.
template <int B, int W>
__device__ __forceinline__ void tile_read(const uint64_t* __restrict__ slots, uint32_t bucket,
                                          uint64_t mask, uint32_t tb, uint32_t lt,
                                          Part<B / W> (&d)[W]) {
  constexpr int S = B / W;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const uint32_t bj = shfl32(bucket, tb + j);
    if ((mask >> (tb + j)) & 1ull) d[j] = load_part<S>(slots + (uint64_t)bj * B + lt * S);
    else d[j] = empty_part<S>();
  }
}

// Listing 2 for the bucket of every tile lane j: hit = some slot holds q_j
// (value = that slot's value), room = some slot is empty.  Each lane gets
// the answer for its own bucket.
template <int B, int W>
__device__ __forceinline__ void tile_match(const Part<B / W> (&d)[W], uint32_t q, uint32_t tb,
                                           uint32_t lt, bool* hit, bool* room, uint32_t* value) {
  constexpr int S = B / W;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const uint32_t qj = shfl32(q, tb + j);
    bool m = false, e = false;
    uint32_t vsel = kEmptyKey;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t k = (uint32_t)d[j].s[s];
      if (k == qj) {
        m = true;
        vsel = (uint32_t)(d[j].s[s] >> 32);
      }
      e |= (k == kEmptyKey);
    }
    const uint64_t hm = tile_bits<W>(ballot(m), tb);
    const uint64_t em = tile_bits<W>(ballot(e), tb);
    const uint32_t src = tb + (hm ? (uint32_t)__builtin_ctzll(hm) : 0u);
    const uint32_t v = shfl32(vsel, src);
    if (lt == (uint32_t)j) {
      *hit = hm != 0;
      *room = em != 0;
      *value = v;
    }
  }
}

// Listing 2 compute_load for the bucket of every tile lane j.
template <int B, int W>
__device__ __forceinline__ uint32_t tile_load(const Part<B / W> (&d)[W], uint32_t tb, uint32_t lt) {
  constexpr int S = B / W;
  uint32_t load = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    uint32_t cnt = 0;
#pragma unroll
    for (int s = 0; s < S; ++s)
      cnt += __popcll(tile_bits<W>(ballot((uint32_t)d[j].s[s] != kEmptyKey), tb));
    if (lt == (uint32_t)j) load = cnt;
  }
  return load;
}

// ------------------------------------------------------- cuckoo (BCHT)

struct BuildArgs32 {
  uint64_t* slots;
  const uint32_t* keys;
  const uint32_t* vals;
  uint64_t n;
  uint32_t* status;
  unsigned long long* probe_total;
  Hash32 H;
  uint32_t max_chain;
  uint32_t rng_seed;
};

struct FindArgs32 {
  const uint64_t* slots;
  const uint32_t* queries;
  uint64_t n;
  uint32_t* out_v;
  uint8_t* out_f;
  uint8_t* probes;
  Hash32 H;
};

enum : uint32_t { kRead = 0, kWalk = 1, kEvict = 2 };

// Bucketed cuckoo insertion (Section III-A, Section V-B) of the pairs in
// range r by the calling wave.  Returns the status flags this lane raised;
// *probes accumulates the lane's bucket reads when COUNT.  EVICTED: every
// pair of the range was just evicted from its first bucket (one exchange
// already made), so it continues at the next bucket of the cuckoo rule with
// one exchange counted.
template <int B, int W, bool COUNT, bool EVICTED = false>
__device__ __forceinline__ uint32_t cuckoo_build_range(const BuildArgs32& g, Range r,
                                                       uint32_t rng, uint32_t* probes_out) {
  const uint32_t lane = __lane_id();
  const uint32_t tb = lane & ~(uint32_t)(W - 1);
  const uint32_t lt = lane & (uint32_t)(W - 1);
  if (rng == 0) rng = 0x2545F491u;

  Feed<uint32_t> fk, fv;
  fk.init(g.keys, r, kEmptyKey);
  fv.init(g.vals, r, 0u);
  bool active = false;
  uint32_t key = 0, val = 0, bucket = 0, chain = 0, slot = 0, phase = kRead;
  uint32_t probes = 0, flags = 0;

  for (;;) {
    uint64_t idx;
    const int64_t off = fk.claim(!active, &idx);
    fv.claim(!active, &idx);
    const uint32_t k_new = fk.value_at(off);
    const uint32_t v_new = fv.value_at(off);
    fk.advance(kEmptyKey);
    fv.advance(0u);
    if (off >= 0) {
      if (k_new == kEmptyKey) {
        flags |= kFlagSentinel;
      } else {
        active = true;
        key = k_new;
        val = v_new;
        bucket = hash32(g.H, 0, key);
        chain = 0;
        if (EVICTED) {
          bucket = next_bucket(g.H, key, bucket);
          chain = 1;
        }
        phase = kRead;
      }
    }
    if (ballot(active) == 0) {
      if (fk.cursor >= fk.end) break;
      continue;
    }

    Part<B / W> d[W];
    tile_read<B, W>(g.slots, bucket, ballot(active && phase == kRead), tb, lt, d);
    const uint32_t load = tile_load<B, W>(d, tb, lt);

    if (active && phase == kRead) {
      if (COUNT) ++probes;
      if (load < (uint32_t)B) {
        phase = kWalk;
        slot = load;
      } else {
        phase = kEvict;
      }
    }
    const uint64_t pair = ((uint64_t)val << 32) | key;
    if (active && phase == kWalk) {
      const uint64_t old = cas64(g.slots + (uint64_t)bucket * B + slot, kEmptyPair, pair);
      if (old == kEmptyPair) active = false;
      else if (++slot == (uint32_t)B) phase = kEvict;
    } else if (active && phase == kEvict) {
      if (chain >= g.max_chain) {
        flags |= kFlagFailed;
        active = false;
      } else {
        rng = xorshift32(rng);
        const uint64_t old = xchg64(g.slots + (uint64_t)bucket * B + (rng % (uint32_t)B), pair);
        if (old == kEmptyPair) {
          active = false;
        } else {
          key = (uint32_t)old;
          val = (uint32_t)(old >> 32);
          bucket = next_bucket(g.H, key, bucket);
          ++chain;
          phase = kRead;
        }
      }
    }
  }
  if (COUNT) *probes_out += probes;
  return flags;
}

// Lane salt for the eviction generator: distinct per lane of the launch.
__device__ __forceinline__ uint32_t lane_salt() {
  const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  return (uint32_t)(gtid * 0x9E3779B9ull) ^ (uint32_t)(gtid >> 32);
}

template <int B, int W, bool COUNT>
__global__ __launch_bounds__(kBlock) void cuckoo_build_kernel(BuildArgs32 g) {
  uint32_t probes = 0;
  const uint32_t flags =
      cuckoo_build_range<B, W, COUNT>(g, wave_range(g.n), g.rng_seed ^ lane_salt(), &probes);
  if (flags) atomicOr(g.status, flags);
  if (COUNT) {
    const uint32_t total = wave_sum(probes);
    if (__lane_id() == 0 && total) atomicAdd(g.probe_total, (unsigned long long)total);
  }
}

// Bucketed cuckoo query (Section V-B): probe H0, H1, ... in order; stop on a
// hit, or with a miss after a bucket that lacks the key and has room.
// Lanes that finish take new queries from the feed (refill schedule).
template <int B, int W, bool COUNT>
__global__ __launch_bounds__(kBlock) void cuckoo_find_kernel(FindArgs32 g) {
  const uint32_t lane = __lane_id();
  const uint32_t tb = lane & ~(uint32_t)(W - 1);
  const uint32_t lt = lane & (uint32_t)(W - 1);
  const Range r = wave_range(g.n);

  Feed<uint32_t> fq;
  fq.init(g.queries, r, kEmptyKey);
  bool active = false;
  uint64_t idx = 0;
  uint32_t q = 0, round = 0, bucket = 0;

  for (;;) {
    uint64_t take;
    const int64_t off = fq.claim(!active, &take);
    const uint32_t q_new = fq.value_at(off);
    fq.advance(kEmptyKey);
    if (off >= 0) {
      idx = take;
      q = q_new;
      if (q == kEmptyKey) {
        g.out_v[idx] = kEmptyKey;
        g.out_f[idx] = 0;
        if (COUNT) g.probes[idx] = 0;
      } else {
        active = true;
        round = 0;
        bucket = hash32(g.H, 0, q);
      }
    }
    const uint64_t act = ballot(active);
    if (act == 0) {
      if (fq.cursor >= fq.end) break;
      continue;
    }

    Part<B / W> d[W];
    tile_read<B, W>(g.slots, bucket, act, tb, lt, d);
    bool hit = false, room = false;
    uint32_t value = kEmptyKey;
    tile_match<B, W>(d, q, tb, lt, &hit, &room, &value);
    if (active) {
      bool done = true;
      if (hit) {
        g.out_v[idx] = value;
        g.out_f[idx] = 1;
      } else if (room || round + 1 >= g.H.h) {
        g.out_v[idx] = kEmptyKey;
        g.out_f[idx] = 0;
      } else {
        done = false;
      }
      if (done) {
        if (COUNT) g.probes[idx] = (uint8_t)(round + 1);
        active = false;
      } else {
        ++round;
        bucket = hash32_dyn(g.H, round, q);
      }
    }
  }
}

// Same query, chunk schedule: a wave answers Q*64 consecutive queries per
// chunk (Q per lane) in up to h rounds (round i probes H_i for the queries
// still open), then writes the results with coalesced stores; the next
// chunk's queries are loaded while the current chunk is probed.  Q > 1 puts
// more bucket reads in flight per wave in the first round.
template <int B, int W, bool COUNT, int Q = 1>
__device__ __forceinline__ void cuckoo_find_chunk_range(const FindArgs32& g, Range r) {
  const uint32_t lane = __lane_id();
  const uint32_t tb = lane & ~(uint32_t)(W - 1);
  const uint32_t lt = lane & (uint32_t)(W - 1);
  constexpr uint32_t C = 64 * Q;
  uint32_t q_next[Q];
#pragma unroll
  for (int u = 0; u < Q; ++u)
    q_next[u] = (r.cursor + u * 64 + lane < r.end) ? g.queries[r.cursor + u * 64 + lane] : kEmptyKey;
  for (uint64_t base = r.cursor; base < r.end; base += C) {
    uint32_t q[Q], out[Q], rounds[Q];
    bool open[Q], valid[Q];
    uint8_t found[Q];
#pragma unroll
    for (int u = 0; u < Q; ++u) {
      const uint64_t idx = base + u * 64 + lane;
      valid[u] = idx < r.end;
      q[u] = q_next[u];
      q_next[u] = (base + C + u * 64 + lane < r.end) ? g.queries[base + C + u * 64 + lane]
                                                     : kEmptyKey;
      open[u] = valid[u] && q[u] != kEmptyKey;
      out[u] = kEmptyKey;
      rounds[u] = 0;
      found[u] = 0;
    }
    for (uint32_t round = 0; round < g.H.h; ++round) {
      uint64_t om[Q], any = 0;
#pragma unroll
      for (int u = 0; u < Q; ++u) {
        om[u] = ballot(open[u]);
        any |= om[u];
      }
      if (any == 0) break;
      Part<B / W> d[Q][W];
#pragma unroll
      for (int u = 0; u < Q; ++u) {
        const uint32_t bucket = open[u] ? hash32_dyn(g.H, round, q[u]) : 0u;
        tile_read<B, W>(g.slots, bucket, om[u], tb, lt, d[u]);
      }
#pragma unroll
      for (int u = 0; u < Q; ++u) {
        bool hit = false, room = false;
        uint32_t value = kEmptyKey;
        tile_match<B, W>(d[u], q[u], tb, lt, &hit, &room, &value);
        if (open[u]) {
          rounds[u] = round + 1;
          if (hit) {
            out[u] = value;
            found[u] = 1;
            open[u] = false;
          } else if (room) {
            open[u] = false;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < Q; ++u) {
      if (valid[u]) {
        const uint64_t idx = base + u * 64 + lane;
        g.out_v[idx] = out[u];
        g.out_f[idx] = found[u];
        if (COUNT) g.probes[idx] = (uint8_t)rounds[u];
      }
    }
  }
}

template <int B, int W, bool COUNT, int Q = 1>
__global__ __launch_bounds__(kBlock) void cuckoo_find_chunk_kernel(FindArgs32 g) {
  cuckoo_find_chunk_range<B, W, COUNT, Q>(g, wave_range(g.n));
}

// Parallel probing (the alternative noted in Section II-A): all h candidate
// buckets of a query are read at once, so a query costs one memory latency
// instead of up to h dependent ones, at h probes per query.  A stored key
// sits in exactly one bucket, so the first hit in hash order is the answer.
// Chunk schedule as above.
template <int B, int W, bool COUNT>
__global__ __launch_bounds__(kBlock) void cuckoo_find_parallel_kernel(FindArgs32 g) {
  const uint32_t lane = __lane_id();
  const uint32_t tb = lane & ~(uint32_t)(W - 1);
  const uint32_t lt = lane & (uint32_t)(W - 1);
  const Range r = wave_range(g.n);
  uint32_t q_next = (r.cursor + lane < r.end) ? g.queries[r.cursor + lane] : kEmptyKey;
  for (uint64_t base = r.cursor; base < r.end; base += 64) {
    const uint64_t idx = base + lane;
    const bool valid = idx < r.end;
    const uint32_t q = q_next;
    q_next = (base + 64 + lane < r.end) ? g.queries[base + 64 + lane] : kEmptyKey;
    const bool open = valid && q != kEmptyKey;
    const uint64_t om = ballot(open);
    Part<B / W> d[4][W];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i < (int)g.H.h) {
        const uint32_t bucket = open ? hash32(g.H, i, q) : 0u;
        tile_read<B, W>(g.slots, bucket, om, tb, lt, d[i]);
      }
    }
    uint32_t out = kEmptyKey;
    uint8_t found = 0;
#pragma unroll
    for (int i = 3; i >= 0; --i) {
      if (i < (int)g.H.h) {
        bool hit = false, room = false;
        uint32_t value = kEmptyKey;
        tile_match<B, W>(d[i], q, tb, lt, &hit, &room, &value);
        if (open && hit) {
          out = value;
          found = 1;
        }
      }
    }
    if (valid) {
      g.out_v[idx] = out;
      g.out_f[idx] = found;
      if (COUNT) g.probes[idx] = open ? (uint8_t)g.H.h : (uint8_t)0;
    }
  }
}

}  // namespace bht
