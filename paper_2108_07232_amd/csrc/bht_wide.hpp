// Bucketed cuckoo table with 64-bit keys and 64-bit values: 16-byte slots,
// 8 slots per 128-byte bucket (not in the paper, whose pairs fit one 64-bit
// atomic, Section II-A).
//
// gfx950 has no 128-bit compare-and-swap, so a slot changes hands through
// its key word, used as a lock: the reserved key BUSY marks a slot whose
// value word is being replaced.  Every step is a device-scope atomic
// (compare-and-swap or exchange with a return value, or a device-scope
// store, which is written through to the level where those atomics are
// performed), and the lane waits for each one to complete before issuing
// the next, so the steps of one slot are ordered without cache-wide release
// or acquire fences:
//   claim an empty slot:  CAS key EMPTY -> BUSY, store value, store key k
//   evict a resident:     CAS key k' -> BUSY, exchange value (returns v'),
//                         store key k, carry (k', v')
// Only the lane whose CAS set BUSY writes the slot until its key store
// releases it, so the releasing stores need no read-modify-write; the two
// words of a slot also share one cache line and so one memory channel.  A
// lane whose CAS takes the slot from key k has seen the key store of k's
// writer, which was issued after that writer's value store completed, so
// its value exchange returns k's value.  A slot is BUSY only inside one loop
// iteration of its owner, so a lane that meets BUSY retries on a later
// iteration; a per-pair attempt cap turns any unforeseen starvation into a
// reported build failure instead of a hang.  Queries run in a later launch
// and never see BUSY.
#pragma once
#include "bht_kernels.hpp"

namespace bht {

constexpr uint64_t kBusy64 = ~0ull - 1;
constexpr uint32_t kWideAttemptCap = 1u << 14;

__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ uint64_t shfl64(uint64_t v, uint32_t src) {
  const uint32_t lo = shfl32((uint32_t)v, src);
  const uint32_t hi = shfl32((uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t load_key_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave feed of 64-bit items (same scheme as Feed<uint32_t>).
struct Feed64 {
  const uint64_t* src;
  uint64_t base, cursor, end;
  uint64_t a, b;
  bool last_reads_b = false;

  __device__ __forceinline__ void init(const uint64_t* s, Range r, uint64_t fill) {
    const uint32_t lane = __lane_id();
    src = s;
    base = cursor = r.cursor;
    end = r.end;
    a = (base + lane < end) ? src[base + lane] : fill;
    b = (base + 64 + lane < end) ? src[base + 64 + lane] : fill;
  }
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
  __device__ __forceinline__ uint64_t value_at(int64_t off) const {
    const uint32_t src_lane = (uint32_t)off & 63u;
    uint64_t x = shfl64(a, src_lane);
    if (last_reads_b) {
      const uint64_t y = shfl64(b, src_lane);
      if (off >= 64) x = y;
    }
    return x;
  }
  __device__ __forceinline__ void advance(uint64_t fill) {
    if (cursor >= base + 64) {
      const uint32_t lane = __lane_id();
      base += 64;
      a = b;
      b = (base + 64 + lane < end) ? src[base + 64 + lane] : fill;
    }
  }
};

struct WideBuildArgs {
  uint64_t* slots;             // 2 words per slot: key, value
  const uint64_t* keys;
  const uint64_t* vals;
  uint64_t n;
  uint32_t* status;
  Hash64 H;
  uint32_t max_chain;
  uint32_t rng_seed;
};

struct WideFindArgs {
  const uint64_t* slots;
  const uint64_t* queries;
  uint64_t n;
  uint64_t* out_v;
  uint8_t* out_f;
  uint8_t* probes;             // per-query bucket reads (COUNT kernels)
  Hash64 H;
};

__device__ __forceinline__ uint32_t next_bucket64(const Hash64& H, uint64_t key, uint32_t left) {
  uint32_t hv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) hv[i] = (i < (int)H.h) ? (uint32_t)hash64(H, i, key) : 0u;
  uint32_t nxt = hv[0];
#pragma unroll
  for (int i = 3; i >= 0; --i)
    if (i < (int)H.h && hv[i] == left) nxt = (i + 1 < (int)H.h) ? hv[i + 1] : hv[0];
  return nxt;
}

enum : uint32_t { kWRead = 0, kWWalk = 1, kWEvict = 2 };

// Inserts the pairs [r.cursor, r.end) of g.keys / g.vals (one wave's range;
// the whole wave calls it).  W lanes per tile, one 16-byte slot per lane:
// B = W = 8 slots per bucket.  EVICTED: each pair was evicted from its
// first bucket H_0 (one exchange made) and continues at the next one.
// Bucket reads are added to *probes; returns the lane's status flags.
template <int W, bool EVICTED>
__device__ __forceinline__ uint32_t wide_build_range(const WideBuildArgs& g, Range r, uint32_t rng,
                                                     uint32_t* probes) {
  constexpr int B = W;
  const uint32_t lane = __lane_id();
  const uint32_t tb = lane & ~(uint32_t)(W - 1);
  const uint32_t lt = lane & (uint32_t)(W - 1);
  if (rng == 0) rng = 0x2545F491u;

  Feed64 fk, fv;
  fk.init(g.keys, r, kEmpty64);
  fv.init(g.vals, r, 0ull);
  bool active = false;
  uint64_t key = 0, val = 0, expect = 0;
  uint32_t bucket = 0, chain = 0, slot = 0, phase = kWRead, attempts = 0, flags = 0;

  for (;;) {
    uint64_t idx;
    const int64_t off = fk.claim(!active, &idx);
    fv.claim(!active, &idx);
    const uint64_t k_new = fk.value_at(off);
    const uint64_t v_new = fv.value_at(off);
    fk.advance(kEmpty64);
    fv.advance(0ull);
    if (off >= 0) {
      if (k_new >= kBusy64) {
        flags |= kFlagSentinel;
      } else {
        active = true;
        key = k_new;
        val = v_new;
        bucket = (uint32_t)hash64(g.H, 0, key);
        chain = 0;
        if constexpr (EVICTED) {
          bucket = next_bucket64(g.H, key, bucket);
          chain = 1;
        }
        attempts = 0;
        phase = kWRead;
      }
    }
    if (ballot(active) == 0) {
      if (fk.cursor >= fk.end) break;
      continue;
    }

    // Tile read: lane lt loads slot lt (key and value) of each bucket.
    const uint64_t rd = ballot(active && phase == kWRead);
    *probes += (uint32_t)((rd >> lane) & 1ull);
    uint64_t dk[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const uint32_t bj = shfl32(bucket, tb + j);
      dk[j] = kEmpty64;
      if ((rd >> (tb + j)) & 1ull) dk[j] = g.slots[2 * ((uint64_t)bj * B + lt)];
    }
    uint32_t load = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const uint32_t cnt = __popcll(tile_bits<W>(ballot(dk[j] != kEmpty64), tb));
      if (lt == (uint32_t)j) load = cnt;
    }
    // victim slot and the key seen there, for lanes about to evict
    if (active && phase == kWRead) {
      if (load < (uint32_t)B) {
        phase = kWWalk;
        slot = load;
      } else {
        phase = kWEvict;
        rng = xorshift32(rng);
        slot = rng % (uint32_t)B;
      }
    }
    uint64_t seen = kEmpty64;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      // key of slot `slot` of lane j's bucket is held by tile lane `slot`
      const uint32_t sj = shfl32(slot, tb + j);
      const uint64_t kj = shfl64(dk[j], tb + sj);
      if (lt == (uint32_t)j && (rd >> lane) & 1ull) seen = kj;
    }
    if (active && ((rd >> lane) & 1ull) && phase == kWEvict) expect = seen;

    if (active && ++attempts > kWideAttemptCap) {
      flags |= kFlagFailed;
      active = false;
    }
    uint64_t* const sk = g.slots + 2 * ((uint64_t)bucket * B + slot);
    if (active && phase == kWWalk) {
      const uint64_t c = cas64(sk, kEmpty64, kBusy64);
      if (c == kEmpty64) {
        wait_memory();
        store_agent(sk + 1, val);
        wait_memory();
        store_agent(sk, key);
        active = false;
      } else if (++slot == (uint32_t)B) {
        // every slot is taken: evict at a random slot whose key is learned
        // with a coherent load on the next iteration
        phase = kWEvict;
        rng = xorshift32(rng);
        slot = rng % (uint32_t)B;
        expect = kBusy64;
      }
    } else if (active && phase == kWEvict) {
      if (chain >= g.max_chain) {
        flags |= kFlagFailed;
        active = false;
      } else if (expect == kEmpty64) {
        phase = kWWalk;                       // the victim slot is free after all
      } else if (expect == kBusy64) {
        expect = load_key_agent(sk);          // learn the slot's key for the next try
      } else {
        const uint64_t c = cas64(sk, expect, kBusy64);
        if (c == expect) {
          wait_memory();
          const uint64_t old_v = xchg64(sk + 1, val);
          wait_memory();
          store_agent(sk, key);
          key = expect;
          val = old_v;
          bucket = next_bucket64(g.H, key, bucket);
          ++chain;
          phase = kWRead;
        } else {
          expect = c;                          // retry with the current key
        }
      }
    }
  }
  return flags;
}

template <int W>
__global__ __launch_bounds__(kBlock) void wide_build_kernel(WideBuildArgs g) {
  uint32_t probes = 0;
  const uint32_t flags = wide_build_range<W, false>(g, wave_range(g.n), g.rng_seed ^ lane_salt(),
                                                    &probes);
  if (flags) atomicOr(g.status, flags);
}

// Bit 0 of every W-lane group of a 64-bit lane mask set iff some bit of the
// group is (wave-uniform: scalar instructions).
template <int W>
__device__ __forceinline__ uint64_t group_any(uint64_t x) {
  uint64_t low = 0;
#pragma unroll
  for (int t = 0; t < 64; t += W) low |= 1ull << t;
#pragma unroll
  for (int sh = 1; sh < W; sh <<= 1) x |= x >> sh;
  return x & low;
}

// Cuckoo query with early exit, chunk schedule (as the 32-bit kernel), with
// the per-slice work kept to compares: the tile's queries are exchanged
// once per chunk and its bucket indices once per round; a slice whose owner
// is closed is not loaded; the tile reductions of the ballots are scalar
// (bit t*W + j of hacc / eacc is tile t's answer for its lane j); the one
// matching lane of a tile (keys are unique) leaves the value in the owner's
// LDS word.  COUNT: each query's bucket reads go to g.probes.
template <int W, bool COUNT = false>
__global__ __launch_bounds__(kBlock) void wide_find_chunk_kernel(WideFindArgs g) {
  constexpr int B = W;
  const uint32_t lane = __lane_id();
  const uint32_t tb = lane & ~(uint32_t)(W - 1);
  const uint32_t lt = lane & (uint32_t)(W - 1);
  __shared__ uint64_t vlds[kBlock];
  uint64_t* const vbuf = vlds + (threadIdx.x & ~63u);
  const Range r = wave_range(g.n);
  u64x2 d[W];
#pragma unroll
  for (int j = 0; j < W; ++j) d[j] = u64x2{kEmpty64, kEmpty64};
  uint64_t q_next = (r.cursor + lane < r.end) ? g.queries[r.cursor + lane] : kEmpty64;
  for (uint64_t base = r.cursor; base < r.end; base += 64) {
    const uint64_t idx = base + lane;
    const bool valid = idx < r.end;
    const uint64_t q = q_next;
    q_next = (base + 64 + lane < r.end) ? g.queries[base + 64 + lane] : kEmpty64;
    bool open = valid && q < kBusy64;
    uint64_t out = kEmpty64;
    uint8_t found = 0, rounds = 0;
    uint64_t qt[W];
#pragma unroll
    for (int j = 0; j < W; ++j) qt[j] = shfl64(q, tb + j);
    for (uint32_t round = 0; round < g.H.h; ++round) {
      const uint64_t om = ballot(open);
      if (om == 0) break;
      const uint32_t bucket = open ? (uint32_t)hash64(sel4(g.H.a, round), sel4(g.H.c, round), q,
                                                      g.H.M, g.H.m)
                                   : 0u;
      uint32_t bj[W];
#pragma unroll
      for (int j = 0; j < W; ++j) bj[j] = shfl32(bucket, tb + j);
      const uint32_t own = (uint32_t)(om >> tb);
#pragma unroll
      for (int j = 0; j < W; ++j)
        if ((own >> j) & 1u) d[j] = reinterpret_cast<const u64x2*>(g.slots)[(uint64_t)bj[j] * B + lt];
      uint64_t hacc = 0, eacc = 0;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const bool hs = d[j].x == qt[j];
        if (hs) vbuf[tb + j] = d[j].y;
        hacc |= group_any<W>(__builtin_amdgcn_ballot_w64(hs)) << j;
        eacc |= group_any<W>(__builtin_amdgcn_ballot_w64(d[j].x == kEmpty64)) << j;
      }
      if (open) {
        rounds = (uint8_t)(round + 1);
        if ((hacc >> lane) & 1ull) {
          out = vbuf[lane];
          found = 1;
          open = false;
        } else if ((eacc >> lane) & 1ull) {
          open = false;
        }
      }
    }
    if (valid) {
      g.out_v[idx] = out;
      g.out_f[idx] = found;
      if (COUNT) g.probes[idx] = rounds;
    }
  }
}

}  // namespace bht
