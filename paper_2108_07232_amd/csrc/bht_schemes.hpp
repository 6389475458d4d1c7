// Comparison schemes on the same tile skeleton as the cuckoo table:
// bucketed power-of-two choices (Section III-B, Section V-C), iceberg
// hashing (Section III-C, Section V-D) and the load-balanced cuckoo table
// (Section III-A's variation), plus one query kernel for every scheme whose
// queries cannot stop early on a bucket with room.
//
// Insertion follows the cuckoo kernel's rules for concurrency: a bucket is
// read once, the lane then claims slot = load with a CAS and walks to the
// next slot when a CAS fails, never re-reading; a bucket whose walk reaches
// its end is full (occupancy only grows during a build).  When a walk
// exhausts the chosen bucket the lane moves to the scheme's next choice from
// the loads it already read, so no step can spin.
#pragma once
#include "bht_kernels.hpp"

namespace bht {

// Tile read of a bucket of BS slots by W lanes when W may exceed BS: lanes
// beyond the bucket hold empty slots.
template <int BS, int W>
struct Slice {
  static constexpr int S = BS >= W ? BS / W : 1;
};

// FRESH: device-scope loads (for placements that compare bucket loads).
template <int BS, int W, bool FRESH = false>
__device__ __forceinline__ void tile_read_any(const uint64_t* __restrict__ base, uint32_t bucket,
                                              uint64_t mask, uint32_t tb, uint32_t lt,
                                              Part<Slice<BS, W>::S> (&d)[W]) {
  constexpr int S = Slice<BS, W>::S;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const uint32_t bj = shfl32(bucket, tb + j);
    if (((mask >> (tb + j)) & 1ull) && lt * S < (uint32_t)BS)
      d[j] = FRESH ? load_part_fresh<S>(base + (uint64_t)bj * BS + lt * S)
                   : load_part<S>(base + (uint64_t)bj * BS + lt * S);
    else
      d[j] = empty_part<S>();
  }
}

template <int BS, int W>
__device__ __forceinline__ uint32_t tile_load_any(const Part<Slice<BS, W>::S> (&d)[W],
                                                  uint32_t tb, uint32_t lt) {
  constexpr int S = Slice<BS, W>::S;
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

template <int BS, int W>
__device__ __forceinline__ void tile_match_any(const Part<Slice<BS, W>::S> (&d)[W], uint32_t q,
                                               uint32_t tb, uint32_t lt, bool* hit,
                                               uint32_t* value) {
  constexpr int S = Slice<BS, W>::S;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const uint32_t qj = shfl32(q, tb + j);
    bool m = false;
    uint32_t vsel = kEmptyKey;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if ((uint32_t)d[j].s[s] == qj) {
        m = true;
        vsel = (uint32_t)(d[j].s[s] >> 32);
      }
    }
    const uint64_t hm = tile_bits<W>(ballot(m), tb);
    const uint32_t v = shfl32(vsel, tb + (hm ? (uint32_t)__builtin_ctzll(hm) : 0u));
    if (lt == (uint32_t)j) {
      *hit = hm != 0;
      *value = v;
    }
  }
}

struct SchemeArgs32 {
  uint64_t* slots;           // primary array (m * B slots)
  uint64_t* slots2;          // iceberg secondary array (m2 * B2 slots) or null
  const uint32_t* keys;
  const uint32_t* vals;
  uint64_t n;
  uint32_t* status;
  unsigned long long* probe_total;
  Hash32 H;                  // buckets of the primary array
  Hash32 H2;                 // buckets of the secondary array (iceberg, two levels)
  uint32_t threshold;        // iceberg t
};

// A bounded walk over one bucket: CAS at slot, slot+1, ... up to limit.
struct Walk {
  uint64_t first;  // slot index of the bucket's first slot in its array
  uint32_t slot, limit;
  bool secondary;
};

enum : uint32_t { kP2Read = 0, kP2Walk1 = 1, kP2Walk2 = 2 };

// Placements that compare bucket loads (power of two, iceberg secondaries)
// read the candidates with device-scope loads, and a pair whose CAS loses
// its slot to a concurrent placement reads both candidates again and
// chooses again, so that a choice is made on current loads.
#ifndef BHT_CHOICE_FRESH
#define BHT_CHOICE_FRESH 1
#endif
constexpr bool kChoiceFresh = BHT_CHOICE_FRESH != 0;
#ifndef BHT_CHOICE_REDECIDE
#define BHT_CHOICE_REDECIDE 1
#endif
constexpr bool kChoiceRedecide = BHT_CHOICE_REDECIDE != 0;

// Power-of-two-choices insertion: read H0 and H1, claim a slot in the less
// loaded bucket (ties to H0); if its walk runs out, the other bucket; if
// both are full the build fails.
template <int B, int W, bool COUNT>
__global__ __launch_bounds__(kBlock) void p2_build_kernel(SchemeArgs32 g) {
  const uint32_t lane = __lane_id();
  const uint32_t tb = lane & ~(uint32_t)(W - 1);
  const uint32_t lt = lane & (uint32_t)(W - 1);
  const Range r = wave_range(g.n);
  Feed<uint32_t> fk, fv;
  fk.init(g.keys, r, kEmptyKey);
  fv.init(g.vals, r, 0u);
  bool active = false;
  uint32_t key = 0, val = 0, b0 = 0, b1 = 0, l_other = 0, other = 0, phase = kP2Read;
  Walk w = {0, 0, 0, false};
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
        b0 = hash32(g.H, 0, key);
        b1 = hash32(g.H, 1, key);
        phase = kP2Read;
      }
    }
    if (ballot(active) == 0) {
      if (fk.cursor >= fk.end) break;
      continue;
    }
    const uint64_t rd = ballot(active && phase == kP2Read);
    if (rd) {
      Part<Slice<B, W>::S> d[W];
      tile_read_any<B, W, kChoiceFresh>(g.slots, b0, rd, tb, lt, d);
      const uint32_t l0 = tile_load_any<B, W>(d, tb, lt);
      tile_read_any<B, W, kChoiceFresh>(g.slots, b1, rd, tb, lt, d);
      const uint32_t l1 = tile_load_any<B, W>(d, tb, lt);
      if (active && phase == kP2Read) {
        if (COUNT) probes += 2;
        if (l0 >= (uint32_t)B && l1 >= (uint32_t)B) {
          flags |= kFlagFailed;
          active = false;
        } else {
          const bool first0 = l0 <= l1;
          w = {(uint64_t)(first0 ? b0 : b1) * B, first0 ? l0 : l1, (uint32_t)B, false};
          other = first0 ? b1 : b0;
          l_other = first0 ? l1 : l0;
          phase = kP2Walk1;
        }
      }
    }
    if (active && phase != kP2Read) {
      const uint64_t pair = ((uint64_t)val << 32) | key;
      if (w.slot < w.limit && cas64(g.slots + w.first + w.slot, kEmptyPair, pair) == kEmptyPair) {
        active = false;
      } else if (kChoiceRedecide) {
        // another placement took the slot since the read: read both
        // buckets again and choose again (each retry follows a placement
        // into one of them, so a pair retries at most 2B times)
        phase = kP2Read;
      } else if (w.slot + 1 < w.limit) {
        ++w.slot;
      } else if (phase == kP2Walk1 && l_other < (uint32_t)B) {
        w = {(uint64_t)other * B, l_other, (uint32_t)B, false};
        phase = kP2Walk2;
      } else {
        flags |= kFlagFailed;
        active = false;
      }
    }
  }
  if (flags) atomicOr(g.status, flags);
  if (COUNT) {
    const uint32_t total = wave_sum(probes);
    if (__lane_id() == 0 && total) atomicAdd(g.probe_total, (unsigned long long)total);
  }
}

enum : uint32_t { kLbRead = 0, kLbPick = 1, kLbWalk = 2, kLbEvict = 3 };

// Load-balanced cuckoo insertion (Section III-A's variation that inserts
// into the least loaded of the h buckets): read all h candidates, claim a
// slot in the least loaded one with room per that read (ties to the lowest
// hash index), walking on CAS failures; a walk that reaches the end proves
// its bucket full and the lane turns to the next candidate from the same
// read.  With every candidate full the pair is exchanged with a random
// resident of a random candidate other than the bucket it was just evicted
// from, and the evicted pair starts over with its own candidates.  A bucket
// is taken as full only when a read showed b pairs (reads can only
// under-report) or a walk failed on every slot, so exchanges hit occupied
// slots and occupied slots stay a prefix; no bucket is read twice for the
// same pair, so no lane can spin on a stale copy.
template <int B, int W, bool COUNT>
__global__ __launch_bounds__(kBlock) void lb_build_kernel(BuildArgs32 g) {
  const uint32_t lane = __lane_id();
  const uint32_t tb = lane & ~(uint32_t)(W - 1);
  const uint32_t lt = lane & (uint32_t)(W - 1);
  const uint32_t h = g.H.h;
  const Range r = wave_range(g.n);
  uint32_t rng = g.rng_seed ^ lane_salt();
  if (rng == 0) rng = 0x2545F491u;
  Feed<uint32_t> fk, fv;
  fk.init(g.keys, r, kEmptyKey);
  fv.init(g.vals, r, 0u);
  bool active = false;
  uint32_t key = 0, val = 0, chain = 0, left = ~0u, phase = kLbRead;
  uint32_t cb[4] = {0u, 0u, 0u, 0u};                       // candidate buckets
  uint32_t cl[4] = {(uint32_t)B, (uint32_t)B, (uint32_t)B, (uint32_t)B};  // their loads
  uint32_t cur = 0, slot = 0, probes = 0, flags = 0;

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
        chain = 0;
        left = ~0u;
        phase = kLbRead;
      }
    }
    if (ballot(active) == 0) {
      if (fk.cursor >= fk.end) break;
      continue;
    }
    const uint64_t rd = ballot(active && phase == kLbRead);
    if (rd) {
      const bool me = active && phase == kLbRead;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i < (int)h) {
          const uint32_t bi = me ? hash32(g.H, i, key) : 0u;
          Part<B / W> d[W];
          tile_read<B, W>(g.slots, bi, rd, tb, lt, d);
          const uint32_t li = tile_load<B, W>(d, tb, lt);
          if (me) {
            cb[i] = bi;
            cl[i] = li;
          }
        }
      }
      if (me) {
        if (COUNT) probes += h;
        phase = kLbPick;
      }
    }
    if (active && phase == kLbPick) {
      uint32_t best = 4, bl = (uint32_t)B;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < (int)h && cl[i] < bl) {
          best = i;
          bl = cl[i];
        }
      if (best < 4) {
        cur = best;
        slot = bl;
        phase = kLbWalk;
      } else {
        phase = kLbEvict;
      }
    }
    const uint64_t pair = ((uint64_t)val << 32) | key;
    if (active && phase == kLbWalk) {
      const uint64_t old = cas64(g.slots + (uint64_t)sel4(cb, cur) * B + slot, kEmptyPair, pair);
      if (old == kEmptyPair) {
        active = false;
      } else if (++slot == (uint32_t)B) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if ((uint32_t)i == cur) cl[i] = (uint32_t)B;   // proven full
        phase = kLbPick;
      }
    } else if (active && phase == kLbEvict) {
      if (chain >= g.max_chain) {
        flags |= kFlagFailed;
        active = false;
      } else {
        uint32_t ne = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i < (int)h && cb[i] != left) ++ne;
        rng = xorshift32(rng);
        const uint32_t want = rng % (ne ? ne : h);
        uint32_t target = cb[0], seen = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i < (int)h && (ne == 0 || cb[i] != left)) {
            if (seen == want) target = cb[i];
            ++seen;
          }
        }
        rng = xorshift32(rng);
        const uint64_t old = xchg64(g.slots + (uint64_t)target * B + (rng % (uint32_t)B), pair);
        if (old == kEmptyPair) {
          active = false;
        } else {
          key = (uint32_t)old;
          val = (uint32_t)(old >> 32);
          left = target;
          ++chain;
          phase = kLbRead;
        }
      }
    }
  }
  if (flags) atomicOr(g.status, flags);
  if (COUNT) {
    const uint32_t total = wave_sum(probes);
    if (__lane_id() == 0 && total) atomicAdd(g.probe_total, (unsigned long long)total);
  }
}

enum : uint32_t { kIcReadP = 0, kIcReadS = 1, kIcWalkP = 2, kIcWalkS1 = 3, kIcWalkS2 = 4,
                  kIcWalkFallback = 5 };

// Iceberg insertion (reading of Section III-C): the primary bucket takes the
// pair while it holds fewer than t pairs; otherwise the two secondary
// buckets are read and the less loaded one (ties to s0) takes it, then the
// other; with both secondaries full the primary is used if it has room.  B2
// = 0 puts the secondary choices in the primary array (one level).  Inserts
// the pairs [r.cursor, r.end) of g.keys / g.vals (the whole wave calls it).
// AFTER_PRIMARY: each pair's primary is known to hold t pairs in its first
// t slots (the partitioned build placed them), so the pair starts at its
// secondary choices.  Bucket reads are added to *probes_out when COUNT;
// returns the lane's status flags.
template <int B, int B2, int W, bool COUNT, bool AFTER_PRIMARY = false>
__device__ __forceinline__ uint32_t iceberg_build_range(const SchemeArgs32& g, Range r,
                                                        uint32_t* probes_out) {
  constexpr int BS2 = B2 ? B2 : B;
  const uint32_t lane = __lane_id();
  const uint32_t tb = lane & ~(uint32_t)(W - 1);
  const uint32_t lt = lane & (uint32_t)(W - 1);
  uint64_t* const sec = B2 ? g.slots2 : g.slots;
  const Hash32& HS = B2 ? g.H2 : g.H;
  Feed<uint32_t> fk, fv;
  fk.init(g.keys, r, kEmptyKey);
  fv.init(g.vals, r, 0u);
  bool active = false;
  uint32_t key = 0, val = 0, p = 0, s0 = 0, s1 = 0, lp = 0, l_other = 0, other = 0;
  uint32_t phase = kIcReadP;
  Walk w = {0, 0, 0, false};
  uint32_t probes = 0, flags = 0;
  const uint32_t t = g.threshold < (uint32_t)B ? g.threshold : (uint32_t)B;

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
        p = hash32(g.H, 0, key);
        phase = kIcReadP;
        if constexpr (AFTER_PRIMARY) {
          lp = t;
          s0 = hash32(HS, 1, key);
          s1 = hash32(HS, 2, key);
          phase = kIcReadS;
        }
      }
    }
    if (ballot(active) == 0) {
      if (fk.cursor >= fk.end) break;
      continue;
    }
    const uint64_t rp = ballot(active && phase == kIcReadP);
    if (rp) {
      Part<Slice<B, W>::S> d[W];
      tile_read_any<B, W>(g.slots, p, rp, tb, lt, d);
      const uint32_t l = tile_load_any<B, W>(d, tb, lt);
      if (active && phase == kIcReadP) {
        if (COUNT) ++probes;
        lp = l;
        if (l < t) {
          w = {(uint64_t)p * B, l, t, false};
          phase = kIcWalkP;
        } else {
          s0 = hash32(HS, 1, key);
          s1 = hash32(HS, 2, key);
          phase = kIcReadS;
        }
      }
    }
    const uint64_t rs = ballot(active && phase == kIcReadS);
    if (rs) {
      Part<Slice<BS2, W>::S> d[W];
      tile_read_any<BS2, W, kChoiceFresh>(sec, s0, rs, tb, lt, d);
      const uint32_t l0 = tile_load_any<BS2, W>(d, tb, lt);
      tile_read_any<BS2, W, kChoiceFresh>(sec, s1, rs, tb, lt, d);
      const uint32_t l1 = tile_load_any<BS2, W>(d, tb, lt);
      if (active && phase == kIcReadS) {
        if (COUNT) probes += 2;
        if (l0 < (uint32_t)BS2 || l1 < (uint32_t)BS2) {
          const bool first0 = l0 <= l1;
          w = {(uint64_t)(first0 ? s0 : s1) * BS2, first0 ? l0 : l1, (uint32_t)BS2, true};
          other = first0 ? s1 : s0;
          l_other = first0 ? l1 : l0;
          phase = kIcWalkS1;
        } else {
          w = {(uint64_t)p * B, lp > t ? lp : t, (uint32_t)B, false};
          phase = kIcWalkFallback;
        }
      }
    }
    if (active && phase >= kIcWalkP) {
      const uint64_t pair = ((uint64_t)val << 32) | key;
      uint64_t* const base = w.secondary ? sec : g.slots;
      if (w.slot < w.limit && cas64(base + w.first + w.slot, kEmptyPair, pair) == kEmptyPair) {
        active = false;
      } else if (kChoiceRedecide && (phase == kIcWalkS1 || phase == kIcWalkS2)) {
        // a concurrent placement took the slot: read both secondaries again
        // and choose again (bounded: each retry follows a placement into one
        // of them)
        phase = kIcReadS;
      } else if (w.slot + 1 < w.limit) {
        ++w.slot;
      } else if (phase == kIcWalkP) {
        // the primary reached t pairs: go to the secondary choices
        lp = t;
        s0 = hash32(HS, 1, key);
        s1 = hash32(HS, 2, key);
        phase = kIcReadS;
      } else if (phase == kIcWalkS1 && l_other < (uint32_t)BS2) {
        w = {(uint64_t)other * BS2, l_other, (uint32_t)BS2, true};
        phase = kIcWalkS2;
      } else if (phase == kIcWalkS1 || phase == kIcWalkS2) {
        w = {(uint64_t)p * B, lp > t ? lp : t, (uint32_t)B, false};
        phase = kIcWalkFallback;
      } else {
        flags |= kFlagFailed;
        active = false;
      }
    }
  }
  if (COUNT) *probes_out += probes;
  return flags;
}

template <int B, int B2, int W, bool COUNT>
__global__ __launch_bounds__(kBlock) void iceberg_build_kernel(SchemeArgs32 g) {
  uint32_t probes = 0;
  const uint32_t flags = iceberg_build_range<B, B2, W, COUNT>(g, wave_range(g.n), &probes);
  if (flags) atomicOr(g.status, flags);
  if (COUNT) {
    const uint32_t total = wave_sum(probes);
    if (__lane_id() == 0 && total) atomicAdd(g.probe_total, (unsigned long long)total);
  }
}

struct SchemeFindArgs32 {
  const uint64_t* slots;
  const uint64_t* slots2;
  const uint32_t* queries;
  uint64_t n;
  uint32_t* out_v;
  uint8_t* out_f;
  uint8_t* probes;
  Hash32 H;
  Hash32 H2;
  uint32_t rounds;           // candidate buckets per query (2 or 3)
  uint32_t early_below;      // iceberg: a miss in a primary holding fewer keys ends the query
};

// Queries of the stable schemes: probe the candidates in order and stop only
// on a hit (Section V-C, Section V-D: no early exit).  Chunk schedule as the
// cuckoo query.  With B2 > 0, rounds after the first read the secondary
// array.  early_below = t > 0 (iceberg): a key reaches a secondary bucket
// only once its primary holds t keys (Section III-C), so a miss in a
// primary holding fewer than t keys proves absence after one probe.
template <int B, int B2, int W, bool COUNT>
__global__ __launch_bounds__(kBlock) void stable_find_chunk_kernel(SchemeFindArgs32 g) {
  constexpr int BS2 = B2 ? B2 : B;
  const uint32_t lane = __lane_id();
  const uint32_t tb = lane & ~(uint32_t)(W - 1);
  const uint32_t lt = lane & (uint32_t)(W - 1);
  const Range r = wave_range(g.n);
  const uint64_t* const sec = B2 ? g.slots2 : g.slots;
  const Hash32& HS = B2 ? g.H2 : g.H;
  uint32_t q_next = (r.cursor + lane < r.end) ? g.queries[r.cursor + lane] : kEmptyKey;
  for (uint64_t base = r.cursor; base < r.end; base += 64) {
    const uint64_t idx = base + lane;
    const bool valid = idx < r.end;
    const uint32_t q = q_next;
    q_next = (base + 64 + lane < r.end) ? g.queries[base + 64 + lane] : kEmptyKey;
    bool open = valid && q != kEmptyKey;
    uint32_t out = kEmptyKey, rounds = 0;
    uint8_t found = 0;
    for (uint32_t round = 0; round < g.rounds; ++round) {
      const uint64_t om = ballot(open);
      if (om == 0) break;
      bool hit = false;
      uint32_t value = kEmptyKey;
      bool below = false;
      if (round == 0) {
        const uint32_t bucket = open ? hash32(g.H, 0, q) : 0u;
        Part<Slice<B, W>::S> d[W];
        tile_read_any<B, W>(g.slots, bucket, om, tb, lt, d);
        tile_match_any<B, W>(d, q, tb, lt, &hit, &value);
        if (g.early_below) below = tile_load_any<B, W>(d, tb, lt) < g.early_below;
      } else {
        const uint32_t bucket = open ? hash32_dyn(HS, round, q) : 0u;
        Part<Slice<BS2, W>::S> d[W];
        tile_read_any<BS2, W>(sec, bucket, om, tb, lt, d);
        tile_match_any<BS2, W>(d, q, tb, lt, &hit, &value);
      }
      if (open) {
        rounds = round + 1;
        if (hit) {
          out = value;
          found = 1;
          open = false;
        } else if (below) {
          open = false;
        }
      }
    }
    if (valid) {
      g.out_v[idx] = out;
      g.out_f[idx] = found;
      if (COUNT) g.probes[idx] = (uint8_t)rounds;
    }
  }
}

}  // namespace bht
