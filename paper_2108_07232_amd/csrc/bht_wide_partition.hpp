// Partitioned bulk build of the 64-bit table (16-byte slots, 8 per bucket).
//
// The same three steps as the 32-bit partitioned build: radix passes that
// group the pairs by the bin of their first bucket, bin placement in LDS,
// and an overflow phase for the pairs evicted during placement.  What
// differs is the on-chip cuckoo step: a 16-byte pair cannot be exchanged
// with one LDS atomic, so the pairs that meet a full first bucket make
// their exchanges in rounds.  The load counter of the bucket ranks them
// (rank = claimed slot - B); in round r each bucket's evictor of rank r
// swaps itself with a random slot, and a barrier separates the rounds.
// Within a bucket this is the serial order of Section III-A: every
// evictor finds the bucket as the earlier ones left it, and may displace
// one of them.  Every displaced pair left its first bucket, so it continues
// at the next bucket of its hash sequence in the overflow kernel, which is
// the 64-bit concurrent insertion started there.
#pragma once
#include "bht_partition.hpp"
#include "bht_wide.hpp"

namespace bht {

constexpr int kBin64Slots = 4096;      // 16-byte slots of one bin (64 KB of LDS)
constexpr int kBin64Per = 8;           // pairs per thread per placement round

__global__ __launch_bounds__(kPassBlock) void part_hist64_kernel(PartPass64 p) {
  uint32_t seg;
  uint64_t begin, end;
  if (!part_chunk(p, blockIdx.x, &seg, &begin, &end)) return;
  uint32_t* h = (p.level == 1 ? p.M.hist1 : p.M.hist2) + (uint64_t)blockIdx.x * p.fan;
  unsigned long long* tot = p.level == 1 ? p.M.total1 : p.M.total2 + (uint64_t)seg * kFan2;
  const PartPlan& P = p.P;
  const uint32_t level = p.level;
  const bool sentinel = hist_range(p.in_k, begin, end, p.fan,
                                   [&](uint64_t k) { return part_digit(P, level, k); }, h, tot,
                                   p.padded != 0, p.lines ? line_words<uint64_t>() : 0u);
  if (level == 1 && sentinel) atomicOr(p.status, kFlagSentinel);
}

__global__ __launch_bounds__(kPassBlock, kScatterBlocksPerCU) void part_scatter64_kernel(PartPass64 p) {
  uint32_t seg;
  uint64_t begin, end;
  if (!part_chunk(p, blockIdx.x, &seg, &begin, &end)) return;
  const uint32_t* h = (p.level == 1 ? p.M.hist1 : p.M.hist2) + (uint64_t)blockIdx.x * p.fan;
  unsigned long long* cur = p.level == 1 ? p.M.cursor1 : p.M.cursor2 + (uint64_t)seg * kFan2;
  const PartPlan& P = p.P;
  const uint32_t level = p.level;
  scatter_range(p.in_k, p.in_v, begin, end, p.fan,
                [&](uint64_t k) { return part_digit(P, level, k); }, h, cur, p.out_k, p.out_v,
                p.padded != 0);
}

struct BinArgs64 {
  uint64_t* slots;               // the table: key word, value word per slot
  uint64_t* keys;                // partitioned pairs; evicted pairs are written back in place
  uint64_t* vals;
  uint32_t* status;
  uint32_t max_chain;
  uint32_t rng_seed;
  PartPlan P;
  PartMeta M;
};

// One bin of 8-slot buckets in LDS: buckets [first, first + nb) of the
// table (nb <= R <= kBin64Slots / 8), pairs keys/vals[s0, s0 + len).
// Evicted pairs are written to the front of that range; returns (in every
// thread) their number.  Every thread of the block calls it.
__device__ __forceinline__ uint32_t place_bin64(const BinArgs64& a, uint32_t R, uint64_t first,
                                                uint32_t nb, uint64_t s0, uint64_t len,
                                                uint32_t salt) {
  constexpr int B = 8;
  constexpr int RMAX = kBin64Slots / B;
  __shared__ u64x2 tbl[kBin64Slots];
  __shared__ uint32_t load[RMAX];
  __shared__ uint32_t top[2];              // 1 + the largest eviction rank of a round
  __shared__ uint32_t ovf;
  const u64x2 e2 = {kEmpty64, kEmpty64};
  for (uint32_t i = threadIdx.x; i < R * B; i += kBinBlock) tbl[i] = e2;
  for (uint32_t i = threadIdx.x; i < R; i += kBinBlock) load[i] = 0;
  if (threadIdx.x == 0) {
    ovf = 0;
    top[0] = 0;
  }
  uint32_t rng = a.rng_seed ^ (salt * 0x9E3779B9u) ^ (threadIdx.x * 0x85EBCA6Bu);
  if (rng == 0) rng = 0x2545F491u;
  uint32_t flags = 0;
  const Hash64& H = a.P.H64;
  __syncthreads();
  uint32_t parity = 0;
  for (uint64_t r0 = 0; r0 < len; r0 += (uint64_t)kBinBlock * kBin64Per, parity ^= 1) {
    uint64_t k[kBin64Per], v[kBin64Per];
    uint32_t fb[kBin64Per], fr[kBin64Per];     // full first bucket (or ~0) and eviction rank
#pragma unroll
    for (int j = 0; j < kBin64Per; ++j) {
      // branch-free loads: indices past the end re-read the bin's last pair
      const uint64_t i = r0 + j * kBinBlock + threadIdx.x;
      k[j] = a.keys[s0 + (i < len ? i : len - 1)];
      v[j] = a.vals[s0 + (i < len ? i : len - 1)];
    }
    uint32_t my_top = 0;
#pragma unroll
    for (int j = 0; j < kBin64Per; ++j) {
      fb[j] = ~0u;
      fr[j] = 0;
      const uint64_t i = r0 + j * kBinBlock + threadIdx.x;
      // the empty key marks padding of a line-writing pass (a caller's
      // reserved key has already failed the build)
      if (i < len && k[j] != kEmpty64) {
        // lb < nb by construction of the partition
        const uint32_t lb = (uint32_t)(hash64(H, 0, k[j]) - first);
        if (lb >= nb) {
          flags |= kFlagFailed;
        } else {
          const uint32_t s = atomicAdd(&load[lb], 1u);
          if (s < (uint32_t)B) {
            const u64x2 pr = {k[j], v[j]};
            tbl[lb * B + s] = pr;
          } else if (a.max_chain == 0) {
            flags |= kFlagFailed;
          } else {
            fb[j] = lb;
            fr[j] = s - B;
            my_top = my_top > s - B + 1 ? my_top : s - B + 1;
          }
        }
      }
    }
    if (my_top) atomicMax(&top[parity], my_top);
    // every claimed slot is written and every pair of this round read
    __syncthreads();
    const uint32_t T = top[parity];
    if (threadIdx.x == 0) top[parity ^ 1] = 0;       // for the next round of pairs
    // Ranks of earlier rounds of pairs are below this round's, so rounds
    // with none of this round's evictors only cost a barrier.
    for (uint32_t round = 0; round < T; ++round) {
#pragma unroll
      for (int j = 0; j < kBin64Per; ++j) {
        if (fb[j] != ~0u && fr[j] == round) {
          rng = xorshift32(rng);
          u64x2* const slot = &tbl[fb[j] * B + rng % (uint32_t)B];
          const u64x2 old = *slot;
          const u64x2 pr = {k[j], v[j]};
          *slot = pr;
          k[j] = old.x;
          v[j] = old.y;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kBin64Per; ++j) {
      if (fb[j] != ~0u) {
        const uint32_t pos = atomicAdd(&ovf, 1u);
        a.keys[s0 + pos] = k[j];
        a.vals[s0 + pos] = v[j];
      }
    }
    // orders the reset of the other top word before its next use
    __syncthreads();
  }
  const uint32_t count = nb * B;
  u64x2* dst = reinterpret_cast<u64x2*>(a.slots) + first * B;
  for (uint32_t i = threadIdx.x; i < count; i += kBinBlock) dst[i] = tbl[i];
  if (flags) atomicOr(a.status, flags);
  return ovf;
}

__global__ __launch_bounds__(kBinBlock) void bin_place64_kernel(BinArgs64 a) {
  const uint32_t R = 1u << a.P.bin_shift;
  const uint32_t bin = blockIdx.x;
  const uint64_t first = (uint64_t)bin * R;
  const uint32_t nb = a.P.H64.m - first < (uint64_t)R ? (uint32_t)(a.P.H64.m - first) : R;
  const uint32_t ovf = place_bin64(a, R, first, nb, a.M.bin_start[bin], a.M.bin_len[bin], bin);
  if (threadIdx.x == 0) {
    a.M.ovf_len[bin] = ovf;
    if (ovf) atomicAdd(a.status + 1, ovf);
  }
}

struct WideOverflowArgs {
  WideBuildArgs g;               // keys / vals = the partitioned arrays
  PartMeta M;
  uint32_t nbins;
};

// Insertion of the pairs evicted during placement, bin by bin from a queue;
// bucket reads are summed into status words 2-3.
template <int W>
__global__ __launch_bounds__(kBlock) void wide_overflow_kernel(WideOverflowArgs a) {
  const uint32_t salt = lane_salt();
  uint32_t flags = 0, probes = 0;
  for (;;) {
    const uint32_t bin = part_queue_pop(a.M.head);
    if (bin >= a.nbins) break;
    const uint32_t len = a.M.ovf_len[bin];
    if (len == 0) continue;
    Range r;
    r.cursor = a.M.bin_start[bin];
    r.end = r.cursor + len;
    flags |= wide_build_range<W, true>(a.g, r, a.g.rng_seed ^ salt ^ (bin * 0x85EBCA6Bu), &probes);
  }
  if (flags) atomicOr(a.g.status, flags);
  const uint32_t total = wave_sum(probes);
  if (__lane_id() == 0 && total)
    atomicAdd(reinterpret_cast<unsigned long long*>(a.g.status + 2), (unsigned long long)total);
}

}  // namespace bht
