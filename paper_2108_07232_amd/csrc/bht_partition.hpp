// Partitioned bulk build of a bucketed cuckoo table (BCHT, and the
// one-slot table); the radix passes and the placement without eviction
// also serve the iceberg table's build.
//
// The paper's build inserts every pair concurrently with one bucket read
// and one slot atomic each (Section V-B).  On MI355X the slot atomics are
// performed at the memory side and cap such a build near 20 G pairs/s
// whatever the load factor.  This path reaches the same kind of layout with
// streaming traffic instead:
//
//   1. partition: the pairs are grouped by the region of their first
//      bucket H_0(k) (a bin of R consecutive buckets whose slots fit in
//      LDS; smaller bins for small tables, so that there are enough of
//      them to fill the device), with one or two radix passes (fan-out at
//      most 1024, then 256); each pass counts digits per chunk of pairs,
//      reserves output ranges per (chunk, digit), and writes each sub-tile
//      in digit order staged through LDS, so stores are contiguous runs;
//      with at most 256 digits a pass writes whole 128-byte lines only: a
//      digit's elements that do not fill a line wait in LDS for the next
//      sub-tile, and each (chunk, digit) range is padded to whole lines with
//      the empty key, which later steps skip;
//   2. bin placement: one workgroup per bin builds its buckets in LDS,
//      placing each pair in its first bucket at the next free slot
//      (a local atomic on the bucket's load); a pair that finds its first
//      bucket full evicts a random resident of that bucket on chip (the
//      first cuckoo step), and the evicted pair is kept, in place at the
//      front of the bin's input range; the whole bin, empty slots included,
//      is written to the table with full-line stores (so no reset pass);
//   3. overflow: the concurrent cuckoo insertion continues every evicted
//      pair at its next bucket, bin by bin from a device work queue.
//
// Steps 2 and 3 are Section III-A's insertion under a deferred-victim
// schedule: every pair first claims a slot of its first bucket (at slot =
// load); each pair that meets a full first bucket exchanges itself with a
// random resident there, on chip, in the order of its claim; the evicted
// pairs' cuckoo chains then run concurrently, as in the concurrent build.
// No step ever empties a slot, so the layout properties of the concurrent
// build hold (every key in a candidate bucket, buckets filled as prefixes,
// the early-exit property), and lookups are unchanged.  Pair order within a
// bin or digit is not preserved and need not be.
#pragma once
#include <type_traits>

#include "bht_kernels.hpp"

namespace bht {

// Threads per counting / scatter block and pairs staged per sub-tile
// (compile-time tuning; by default 16 pairs per thread).
#ifndef BHT_PASS_BLOCK
#define BHT_PASS_BLOCK 1024
#endif
#ifndef BHT_PASS_PER
#define BHT_PASS_PER 16
#endif
#ifndef BHT_SCATTER_BLOCKS_PER_CU
#define BHT_SCATTER_BLOCKS_PER_CU 1
#endif
#ifndef BHT_SCATTER_STAGE_DIGITS
#define BHT_SCATTER_STAGE_DIGITS 1
#endif
#ifndef BHT_SCATTER_LINES
#define BHT_SCATTER_LINES 1
#endif
constexpr bool kScatterLines = BHT_SCATTER_LINES != 0;         // line-writing scatter where it applies
constexpr int kScatterBlocksPerCU = BHT_SCATTER_BLOCKS_PER_CU;   // occupancy the scatter is compiled for
constexpr bool kScatterStageDigits = BHT_SCATTER_STAGE_DIGITS != 0; // digits staged beside the pairs
constexpr int kPartBlock = 256;                        // threads per scan block
constexpr int kPassBlock = BHT_PASS_BLOCK;
constexpr int kPartSub = BHT_PASS_PER * kPassBlock;   // pairs per sub-tile (4-byte words)
// Pairs per partition block of one table's build, at most: 128 K (at 2^28
// pairs, 2,048 first-pass chunks; a line-writing pass pads each (chunk,
// digit) range, so larger chunks pad less: 1.7% and 3.2% of the pairs at
// 2^28 against 3.4% and 6.3% with 64 K chunks, and the padded first pass
// fits the slot array up to LF 0.96 at 2^28 pairs, 0.98 at 2^27); the
// batched build keeps 64 K-pair chunks.
#ifndef BHT_PART_CHUNK_SUBS
#define BHT_PART_CHUNK_SUBS 8
#endif
constexpr uint32_t kPartChunkMax = BHT_PART_CHUNK_SUBS * kPartSub;
constexpr uint32_t kBatchChunk = 4 * kPartSub;
constexpr uint32_t kMaxFan = 1024;                     // digits of the first pass, at most
constexpr uint32_t kFan2 = 256;                        // digits of the second pass
constexpr int kLineSub = 8 * kPassBlock;               // pairs per sub-tile of the line-writing scatter
constexpr uint32_t kLineMaxFan = 256;                  // its digits, at most (carried lines fill 64 KB)
constexpr uint32_t kLineWords = 32;                    // 4-byte words per 128-byte line
constexpr int kBinBlock = 512;                         // threads per bin placement block
constexpr int kBinPer = 16;                            // pairs per thread per round

// Slots of one bin (64 KB of LDS as 8-byte slots; the one-slot table keeps
// a 4-byte load counter per bucket beside them, so its bins are halved).
template <int B>
constexpr int bin_slots() { return B == 1 ? 4096 : 8192; }

struct PartPlan {
  Hash32 H;             // first hash (index 0) and bucket count, 32-bit keys
  Hash64 H64;           // the same for 64-bit keys
  uint32_t bin_shift;   // bin = H_0(k) >> bin_shift: 2^bin_shift buckets per bin
  uint32_t levels;      // radix passes: 1 or 2
  uint32_t fan1;        // digits of the first pass
  uint32_t nbins;
  uint32_t chunk;       // pairs per partition block (a multiple of the sub-tile)
  uint32_t lines1;      // the first pass writes whole lines (ranges padded with the empty key)
  uint32_t lines2;      // the same for the second pass
  uint32_t chunks2_cap; // second-pass chunks the workspace holds
  uint32_t resident2;   // second-pass scatter blocks resident at once (0: unknown)
};

// Words of T per 128-byte line, and the words of a (chunk, digit) range of
// c pairs when a pass writes whole lines of lw words.
template <typename T>
constexpr uint32_t line_words() { return 128 / sizeof(T); }
__host__ __device__ __forceinline__ uint32_t line_pad(uint32_t c, uint32_t lw = kLineWords) {
  return (c + lw - 1) & ~(lw - 1);
}

// Device metadata of one partitioned build (one allocation, see the host).
struct PartMeta {
  uint32_t* hist1;               // [chunks1][fan1]
  uint32_t* hist2;               // [chunks2 bound][256]
  unsigned long long* total1;    // [fan1]
  unsigned long long* cursor1;   // [fan1]
  unsigned long long* seg_start; // [fan1]  first-pass digit ranges
  unsigned long long* seg_len;   // [fan1]
  uint32_t* chunk_first;         // [fan1 + 1] second-pass chunks per range, prefix
  uint32_t* chunk_seg;           // [second-pass chunks] the range of each chunk
  unsigned long long* total2;    // [fan1 * 256]
  unsigned long long* cursor2;   // [fan1 * 256]
  unsigned long long* bin_start; // [nbins]
  unsigned long long* bin_len;   // [nbins]
  uint32_t* ovf_len;             // [nbins]
  unsigned int* head;            // overflow queue head
};

// One radix pass over pairs of T keys and T values.  Level 1 reads the
// caller's arrays as a single range of n pairs; level 2 reads the first
// pass's output as fan1 ranges (seg_*).
template <typename T>
struct PartPassT {
  const T* in_k;
  const T* in_v;
  T* out_k;
  T* out_v;
  uint64_t n;
  uint32_t level;
  uint32_t fan;
  uint32_t lines;      // this pass writes whole lines (line-writing scatter)
  uint32_t padded;     // its input may hold padding (the empty key), skipped
  uint32_t* status;
  PartPlan P;
  PartMeta M;
};
using PartPass64 = PartPassT<uint64_t>;

__device__ __forceinline__ uint32_t part_split(const PartPlan& P, uint32_t level, uint32_t bin) {
  if (P.levels == 1) return bin;
  return level == 1 ? bin >> 8 : bin & (kFan2 - 1);
}

__device__ __forceinline__ uint32_t part_digit(const PartPlan& P, uint32_t level, uint32_t key) {
  return part_split(P, level, hash32(P.H, 0, key) >> P.bin_shift);
}

__device__ __forceinline__ uint32_t part_digit(const PartPlan& P, uint32_t level, uint64_t key) {
  return part_split(P, level, (uint32_t)hash64(P.H64, 0, key) >> P.bin_shift);
}

// Block -> (range, chunk): [*begin, *end) of the pass input; false when the
// block has no chunk (the second pass launches an upper bound of blocks).
template <typename T>
__device__ __forceinline__ bool part_chunk(const PartPassT<T>& p, uint32_t blk, uint32_t* seg,
                                           uint64_t* begin, uint64_t* end) {
  const uint64_t C = p.P.chunk;
  if (p.level == 1) {
    const uint64_t b = (uint64_t)blk * C;
    if (b >= p.n) return false;
    *seg = 0;
    *begin = b;
    *end = b + C < p.n ? b + C : p.n;
    return true;
  }
  (void)C;
  // A second-pass range of len words is cut into k chunks of equal length
  // (cuts on whole lines), k chosen by part_scan1_kernel.
  const uint32_t* cf = p.M.chunk_first;
  if (blk >= cf[p.P.fan1]) return false;
  const uint32_t lo = p.M.chunk_seg[blk];  // cf[lo] <= blk < cf[lo + 1]
  const uint64_t s0 = p.M.seg_start[lo], len = p.M.seg_len[lo];
  const uint32_t j = blk - cf[lo], k = cf[lo + 1] - cf[lo];
  auto cut = [&](uint32_t i) -> uint64_t {
    return i >= k ? len : ((uint64_t)i * len / k) & ~(uint64_t)(kLineWords - 1);
  };
  *seg = lo;
  *begin = s0 + cut(j);
  *end = s0 + cut(j + 1);
  return true;
}

// Exclusive prefix sums of v[0, count) into out[], count <= 4 * NT; returns
// the total.  Every thread of the block must call it.  wt: NT / 64 words of
// LDS.
template <int NT, typename T, typename PI, typename PO>
__device__ __forceinline__ T block_exclusive_scan(PI v, PO out, uint32_t count, T* wt) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  T x[4];
  T s = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t idx = tid * 4 + j;
    x[j] = idx < count ? (T)v[idx] : (T)0;
    s += x[j];
  }
  T inc = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(inc, off, 64);
    if (lane >= (uint32_t)off) inc += y;
  }
  if (lane == 63) wt[wave] = inc;
  __syncthreads();
  T before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const T t = wt[w];
    if ((uint32_t)w < wave) before += t;
    total += t;
  }
  T run = before + inc - s;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t idx = tid * 4 + j;
    if (idx < count) out[idx] = run;
    run += x[j];
  }
  __syncthreads();
  return total;
}

// Clears the counters a build accumulates into and the build status.
__global__ void part_clear_kernel(PartMeta M, uint32_t fan1, uint32_t levels,
                                  uint32_t* __restrict__ status) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t j = i; j < fan1; j += stride) M.total1[j] = 0;
  if (levels == 2)
    for (uint32_t j = i; j < fan1 * kFan2; j += stride) M.total2[j] = 0;
  if (i == 0) *M.head = 0;
  if (i < 8) status[i] = 0;
}

// Keys reserved by the tables (the empty marker; for 64-bit keys also the
// slot-lock key).
__device__ __forceinline__ bool reserved_key(uint32_t k) { return k == kEmptyKey; }
__device__ __forceinline__ bool reserved_key(uint64_t k) { return k >= ~0ull - 1; }

// Pairs staged per sub-tile for keys and values of type T (LDS holds two
// sub-tile arrays of T: 128 KB for 4- and for 8-byte words).
template <typename T>
constexpr int sub_tile() { return sizeof(T) == 4 ? kPartSub : kPartSub / 2; }

// Digit counts of the pairs [begin, end) of in_k: stored in hrow (for the
// scatter's reservations) and added to tot, rounded up to whole lines of
// pad_to words when the scatter writes lines (pad_to = 0: not rounded);
// returns whether the range held a reserved key.  With skip_pads, empty
// keys are padding and not counted.  Every thread of the block calls it.
template <typename T, typename DigitFn>
__device__ __forceinline__ bool hist_range(const T* __restrict__ in_k, uint64_t begin,
                                           uint64_t end, uint32_t fan, DigitFn digit,
                                           uint32_t* __restrict__ hrow,
                                           unsigned long long* __restrict__ tot,
                                           bool skip_pads = false, uint32_t pad_to = 0) {
  __shared__ uint32_t cnt[kMaxFan];
  for (uint32_t d = threadIdx.x; d < fan; d += kPassBlock) cnt[d] = 0;
  __syncthreads();
  bool sentinel = false;
  constexpr int U = 8;
  // 32-bit offsets from the range's start (a range is one chunk, under 2^32
  // pairs), so the address arithmetic stays in single registers
  const T* __restrict__ kb = in_k + begin;
  const uint32_t len = (uint32_t)(end - begin);
  for (uint32_t base = 0; base < len; base += U * kPassBlock) {
    T k[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      // branch-free loads: offsets past the end re-read the last pair
      const uint32_t o = base + j * kPassBlock + threadIdx.x;
      k[j] = kb[o < len ? o : len - 1];
    }
    // a full group of U pairs per thread is counted without per-pair guards,
    // so the counting atomics issue back to back
    auto count_group = [&](auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const uint32_t o = base + j * kPassBlock + threadIdx.x;
        if ((FULL || o < len) && !(skip_pads && reserved_key(k[j]))) {
          sentinel |= reserved_key(k[j]);
          atomicAdd(&cnt[digit(k[j])], 1u);
        }
      }
    };
    if (base + U * kPassBlock <= len) count_group(std::integral_constant<bool, true>());
    else count_group(std::integral_constant<bool, false>());
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < fan; d += kPassBlock) {
    const uint32_t c = cnt[d];
    hrow[d] = c;
    if (c) atomicAdd(&tot[d], (unsigned long long)(pad_to ? line_pad(c, pad_to) : c));
  }
  return sentinel;
}

// Digit counts of one chunk: stored per chunk (for the scatter's
// reservations) and added to the range's digit totals.
template <typename T>
__global__ __launch_bounds__(kPassBlock) void part_hist_kernel(PartPassT<T> p) {
  uint32_t seg;
  uint64_t begin, end;
  if (!part_chunk(p, blockIdx.x, &seg, &begin, &end)) return;
  uint32_t* h = (p.level == 1 ? p.M.hist1 : p.M.hist2) + (uint64_t)blockIdx.x * p.fan;
  unsigned long long* tot = p.level == 1 ? p.M.total1 : p.M.total2 + (uint64_t)seg * kFan2;
  const PartPlan& P = p.P;
  const uint32_t level = p.level;
  const bool sentinel = hist_range(p.in_k, begin, end, p.fan,
                                   [&](T k) { return part_digit(P, level, k); }, h, tot,
                                   p.padded != 0, p.lines ? line_words<T>() : 0u);
  if (level == 1 && sentinel) atomicOr(p.status, kFlagSentinel);
}

// Status words 4-5 and 6-7 (64-bit): words the first and the second pass
// write, padding included.
constexpr int kStatusPass1Words = 4;
constexpr int kStatusPass2Words = 6;

// Chunks of the second pass: how many equal pieces each first-pass range
// (len[d] words of `words` in all) is cut into.  The pass's blocks run in
// rounds of `resident2` (one block per CU for the scatter), so the pass
// takes about ceil(chunks / resident2) times its longest chunk.  Candidate 0
// cuts each range into pieces of at most P.chunk words; candidates 1-4 aim
// at K = r * resident2 chunks in all (r around candidate 0's rounds) and give
// range d floor(len[d] * K / words) of them, at least 1 and at most one per
// 64 words, so their sum stays within K wherever the ranges are not tiny.
// The cheapest estimate wins (ties: fewer chunks); candidates over the
// workspace bound are skipped.  Every thread of the block calls it.
__device__ __forceinline__ void split_ranges(const PartPlan& P,
                                             const unsigned long long* __restrict__ len,
                                             unsigned long long words,
                                             unsigned long long* __restrict__ chunks) {
  constexpr int kCand = 5;
  __shared__ unsigned int sum[kCand], longest[kCand];
  __shared__ unsigned long long target[kCand];
  __shared__ int pick;
  const uint32_t R = P.resident2;
  // range lengths are below 2^32 words (positions are 32-bit)
  auto pieces = [&](int c, uint32_t l) -> uint32_t {
    if (l == 0) return 0;
    if (c == 0) return (uint32_t)(((uint64_t)l + P.chunk - 1) / P.chunk);
    uint32_t k = (uint32_t)((double)l * (double)target[c] / (double)words);
    const uint32_t most = l / 64 > 1 ? l / 64 : 1;
    k = k < 1 ? 1 : k;
    return k < most ? k : most;
  };
  // per-thread partial sums and maxima, reduced per wave, one LDS atomic
  // per wave (same-address atomics from every lane would serialize)
  auto wave_max = [](uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
  };
  const bool lead = (threadIdx.x & 63) == 0;
  if (threadIdx.x < kCand) {
    sum[threadIdx.x] = 0;
    longest[threadIdx.x] = 0;
  }
  __syncthreads();
  {
    uint32_t part = 0;
    for (uint32_t d = threadIdx.x; d < P.fan1; d += kPartBlock)
      part += (uint32_t)pieces(0, len[d]);
    part = wave_sum(part);
    if (lead) atomicAdd(&sum[0], part);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long rounds0 = R ? ((long long)sum[0] + R - 1) / R : 0;
    for (int c = 1; c < kCand; ++c) {
      const long long r = rounds0 + c - 2;
      target[c] = R && words ? (unsigned long long)(r > 1 ? r : 1) * R : 0;
    }
  }
  __syncthreads();
  for (int c = 0; c < kCand; ++c) {
    uint32_t part = 0, most = 0;
    if (c == 0 || target[c] != 0) {
      for (uint32_t d = threadIdx.x; d < P.fan1; d += kPartBlock) {
        const uint32_t l = (uint32_t)len[d];
        const uint32_t k = (uint32_t)pieces(c, l);
        part += k;
        if (k) most = max(most, (uint32_t)(((uint64_t)l + k - 1) / k));
      }
    }
    part = wave_sum(part);
    most = wave_max(most);
    if (lead) {
      if (c > 0) atomicAdd(&sum[c], part);
      atomicMax(&longest[c], most);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int best = 0;
    unsigned long long best_cost = ~0ull;
    for (int c = 0; c < kCand; ++c) {
      if (c > 0 && (target[c] == 0 || sum[c] > P.chunks2_cap)) continue;
      const unsigned long long rounds = R ? (sum[c] + R - 1) / R : 1;
      const unsigned long long cost = rounds * longest[c];
      if (cost < best_cost || (cost == best_cost && sum[c] < sum[best])) {
        best = c;
        best_cost = cost;
      }
    }
    pick = best;
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < P.fan1; d += kPartBlock)
    chunks[d] = pieces(pick, (uint32_t)len[d]);
  __syncthreads();
}

// First-pass totals -> output ranges.  One block.  With one pass the digits
// are the bins; with two, the ranges of the second pass and its chunk counts.
__global__ __launch_bounds__(kPartBlock) void part_scan1_kernel(PartPlan P, PartMeta M,
                                                                uint32_t* __restrict__ status) {
  __shared__ unsigned long long wt[kPartBlock / 64];
  __shared__ unsigned long long base[kMaxFan];
  __shared__ unsigned long long chunks[kMaxFan];
  const unsigned long long words =
      block_exclusive_scan<kPartBlock, unsigned long long>(M.total1, base, P.fan1, wt);
  if (threadIdx.x == 0)
    *reinterpret_cast<unsigned long long*>(status + kStatusPass1Words) = words;
  for (uint32_t d = threadIdx.x; d < P.fan1; d += kPartBlock) {
    const unsigned long long c = M.total1[d];
    M.cursor1[d] = base[d];
    if (P.levels == 1) {
      M.bin_start[d] = base[d];
      M.bin_len[d] = c;
    } else {
      M.seg_start[d] = base[d];
      M.seg_len[d] = c;
    }
  }
  if (P.levels == 1) return;          // uniform
  split_ranges(P, M.total1, words, chunks);
  const unsigned long long total =
      block_exclusive_scan<kPartBlock, unsigned long long>(chunks, base, P.fan1, wt);
  for (uint32_t d = threadIdx.x; d < P.fan1; d += kPartBlock) {
    M.chunk_first[d] = (uint32_t)base[d];
    for (uint64_t c = base[d]; c < base[d] + chunks[d]; ++c) M.chunk_seg[c] = d;
  }
  if (threadIdx.x == 0) M.chunk_first[P.fan1] = (uint32_t)total;
}

// Words of padding a line-writing second pass adds to one chunk, at most.
constexpr uint64_t kLinePadPerChunk2 = (uint64_t)kFan2 * (kLineWords - 1);

// Second-pass totals -> bin ranges.  One block per first-pass range.  The
// range's output starts where its input does; when the pass writes lines,
// rounded up to a whole line (the first pass may not have padded) and
// shifted by a line per earlier range and by the most padding the earlier
// ranges' chunks can add, so ranges never overlap.
__global__ __launch_bounds__(kPartBlock) void part_scan2_kernel(PartPlan P, PartMeta M,
                                                                uint32_t* __restrict__ status) {
  __shared__ unsigned long long wt[kPartBlock / 64];
  __shared__ unsigned long long base[kFan2];
  const uint32_t s = blockIdx.x;
  const unsigned long long* tot = M.total2 + (uint64_t)s * kFan2;
  const unsigned long long words =
      block_exclusive_scan<kPartBlock, unsigned long long>(tot, base, kFan2, wt);
  if (threadIdx.x == 0 && words)
    atomicAdd(reinterpret_cast<unsigned long long*>(status + kStatusPass2Words), words);
  const uint32_t d = threadIdx.x;          // kPartBlock == kFan2
  const unsigned long long start =
      P.lines2 ? (M.seg_start[s] + kLineWords - 1) / kLineWords * kLineWords +
                     (unsigned long long)kLineWords * s + kLinePadPerChunk2 * M.chunk_first[s]
               : M.seg_start[s];
  const unsigned long long pos = start + base[d];
  M.cursor2[(uint64_t)s * kFan2 + d] = pos;
  const uint64_t bin = (uint64_t)s * kFan2 + d;
  if (bin < P.nbins) {
    M.bin_start[bin] = pos;
    M.bin_len[bin] = tot[d];
  }
}

// Writes the pairs [begin, end) in digit order: reserves the range of every
// digit (hrow holds the range's digit counts, cur the digits' next output
// positions), then per sub-tile ranks pairs by digit in LDS and stores each
// digit's run contiguously.  The next sub-tile's loads are issued before the
// current one is ranked, so they overlap the on-chip work.  Positions are
// below 2^32 (the partitioned path takes fewer than 2^32 pairs).  Every
// thread of the block calls it.
template <typename T, typename DigitFn>
__device__ __forceinline__ void scatter_range(const T* __restrict__ in_k,
                                              const T* __restrict__ in_v, uint64_t begin,
                                              uint64_t end, uint32_t fan, DigitFn digit,
                                              const uint32_t* __restrict__ hrow,
                                              unsigned long long* __restrict__ cur,
                                              T* __restrict__ out_k, T* __restrict__ out_v,
                                              bool padded = false) {
  constexpr int SUB = sub_tile<T>();
  constexpr int PER = SUB / kPassBlock;
  __shared__ T sk[SUB];
  __shared__ T sv[SUB];
  __shared__ uint8_t sd[kScatterStageDigits ? SUB : 1];
  __shared__ uint32_t cnt[kMaxFan];
  __shared__ uint32_t start[kMaxFan];
  __shared__ uint32_t run[kMaxFan];
  __shared__ uint32_t wt[kPassBlock / 64];
  // With at most 256 digits each staged pair's digit is kept as a byte, so
  // the write-out needs no second hash evaluation.
  const bool staged = kScatterStageDigits && fan <= 256;
  for (uint32_t d = threadIdx.x; d < fan; d += kPassBlock) {
    const uint32_t c = hrow[d];
    run[d] = c ? (uint32_t)atomicAdd(&cur[d], (unsigned long long)c) : 0u;
    cnt[d] = 0;
  }
  // Loads are branch-free (offsets past the end re-read the last pair, and
  // those copies are never ranked), so the compiler can leave the next
  // sub-tile's loads in flight while the current one is ranked.  Offsets
  // are 32-bit, from the range's start (a range is one chunk, under 2^32
  // pairs), so the address arithmetic stays in single registers.
  const T* __restrict__ kb = in_k + begin;
  const T* __restrict__ vb = in_v + begin;
  const uint32_t len = (uint32_t)(end - begin);
  const uint32_t last = len - 1;
  T k[PER], v[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const uint32_t o = j * kPassBlock + threadIdx.x;
    k[j] = kb[o < len ? o : last];
    v[j] = vb[o < len ? o : last];
  }
  for (uint32_t sub = 0; sub < len; sub += SUB) {
    T nk[PER], nv[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t o = sub + SUB + j * kPassBlock + threadIdx.x;
      nk[j] = kb[o < len ? o : last];
      nv[j] = vb[o < len ? o : last];
    }
    // cnt was cleared before the loop or by the previous sub-tile, ahead of
    // a barrier
    __syncthreads();
    // rank within the digit (< 2^14) and digit (< 2^10) share a register
    static_assert(SUB <= (1 << 22) && kMaxFan <= 1024, "rank and digit packing");
    const uint32_t count = len - sub < (uint32_t)SUB ? len - sub : (uint32_t)SUB;
    // One body, instantiated for a full sub-tile without padding (no
    // per-pair guards, so the compiler can issue a thread's LDS accesses
    // back to back instead of one guarded block at a time) and for the
    // rest; and for digits staged in LDS or recomputed.  Both choices are
    // uniform over the block.  With padded input, empty keys are padding of
    // a line-writing pass: not ranked, not written.
    auto body = [&](auto full_tag, auto staged_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      constexpr bool STAGED = decltype(staged_tag)::value;
      uint32_t rd[PER];   // ~0: no pair
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const uint32_t i = j * kPassBlock + threadIdx.x;
        rd[j] = ~0u;
        if (FULL || (i < count && !(padded && reserved_key(k[j])))) {
          const uint32_t d = digit(k[j]);
          rd[j] = (atomicAdd(&cnt[d], 1u) << 10) | d;
        }
      }
      __syncthreads();
      // staged pairs of this sub-tile (count, less any padding)
      const uint32_t staged_n = block_exclusive_scan<kPassBlock, uint32_t>(cnt, start, fan, wt);
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        if (FULL || rd[j] != ~0u) {
          const uint32_t d = rd[j] & 1023u;
          const uint32_t pos = start[d] + (rd[j] >> 10);
          sk[pos] = k[j];
          sv[pos] = v[j];
          if (STAGED) sd[pos] = (uint8_t)d;
        }
      }
      __syncthreads();
      // start[d] becomes the offset from a staged position to its output
      // position; the digit's run advances and its count clears for the
      // next sub-tile (whose ranking follows this write-out without a
      // barrier)
      for (uint32_t d = threadIdx.x; d < fan; d += kPassBlock) {
        const uint32_t c = cnt[d];
        start[d] = run[d] - start[d];
        run[d] += c;
        cnt[d] = 0;
      }
      __syncthreads();
      // fixed trip count (no inner loop), so the prefetched loads stay in
      // flight across the stores
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const uint32_t i = j * kPassBlock + threadIdx.x;
        if (FULL || i < staged_n) {
          const T key = sk[i];
          const uint32_t d = STAGED ? (uint32_t)sd[i] : digit(key);
          const uint32_t dst = start[d] + i;
          out_k[dst] = key;
          out_v[dst] = sv[i];
        }
      }
    };
    using yes = std::integral_constant<bool, true>;
    using no = std::integral_constant<bool, false>;
    const bool full = count == (uint32_t)SUB && !padded;
    if (staged) {
      if (full) body(yes(), yes());
      else body(no(), yes());
    } else {
      if (full) body(yes(), no());
      else body(no(), no());
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      k[j] = nk[j];
      v[j] = nv[j];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kPassBlock, kScatterBlocksPerCU) void part_scatter_kernel(PartPassT<T> p) {
  uint32_t seg;
  uint64_t begin, end;
  if (!part_chunk(p, blockIdx.x, &seg, &begin, &end)) return;
  const uint32_t* h = (p.level == 1 ? p.M.hist1 : p.M.hist2) + (uint64_t)blockIdx.x * p.fan;
  unsigned long long* cur = p.level == 1 ? p.M.cursor1 : p.M.cursor2 + (uint64_t)seg * kFan2;
  const PartPlan& P = p.P;
  const uint32_t level = p.level;
  scatter_range(p.in_k, p.in_v, begin, end, p.fan,
                [&](T k) { return part_digit(P, level, k); }, h, cur, p.out_k, p.out_v,
                p.padded != 0);
}

// Per-digit work items packed beside the digit counts, for one scan: the
// digit's new pairs (< 2^16) in the low half, its items in the high half.
// An item is a whole line to write (all pairs and carried words when the
// sub-tile ends the range, else only the full lines); a digit with pairs
// but no full line gets one item that only carries them.
template <uint32_t LW>
struct LinePack {
  const uint32_t* cnt;
  const uint32_t* carry;
  bool last;
  __device__ __forceinline__ uint32_t lines(uint32_t d) const {
    const uint32_t tot = carry[d] + cnt[d];
    return last ? (tot + LW - 1) / LW : tot / LW;
  }
  __device__ __forceinline__ uint32_t operator[](uint32_t d) const {
    const uint32_t n = lines(d);
    return ((n ? n : (cnt[d] ? 1u : 0u)) << 16) | cnt[d];
  }
};

// Pair staged in LDS by the line-writing scatter, and the padding pair.
template <typename T> struct LinePair;
template <> struct LinePair<uint32_t> {
  using type = uint2;
  __device__ static uint2 make(uint32_t k, uint32_t v) { return make_uint2(k, v); }
  __device__ static uint2 pad() { return make_uint2(kEmptyKey, 0u); }
};
template <> struct LinePair<uint64_t> {
  using type = u64x2;
  __device__ static u64x2 make(uint64_t k, uint64_t v) { return u64x2{k, v}; }
  __device__ static u64x2 pad() { return u64x2{kEmpty64, 0ull}; }
};

// scatter_range for at most kLineMaxFan digits that stores whole 128-byte
// lines only (32 pairs of 4-byte words, or 16 of 8-byte words; 8 K or 4 K
// pairs per sub-tile).  Each digit's range of this chunk (hrow[d] pairs) is
// reserved rounded up to whole lines at a line-aligned cursor.  Per
// sub-tile the pairs are ranked and staged by digit as in scatter_range; a
// digit's output then continues with the pairs carried from the previous
// sub-tile followed by its staged pairs, and only the lines that are full
// are written (half a wave or a quarter per line, from a descriptor built
// per line); the remainder (less than a line) is carried in LDS, copied
// there by the digit's first item after it has read the pairs carried
// before.  The range's last sub-tile writes the remainder too, padded with
// the empty key and value 0.  With padded input, empty keys are padding and
// skipped.  Partial lines, each written twice from different times or
// different workgroups, are what slows the plain scatter.  Every thread of
// the block calls it.
template <typename T, typename DigitFn>
__device__ __forceinline__ void scatter_lines_range(const T* __restrict__ in_k,
                                                    const T* __restrict__ in_v,
                                                    uint64_t begin, uint64_t end, uint32_t fan,
                                                    bool padded, DigitFn digit,
                                                    const uint32_t* __restrict__ hrow,
                                                    unsigned long long* __restrict__ cur,
                                                    T* __restrict__ out_k,
                                                    T* __restrict__ out_v) {
  using Pair = typename LinePair<T>::type;
  constexpr int SUB = kLineSub * 4 / (int)sizeof(T);
  constexpr int PER = SUB / kPassBlock;
  constexpr uint32_t LW = line_words<T>();
  constexpr uint32_t FMAX = kLineMaxFan;
  // items of one sub-tile, at most: every word once, plus a partial line
  // (or a carry-only item) per digit
  constexpr int MAXLINES = (SUB + FMAX * (LW - 1)) / LW + FMAX;
  static_assert(SUB < (1 << 16) && MAXLINES < (1 << 16), "packed scan fields");
  static_assert(kPassBlock % LW == 0, "half waves per block");
  // staged pairs [0, SUB), then LW carried pairs per digit, key and value
  // side by side (one 8-byte LDS access per pair)
  __shared__ Pair skv[SUB + FMAX * LW];
  __shared__ uint32_t cnt[FMAX];          // new pairs per digit in this sub-tile
  __shared__ uint32_t pre[FMAX];          // packed exclusive prefix (first line, first staged pair)
  __shared__ uint32_t carry[FMAX];        // carried words per digit
  __shared__ uint32_t run[FMAX];          // next output position per digit (line-aligned)
  // per item: .x output position of its line; .y index (into skv) of the
  // staged pair for lane 0; .z bits 0-14 index of the carried pair for
  // lane 0, bits 15-28 the staged index of the first pair to carry on;
  // .w bits 0-5 lanes taking carried pairs, 8-13 lanes taking carried or
  // staged pairs (the rest write padding), 16-21 pairs to carry on, 24-28
  // their offset in the digit's carry slots, bit 31 set when the item
  // writes a line
  static_assert(SUB + FMAX * LW < (1 << 15) && SUB < (1 << 14), "item fields");
  __shared__ uint4 line_desc[MAXLINES];
  __shared__ uint32_t wt[kPassBlock / 64];
  const uint32_t tid = threadIdx.x, hl = tid / LW, l = tid % LW;
  for (uint32_t d = tid; d < fan; d += kPassBlock) {
    const uint32_t c = hrow[d];
    run[d] = c ? (uint32_t)atomicAdd(&cur[d], (unsigned long long)line_pad(c, LW)) : 0u;
    cnt[d] = 0;
    carry[d] = 0;
  }
  const T* __restrict__ kb = in_k + begin;
  const T* __restrict__ vb = in_v + begin;
  const uint32_t len = (uint32_t)(end - begin);
  const uint32_t last_i = len - 1;
  T k[PER], v[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const uint32_t o = j * kPassBlock + tid;
    k[j] = kb[o < len ? o : last_i];
    v[j] = vb[o < len ? o : last_i];
  }
  for (uint32_t sub = 0; sub < len; sub += SUB) {
    T nk[PER], nv[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t o = sub + SUB + j * kPassBlock + tid;
      nk[j] = kb[o < len ? o : last_i];
      nv[j] = vb[o < len ? o : last_i];
    }
    // the previous sub-tile's carries and cleared counts are in place
    __syncthreads();
    const uint32_t count = len - sub < (uint32_t)SUB ? len - sub : (uint32_t)SUB;
    const bool last = len - sub <= (uint32_t)SUB;
    // rank within the digit (< 2^13) above the digit (< 2^8); ~0 = no pair
    uint32_t rd[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t i = j * kPassBlock + tid;
      rd[j] = ~0u;
      if (i < count && !(padded && reserved_key(k[j]))) {
        const uint32_t d = digit(k[j]);
        rd[j] = (atomicAdd(&cnt[d], 1u) << 8) | d;
      }
    }
    __syncthreads();
    const uint32_t total =
        block_exclusive_scan<kPassBlock, uint32_t>(LinePack<LW>{cnt, carry, last}, pre, fan, wt);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (rd[j] != ~0u) {
        const uint32_t d = rd[j] & 255u;
        const uint32_t pos = (pre[d] & 0xFFFFu) + (rd[j] >> 8);
        skv[pos] = LinePair<T>::make(k[j], v[j]);
      }
    }
    // items of each digit; then the digit's output advances by the lines
    // written, its carry count becomes the new one and its pair count
    // clears (the items hold everything the write-out needs)
    for (uint32_t d = tid; d < fan; d += kPassBlock) {
      const LinePack<LW> lp{cnt, carry, last};
      const uint32_t p = pre[d], cf = carry[d], c = cnt[d];
      const uint32_t first = p >> 16, p_low = p & 0xFFFFu;
      const uint32_t lines = lp.lines(d), tot = cf + c;
      // pairs carried on: those past the last whole line, all staged when
      // a line is written, else appended after the carried ones
      const uint32_t nc_new = last ? 0u : tot - lines * LW;
      const uint32_t t_src = lines ? p_low + lines * LW - cf : p_low;
      const uint32_t t_off = lines ? 0u : cf;
      const uint32_t t_cnt = lines ? nc_new : c;
      const uint32_t items = lines ? lines : (c ? 1u : 0u);
      for (uint32_t q = 0; q < items; ++q) {
        // words of this line: e = q * LW + lane over [carried, staged, padding)
        const uint32_t e0 = q * LW;
        const uint32_t nc = cf > e0 ? cf - e0 : 0u;                 // carried lanes
        const uint32_t nw = cf + c > e0 ? min(cf + c - e0, LW) : 0u; // carried + staged lanes
        const uint32_t carry_on = q == 0 ? (t_cnt << 16) | (t_off << 24) : 0u;
        line_desc[first + q] =
            make_uint4(run[d] + e0, p_low + e0 - cf, (SUB + d * LW) | (t_src << 15),
                       nc | (nw << 8) | carry_on | (lines ? 0x80000000u : 0u));
      }
      run[d] += lines * LW;
      carry[d] = nc_new;
      cnt[d] = 0;
    }
    __syncthreads();
    // whole lines: carried pairs first, then the staged pairs, then
    // padding; the digit's first item then carries its remainder on (the
    // staging is only read here, and only this item touches the digit's
    // carry slots)
    const uint32_t nitems = total >> 16;
    for (uint32_t it = hl; it < nitems; it += kPassBlock / LW) {
      const uint4 ld = line_desc[it];
      const uint32_t cbase = ld.z & 0x7FFFu;
      if (ld.w >> 31) {
        Pair kv = LinePair<T>::pad();
        if (l < ((ld.w >> 8) & 63u)) kv = skv[l < (ld.w & 63u) ? cbase + l : ld.y + l];
        out_k[ld.x + l] = kv.x;
        out_v[ld.x + l] = kv.y;
      }
      if (l < ((ld.w >> 16) & 63u))
        skv[cbase + ((ld.w >> 24) & 31u) + l] = skv[(ld.z >> 15) + l];
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      k[j] = nk[j];
      v[j] = nv[j];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kPassBlock, 1) void part_scatter_lines_kernel(PartPassT<T> p) {
  uint32_t seg;
  uint64_t begin, end;
  if (!part_chunk(p, blockIdx.x, &seg, &begin, &end)) return;
  const uint32_t* h = (p.level == 1 ? p.M.hist1 : p.M.hist2) + (uint64_t)blockIdx.x * p.fan;
  unsigned long long* cur = p.level == 1 ? p.M.cursor1 : p.M.cursor2 + (uint64_t)seg * kFan2;
  const PartPlan& P = p.P;
  const uint32_t level = p.level;
  scatter_lines_range(p.in_k, p.in_v, begin, end, p.fan, p.padded != 0,
                      [&](T k) { return part_digit(P, level, k); }, h, cur, p.out_k,
                      p.out_v);
}

struct BinArgs {
  uint64_t* slots;               // the table
  uint32_t* keys;                // partitioned pairs; evicted pairs are written back in place
  uint32_t* vals;
  uint32_t* status;
  uint32_t max_chain;
  uint32_t rng_seed;
  uint32_t cap;                  // pairs a first bucket takes on chip (b; iceberg: t)
  PartPlan P;
  PartMeta M;
};

// One bin in LDS.  Each pair claims the next slot of its first bucket (a
// local atomic on the bucket's load) while the bucket holds fewer than cap
// pairs.  EVICT (cuckoo, cap = B): a pair that finds the bucket full makes
// the cuckoo step of Section III-A on chip: after a barrier (every claimed
// slot is then written) it exchanges itself with a random slot of the
// bucket, and the evicted pair is written to the front of the bin's input
// range, to continue at its next bucket in the overflow kernel.  Without
// EVICT (iceberg, cap = t, Section III-C) the pair itself goes there, to
// continue at its secondary choices.  The bin's buckets, empty slots
// included, are then stored whole.  The bin is buckets [first, first + nb)
// of the table (nb <= R <= slots / B); its pairs are keys/vals[s0, s0 +
// len).  Returns (in every thread) the number of pairs written back; raises
// flags in *status.  Every thread of the block calls it.
template <int B, bool EVICT = true>
__device__ __forceinline__ uint32_t place_bin(uint64_t* __restrict__ slots,
                                              uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ vals, const Hash32& H,
                                              uint32_t R, uint64_t first, uint32_t nb,
                                              uint64_t s0, uint64_t len, uint32_t max_chain,
                                              uint32_t rng_seed, uint32_t salt, uint32_t cap,
                                              uint32_t* __restrict__ status) {
  constexpr int S = bin_slots<B>();
  constexpr int RMAX = S / B;                    // buckets per bin, at most
  __shared__ u64x2 tbl2[S / 2];
  // [RMAX + lane]: counter of a lane without a pair (one per lane, so a
  // wave's idle lanes do not serialize on one address)
  __shared__ uint32_t load[RMAX + 64];
  __shared__ unsigned long long spill[64];       // target of the stores of those lanes
  __shared__ uint32_t ovf;
  unsigned long long* tbl = reinterpret_cast<unsigned long long*>(tbl2);
  const u64x2 e2 = {kEmptyPair, kEmptyPair};
  for (uint32_t i = threadIdx.x; i < (R * B + 1) / 2; i += kBinBlock) tbl2[i] = e2;
  for (uint32_t i = threadIdx.x; i < R; i += kBinBlock) load[i] = 0;
  if (threadIdx.x == 0) ovf = 0;
  uint32_t rng = rng_seed ^ (salt * 0x9E3779B9u) ^ (threadIdx.x * 0x85EBCA6Bu);
  if (rng == 0) rng = 0x2545F491u;
  uint32_t flags = 0;
  // the bin's pairs, addressed by 32-bit offsets (the partitioned path
  // takes fewer than 2^32 pairs)
  uint32_t* __restrict__ kb = keys + s0;
  uint32_t* __restrict__ vb = vals + s0;
  const uint32_t n_bin = (uint32_t)len;
  __syncthreads();
  for (uint32_t r0 = 0; r0 < n_bin; r0 += kBinBlock * kBinPer) {
    uint32_t k[kBinPer], v[kBinPer], full[kBinPer];
#pragma unroll
    for (int j = 0; j < kBinPer; ++j) {
      // branch-free loads: offsets past the end re-read the bin's last pair
      const uint32_t i = r0 + j * kBinBlock + threadIdx.x;
      k[j] = kb[i < n_bin ? i : n_bin - 1];
      v[j] = vb[i < n_bin ? i : n_bin - 1];
    }
#pragma unroll
    for (int j = 0; j < kBinPer; ++j) {
      full[j] = ~0u;
      const uint32_t i = r0 + j * kBinBlock + threadIdx.x;
      // No branch per pair: a lane without a pair (past the bin's end, or
      // padding) counts on a spare counter and stores to a spare word of
      // its own, so the claims of a thread's pairs issue back to back.
      // lb < nb by construction of the partition; otherwise the build
      // fails.
      const uint32_t lb = hash32(H, 0, k[j]) - (uint32_t)first;
      // the empty key marks padding of a line-writing pass (a caller's
      // empty key has already failed the build)
      const bool valid = i < n_bin && k[j] != kEmptyKey;
      const bool inside = lb < nb;
      if (valid && !inside) flags |= kFlagFailed;
      const bool claim = valid && inside;
      const uint32_t s = atomicAdd(&load[claim ? lb : (uint32_t)RMAX + __lane_id()], 1u);
      const bool placed = claim && s < cap;
      unsigned long long* dst = placed ? &tbl[lb * B + s] : &spill[__lane_id()];
      *dst = ((unsigned long long)v[j] << 32) | k[j];
      if (claim && !placed) full[j] = lb;
    }
    // Every claimed slot is written, and every pair of this round has been
    // read: evicted pairs go to positions below the running eviction count.
    __syncthreads();
    // all exchanges first, then the stores of the evicted pairs (a store
    // between two exchanges would make each exchange wait for it)
#pragma unroll
    for (int j = 0; j < kBinPer; ++j) {
      if (full[j] != ~0u) {
        if constexpr (!EVICT) {
          full[j] = atomicAdd(&ovf, 1u);
        } else if (max_chain == 0) {
          flags |= kFlagFailed;
          full[j] = ~0u;
        } else {
          rng = xorshift32(rng);
          const unsigned long long old = atomicExch(
              &tbl[full[j] * B + rng % (uint32_t)B], ((unsigned long long)v[j] << 32) | k[j]);
          full[j] = atomicAdd(&ovf, 1u);
          k[j] = (uint32_t)old;
          v[j] = (uint32_t)(old >> 32);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kBinPer; ++j) {
      if (full[j] != ~0u) {
        kb[full[j]] = k[j];
        vb[full[j]] = v[j];
      }
    }
  }
  __syncthreads();
  const uint64_t words = (uint64_t)nb * B;
  u64x2* dst2 = reinterpret_cast<u64x2*>(slots + first * B);
  for (uint32_t i = threadIdx.x; i < words / 2; i += kBinBlock) dst2[i] = tbl2[i];
  if ((words & 1) && threadIdx.x == 0) slots[first * B + words - 1] = tbl[words - 1];
  if (flags) atomicOr(status, flags);
  return ovf;
}

template <int B, bool EVICT = true>
__global__ __launch_bounds__(kBinBlock) void bin_place_kernel(BinArgs a) {
  const uint32_t R = 1u << a.P.bin_shift;        // buckets per bin of this plan
  const uint32_t bin = blockIdx.x;
  const uint64_t first = (uint64_t)bin * R;
  const uint32_t nb = (uint64_t)a.P.H.m - first < (uint64_t)R ? (uint32_t)(a.P.H.m - first) : R;
  const uint32_t ovf =
      place_bin<B, EVICT>(a.slots, a.keys, a.vals, a.P.H, R, first, nb, a.M.bin_start[bin],
                          a.M.bin_len[bin], a.max_chain, a.rng_seed, bin, a.cap, a.status);
  if (threadIdx.x == 0) {
    a.M.ovf_len[bin] = ovf;
    if (ovf) atomicAdd(a.status + 1, ovf);       // evicted pairs of the build
  }
}

struct OverflowArgs {
  BuildArgs32 g;                 // keys / vals = the partitioned arrays
  PartMeta M;
  uint32_t nbins;
};

__device__ __forceinline__ uint32_t part_queue_pop(unsigned int* head) {
  unsigned int v = 0;
  if (__lane_id() == 0) v = atomicAdd(head, 1u);
  return (uint32_t)__builtin_amdgcn_readfirstlane(v);
}

// Cuckoo insertion (Section III-A) of the pairs evicted during placement,
// each continuing at its next bucket with one exchange counted; waves take
// bins from a queue.
// The bucket reads of this phase are summed into status words 2-3 (one
// atomic per wave).
template <int B, int W>
__global__ __launch_bounds__(kBlock) void overflow_build_kernel(OverflowArgs a) {
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
    flags |= cuckoo_build_range<B, W, true, true>(
        a.g, r, a.g.rng_seed ^ salt ^ (bin * 0x85EBCA6Bu), &probes);
  }
  if (flags) atomicOr(a.g.status, flags);
  const uint32_t total = wave_sum(probes);
  if (__lane_id() == 0 && total)
    atomicAdd(reinterpret_cast<unsigned long long*>(a.g.status + 2), (unsigned long long)total);
}

}  // namespace bht
