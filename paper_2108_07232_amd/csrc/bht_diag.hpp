// Diagnostic kernels: random-access ceilings of the device, used as the
// practical roofline for bucket probes and slot atomics.
#pragma once
#include "bht_kernels.hpp"

namespace bht {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

// Random reads of LB-byte aligned blocks (LB / 16 lanes x 16 bytes each)
// with no table logic: at LB = 128 the access pattern of one bucket probe,
// hence the practical ceiling for probes on a buffer of this size.
// The block index costs a few integer operations (no division), so the
// loop is bound by memory, not by index arithmetic.
template <int LB>
__global__ __launch_bounds__(kBlock) void diag_gather_kernel(const uint64_t* __restrict__ buf,
                                                            uint32_t units, uint64_t reads,
                                                            uint64_t seed,
                                                            unsigned long long* __restrict__ sink) {
  constexpr int W = LB / 16;
  const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t tiles = ((uint64_t)gridDim.x * blockDim.x) / W;
  const uint32_t lt = threadIdx.x % W;
  const uint64_t M = fastmod32_constant(units);
  uint64_t acc = 0;
  for (uint64_t r = gtid / W; r < reads; r += tiles) {
    const uint64_t u = fastmod32((uint32_t)mix64(r ^ seed), M, units);
    const u64x2 v = reinterpret_cast<const u64x2*>(buf + u * (LB / 8))[lt];
    acc ^= v.x ^ v.y;
  }
  if (acc == 0x9E3779B97F4A7C15ull) atomicAdd(sink, 1ull);
}

// Random 8-byte compare-and-swaps that never change memory (the swapped-in
// value equals the expected one): the device's rate for slot atomics.
__global__ __launch_bounds__(kBlock) void diag_cas_kernel(uint64_t* __restrict__ buf,
                                                         uint32_t slots, uint64_t ops,
                                                         uint64_t seed,
                                                         unsigned long long* __restrict__ sink) {
  const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t M = fastmod32_constant(slots);
  uint64_t acc = 0;
  for (uint64_t r = gtid; r < ops; r += stride) {
    const uint64_t s = fastmod32((uint32_t)mix64(r ^ seed), M, slots);
    acc ^= cas64(buf + s, 0x5555555555555555ull, 0x5555555555555555ull);
  }
  if (acc == 0x9E3779B97F4A7C15ull) atomicAdd(sink, 1ull);
}

// Streaming ceiling: reads n16 16-byte words of src in order and, with
// WRITE, writes them to dst (a device copy); without, folds them into one
// value (a read-only pass).  Each block streams one contiguous 64 KB
// chunk, four words per lane in flight per step (on this part contiguous
// per-block chunks stream faster than a grid-wide stride).  The streaming
// phases of the partitioned build are priced against these.
constexpr uint64_t kStreamChunk = 4096;          // 16-byte words per block
template <bool WRITE>
__global__ __launch_bounds__(kBlock) void diag_stream_kernel(const u64x2* __restrict__ src,
                                                            u64x2* __restrict__ dst, uint64_t n16,
                                                            unsigned long long* __restrict__ sink) {
  constexpr int U = 4;
  const uint64_t b0 = (uint64_t)blockIdx.x * kStreamChunk;
  const uint64_t b1 = b0 + kStreamChunk < n16 ? b0 + kStreamChunk : n16;
  uint64_t acc = 0;
  for (uint64_t i = b0 + threadIdx.x; i < b1; i += (uint64_t)kBlock * U) {
    u64x2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t idx = i + (uint64_t)u * kBlock;
      if (idx < b1) v[u] = src[idx];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t idx = i + (uint64_t)u * kBlock;
      if (idx < b1) {
        if (WRITE) dst[idx] = v[u];
        else acc ^= v[u].x ^ v[u].y;
      }
    }
  }
  if (!WRITE && acc == 0x9E3779B97F4A7C15ull) atomicAdd(sink, 1ull);
}

}  // namespace bht
