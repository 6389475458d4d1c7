// Partitioned bulk build of the iceberg table (Section III-C).
//
// The radix passes and the bin placement are the cuckoo table's: pairs are
// grouped by the bin of their primary bucket, and a bin's primaries are
// filled on chip, each up to t pairs (the placement without eviction).  A
// pair that meets a primary already holding t pairs is written back to the
// front of its bin's input range and continues at its two secondary
// choices in the insertion kernel below, which is the concurrent iceberg
// insertion started after the primary step: first every pair whose primary
// is below t takes it, then the rest run the secondary step concurrently.
// The threshold rule holds exactly: a pair reaches the secondary level only
// once its primary holds t pairs.
#pragma once
#include "bht_partition.hpp"
#include "bht_schemes.hpp"

namespace bht {

struct IcebergOverflowArgs {
  SchemeArgs32 g;                // keys / vals = the partitioned arrays
  PartMeta M;
  uint32_t nbins;
};

// Bucket reads of this phase are summed into status words 2-3.
template <int B, int B2, int W>
__global__ __launch_bounds__(kBlock) void iceberg_overflow_kernel(IcebergOverflowArgs a) {
  uint32_t flags = 0, probes = 0;
  for (;;) {
    const uint32_t bin = part_queue_pop(a.M.head);
    if (bin >= a.nbins) break;
    const uint32_t len = a.M.ovf_len[bin];
    if (len == 0) continue;
    Range r;
    r.cursor = a.M.bin_start[bin];
    r.end = r.cursor + len;
    flags |= iceberg_build_range<B, B2, W, true, true>(a.g, r, &probes);
  }
  if (flags) atomicOr(a.g.status, flags);
  const uint32_t total = wave_sum(probes);
  if (__lane_id() == 0 && total)
    atomicAdd(reinterpret_cast<unsigned long long*>(a.g.status + 2), (unsigned long long)total);
}

}  // namespace bht
