// Hash family of Section VII evaluated with exact integer arithmetic and no
// division: h(k; a, b) = ((a k + b) mod p) mod m.
//
// 32-bit keys, p = 2^32 - 5: a k + b < 2^64 is folded with 2^32 = 5 (mod p)
// twice and corrected once; the bucket index uses Lemire, Kaser and Kurz,
// "Faster remainder by direct computation" (2019), exact for 32-bit
// numerators and divisors with the 64-bit constant ceil(2^64 / m).
//
// 64-bit keys, q = 2^61 - 1: the 125-bit product is folded with 2^64 = 8 and
// 2^61 = 1 (mod q); the bucket index takes the quotient estimate
// floor(r * floor((2^64-1)/m) / 2^64), which is exact or one short for
// r < 2^61, and corrects it once.
#pragma once
#include <stdint.h>

namespace bht {

constexpr uint64_t kP32 = 4294967291ull;
constexpr uint64_t kP61 = (1ull << 61) - 1;

__host__ __device__ __forceinline__ uint64_t mul64hi(uint64_t x, uint64_t y) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(x, y);
#else
  return (uint64_t)(((unsigned __int128)x * y) >> 64);
#endif
}

__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t x, uint32_t y) {
  return (uint32_t)(((uint64_t)x * y) >> 32);
}

// x mod (2^32 - 5) for any 64-bit x.
__host__ __device__ __forceinline__ uint32_t mod_p32(uint64_t x) {
  uint64_t y = (uint64_t)(uint32_t)(x >> 32) * 5u + (uint32_t)x;   // < 6 * 2^32
  uint64_t z = (uint64_t)(uint32_t)(y >> 32) * 5u + (uint32_t)y;   // < 2^32 + 25
  return (uint32_t)(z >= kP32 ? z - kP32 : z);
}

// Divisor constant for fastmod32: ceil(2^64 / m); m = 1 gives 0, which
// yields remainder 0 as required.
__host__ __device__ __forceinline__ uint64_t fastmod32_constant(uint32_t m) {
  return UINT64_MAX / m + 1;
}

// r mod m for 32-bit r and m: the high 64 bits of (M r mod 2^64) * m.
__host__ __device__ __forceinline__ uint32_t fastmod32(uint32_t r, uint64_t M, uint32_t m) {
  uint64_t low = M * r;
  uint64_t t = (uint64_t)(uint32_t)(low >> 32) * m + mulhi32((uint32_t)low, m);
  return (uint32_t)(t >> 32);
}

struct Hash32 {
  uint32_t a[4];
  uint32_t c[4];
  uint64_t M;      // fastmod constant of m
  uint32_t m;      // number of buckets
  uint32_t h;      // number of hash functions
};

__host__ __device__ __forceinline__ uint32_t hash32(uint32_t a, uint32_t c, uint32_t k,
                                                    uint64_t M, uint32_t m) {
  return fastmod32(mod_p32((uint64_t)a * k + c), M, m);
}

__host__ __device__ __forceinline__ uint32_t hash32(const Hash32& H, int i, uint32_t k) {
  return hash32(H.a[i], H.c[i], k, H.M, H.m);
}

// (hi 2^64 + lo) mod (2^61 - 1) for hi < 2^61.
__host__ __device__ __forceinline__ uint64_t mod_p61(uint64_t hi, uint64_t lo) {
  uint64_t t0 = (lo & kP61) + (lo >> 61);
  uint64_t h8 = hi << 3;
  uint64_t t1 = (h8 & kP61) + (h8 >> 61);
  uint64_t s = t0 + t1;
  s = (s & kP61) + (s >> 61);
  return s >= kP61 ? s - kP61 : s;
}

struct Hash64 {
  uint64_t a[4];
  uint64_t c[4];
  uint64_t M;      // floor((2^64 - 1) / m)
  uint64_t m;
  uint32_t h;
};

__host__ __device__ __forceinline__ uint64_t hash64(uint64_t a, uint64_t c, uint64_t k,
                                                    uint64_t M, uint64_t m) {
  uint64_t lo = a * k;
  uint64_t hi = mul64hi(a, k);
  uint64_t lo2 = lo + c;
  hi += lo2 < lo;
  uint64_t r = mod_p61(hi, lo2);
  uint64_t q = mul64hi(r, M);
  uint64_t rem = r - q * m;
  return rem >= m ? rem - m : rem;
}

__host__ __device__ __forceinline__ uint64_t hash64(const Hash64& H, int i, uint64_t k) {
  return hash64(H.a[i], H.c[i], k, H.M, H.m);
}

}  // namespace bht
