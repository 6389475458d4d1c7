/*
 * Seeded synthetic workload generator (inputs only; no hash-table logic).
 *
 * Streams are splitmix64 (Steele, Lea, Flood 2014): output i of a stream
 * with seed s is mix(s + (i + 1) * 0x9E3779B97F4A7C15).  Distinct keys are
 * images of a counter under a keyed Feistel permutation (four rounds), so a
 * set of n keys needs no duplicate rejection; the all-ones sentinel is
 * cycle-walked out of the range.  Index permutations of [0, n) use the same
 * construction on the smallest even bit width covering n, cycle-walking
 * images that fall outside [0, n).
 */
#include <stdint.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t dg_splitmix64_at(uint64_t seed, uint64_t i) { return mix64(seed + (i + 1) * GAMMA); }

void dg_splitmix64(uint64_t seed, uint64_t start, uint64_t count, uint64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; i++) out[i] = mix64(seed + (start + i + 1) * GAMMA);
}

/* uint32 values: the high halves of a splitmix64 stream. */
void dg_values32(uint64_t seed, uint64_t count, uint32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; i++)
    out[i] = (uint32_t)(mix64(seed + (uint64_t)(i + 1) * GAMMA) >> 32);
}

static inline uint32_t fmix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  x *= 0xC2B2AE35u;
  x ^= x >> 16;
  return x;
}

/* Keyed bijection of [0, 2^32): four Feistel rounds on 16-bit halves. */
static inline uint32_t feistel32(uint32_t x, const uint32_t rk[4]) {
  uint32_t l = x >> 16, r = x & 0xFFFFu;
  for (int i = 0; i < 4; i++) {
    uint32_t f = fmix32(r * 0x9E3779B1u + rk[i]) >> 16;
    uint32_t nl = r;
    r = (l ^ f) & 0xFFFFu;
    l = nl;
  }
  return (l << 16) | r;
}

uint32_t dg_feistel32(uint32_t x, uint32_t k0, uint32_t k1, uint32_t k2, uint32_t k3) {
  const uint32_t rk[4] = {k0, k1, k2, k3};
  return feistel32(x, rk);
}

static inline uint32_t key32(uint64_t j, const uint32_t rk[4], uint32_t walk) {
  uint32_t y = feistel32((uint32_t)j, rk);
  return (y == 0xFFFFFFFFu) ? walk : y;
}

/* Images of indices start .. start+count-1: distinct, never 0xFFFFFFFF. */
void dg_keys32(const uint32_t rk[4], uint64_t start, uint64_t count, uint32_t* out) {
  const uint32_t walk = feistel32(0xFFFFFFFFu, rk);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; i++) out[i] = key32(start + (uint64_t)i, rk, walk);
}

static inline uint64_t fmix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xFF51AFD7ED558CCDULL;
  x ^= x >> 33;
  x *= 0xC4CEB9FE1A85EC53ULL;
  x ^= x >> 33;
  return x;
}

/* Keyed bijection of [0, 2^(2*half)): four Feistel rounds on half-bit halves. */
static inline uint64_t feistel_bits(uint64_t x, const uint64_t rk[4], int half) {
  const uint64_t mask = (half == 32) ? 0xFFFFFFFFULL : ((1ULL << half) - 1);
  uint64_t l = (x >> half) & mask, r = x & mask;
  for (int i = 0; i < 4; i++) {
    uint64_t f = fmix64(r * GAMMA + rk[i]) >> 32;
    uint64_t nl = r;
    r = (l ^ f) & mask;
    l = nl;
  }
  return (l << half) | r;
}

uint64_t dg_feistel64(uint64_t x, uint64_t k0, uint64_t k1, uint64_t k2, uint64_t k3) {
  const uint64_t rk[4] = {k0, k1, k2, k3};
  return feistel_bits(x, rk, 32);
}

/* Distinct uniform uint64 keys other than the all-ones empty-key sentinel:
 * images cycle-walked out of that one value. */
static inline uint64_t key64(uint64_t j, const uint64_t rk[4]) {
  uint64_t y = feistel_bits(j, rk, 32);
  while (y == 0xFFFFFFFFFFFFFFFFULL) y = feistel_bits(y, rk, 32);
  return y;
}

void dg_keys64(const uint64_t rk[4], uint64_t start, uint64_t count, uint64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; i++) out[i] = key64(start + (uint64_t)i, rk);
}

static int half_bits(uint64_t n) {
  int bits = 2;
  while (bits < 64 && (1ULL << bits) < n) bits += 2;
  return bits / 2;
}

/* P(i) for a keyed bijection P of [0, n), i < n. */
static inline uint64_t perm_at(uint64_t i, uint64_t n, const uint64_t rk[4], int half) {
  uint64_t y = feistel_bits(i, rk, half);
  while (y >= n) y = feistel_bits(y, rk, half);
  return y;
}

void dg_permutation(const uint64_t rk[4], uint64_t n, int64_t* out) {
  const int half = half_bits(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; i++) out[i] = (int64_t)perm_at((uint64_t)i, n, rk, half);
}

/* Queries over the key stream without materialising the keys: position i
 * takes j = Pmix(i); j < npos names positive j, the key of index
 * Ppos(j mod n) (a shuffle of the inserted keys, repeated if npos > n);
 * j >= npos names the (j - npos)-th key after the n inserted ones. */
void dg_queries32(const uint32_t rk_keys[4], const uint64_t rk_pos[4], uint64_t n,
                  const uint64_t rk_mix[4], uint64_t count, uint64_t npos, int shuffle,
                  uint32_t* out) {
  const uint32_t walk = feistel32(0xFFFFFFFFu, rk_keys);
  const int hn = half_bits(n ? n : 1), hc = half_bits(count ? count : 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; i++) {
    uint64_t j = shuffle ? perm_at((uint64_t)i, count, rk_mix, hc) : (uint64_t)i;
    uint64_t idx = (j < npos) ? perm_at(j % n, n, rk_pos, hn) : n + (j - npos);
    out[i] = key32(idx, rk_keys, walk);
  }
}

/* Key-stream position of every query dg_queries32/64 emit with the same
 * arguments: below n the query is inserted key number idx, from n on it is
 * an absent key.  Lets a caller state every expected lookup result from the
 * input arrays alone. */
void dg_query_sources(const uint64_t rk_pos[4], uint64_t n, const uint64_t rk_mix[4],
                      uint64_t count, uint64_t npos, int shuffle, uint64_t* out) {
  const int hn = half_bits(n ? n : 1), hc = half_bits(count ? count : 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; i++) {
    uint64_t j = shuffle ? perm_at((uint64_t)i, count, rk_mix, hc) : (uint64_t)i;
    out[i] = (j < npos) ? perm_at(j % n, n, rk_pos, hn) : n + (j - npos);
  }
}

void dg_queries64(const uint64_t rk_keys[4], const uint64_t rk_pos[4], uint64_t n,
                  const uint64_t rk_mix[4], uint64_t count, uint64_t npos, int shuffle,
                  uint64_t* out) {
  const int hn = half_bits(n ? n : 1), hc = half_bits(count ? count : 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; i++) {
    uint64_t j = shuffle ? perm_at((uint64_t)i, count, rk_mix, hc) : (uint64_t)i;
    uint64_t idx = (j < npos) ? perm_at(j % n, n, rk_pos, hn) : n + (j - npos);
    out[i] = key64(idx, rk_keys);
  }
}
