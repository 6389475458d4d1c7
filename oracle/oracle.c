/*
 * CPU oracle for static bucketed hash tables — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, serial, unoptimised statement of the method of "Better GPU Hash
 * Tables" (Awad, Ashkiani, Porumbescu, Farach-Colton, Owens; arXiv
 * 2108.07232).  Each function cites the passage it follows.  Keys are
 * inserted one at a time in input order, so no concurrency rule (CAS retry,
 * tile queue) appears here: only the per-key algorithm of Section III and
 * Section V.  Only tests/, the smoke check and the benchmark's CPU baseline
 * may load this file's library; the product library never does.
 *
 * Readings taken where the paper is silent or its listings are garbled are
 * listed in the design notes; the ones that change arithmetic are repeated
 * at the function they affect.
 */
#include "oracle.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define P32 4294967291ULL            /* Section VII: p = 4294967291 */
#define P61 ((1ULL << 61) - 1ULL)    /* 64-bit keys: Mersenne prime 2^61 - 1 */
#define EMPTY32 0xFFFFFFFFu          /* Section V: sentinel = uint32 maximum */
#define EMPTY64 0xFFFFFFFFFFFFFFFFULL
#define EMPTY_PAIR 0xFFFFFFFFFFFFFFFFULL

/* ------------------------------------------------------------------ hash */

/* Section VII: h(k; a, b) = ((a k + b) mod p) mod L, L = number of buckets.
 * With a, b < p < 2^32 and k < 2^32, a*k + b < 2^64: exact in uint64. */
uint64_t orc_hash32(uint64_t a, uint64_t c, uint32_t k, uint64_t m) {
  uint64_t x = a * (uint64_t)k + c;
  return (x % P32) % m;
}

/* Same family for 64-bit keys with p = 2^61 - 1 (not in the paper: a
 * 32-bit prime would map many distinct 64-bit keys to the same buckets).
 * 128-bit intermediate, plain remainder. */
uint64_t orc_hash64(uint64_t a, uint64_t c, uint64_t k, uint64_t m) {
  unsigned __int128 x = (unsigned __int128)a * k + c;
  return (uint64_t)(x % P61) % m;
}

/* Marsaglia, "Xorshift RNGs" (2003), the 32-bit generator with shifts
 * (13, 17, 5).  Section V-B draws the eviction victim with it. */
uint32_t orc_xorshift32(uint32_t x) {
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}

/* ---------------------------------------------------------- table access */

typedef struct {
  uint64_t first_slot;   /* word index (32-bit) or slot index (64-bit) */
  uint32_t size;         /* slots in this bucket                        */
} bucket_ref;

/* Bucket chosen by hash function i for a key.  Hash 0 always indexes the
 * primary array.  For a two-level iceberg table (b2 > 0) hashes 1 and 2 are
 * the secondary choices and index the secondary array, which follows the
 * primary array in memory. */
static bucket_ref bucket_for(const orc_params* p, uint32_t i, uint64_t hv_primary,
                             uint64_t hv_secondary) {
  bucket_ref r;
  if (p->scheme == ORC_IHT && p->b2 > 0 && i > 0) {
    r.first_slot = p->m * p->b + hv_secondary * p->b2;
    r.size = p->b2;
  } else {
    r.first_slot = hv_primary * p->b;
    r.size = p->b;
  }
  return r;
}

static bucket_ref bucket32(const orc_params* p, uint32_t i, uint32_t key) {
  if (p->mock_n) {
    uint64_t v = p->mock_hash[(uint64_t)key * p->h + i];
    return bucket_for(p, i, v, v);
  }
  uint64_t mp = orc_hash32(p->a[i], p->c[i], key, p->m);
  uint64_t ms = (p->b2 > 0) ? orc_hash32(p->a[i], p->c[i], key, p->m2) : 0;
  return bucket_for(p, i, mp, ms);
}

static bucket_ref bucket64(const orc_params* p, uint32_t i, uint64_t key) {
  uint64_t mp = orc_hash64(p->a[i], p->c[i], key, p->m);
  uint64_t ms = (p->b2 > 0) ? orc_hash64(p->a[i], p->c[i], key, p->m2) : 0;
  return bucket_for(p, i, mp, ms);
}

static uint32_t key_of(uint64_t slot) { return (uint32_t)(slot & 0xFFFFFFFFu); }
static uint32_t val_of(uint64_t slot) { return (uint32_t)(slot >> 32); }
static uint64_t pack(uint32_t k, uint32_t v) { return ((uint64_t)v << 32) | k; }

/* Listing 2, compute_load: number of slots whose key is not the sentinel. */
static uint32_t load32(const uint64_t* t, bucket_ref B) {
  uint32_t n = 0;
  for (uint32_t s = 0; s < B.size; s++)
    if (key_of(t[B.first_slot + s]) != EMPTY32) n++;
  return n;
}

static uint32_t load64(const uint64_t* t, bucket_ref B) {
  uint32_t n = 0;
  for (uint32_t s = 0; s < B.size; s++)
    if (t[2 * (B.first_slot + s)] != EMPTY64) n++;
  return n;
}

static int same_bucket(bucket_ref x, bucket_ref y) { return x.first_slot == y.first_slot; }

uint64_t orc_table_words(const orc_params* p, int wide) {
  uint64_t slots = p->m * p->b;
  if (p->scheme == ORC_IHT && p->b2 > 0) slots += p->m2 * p->b2;
  return wide ? 2 * slots : slots;
}

static int check_params(const orc_params* p) {
  if (p->b == 0 || p->m == 0 || p->h == 0 || p->h > 4) return 0;
  if (p->scheme == ORC_BP2HT && p->h != 2) return 0;
  if (p->scheme == ORC_IHT && p->h != 3) return 0;
  if (p->scheme == ORC_CHT1 && p->b != 1) return 0;
  if (p->scheme < ORC_BCHT || p->scheme > ORC_BCHT_LB) return 0;
  if (p->scheme == ORC_IHT && p->b2 > 0 && p->m2 == 0) return 0;
  return 1;
}

/* ------------------------------------------------------------ insertion */

/* The cuckoo walk of Section III-A from bucket B with `chain` exchanges
 * already made: the carried pair takes slot = load of a bucket with room;
 * at a full bucket it exchanges with a random slot and the evicted pair
 * continues at H_{(j+1) mod h}, j the lowest index whose hash names the
 * bucket it left; a full bucket met after max_chain exchanges fails. */
static int cuckoo_walk32(const orc_params* p, uint64_t* t, uint64_t cur, bucket_ref B,
                         uint32_t chain, uint32_t* rng, uint64_t* probes) {
  for (;;) {
    (*probes)++;
    uint32_t load = load32(t, B);
    if (load < B.size) {
      t[B.first_slot + load] = cur;
      return ORC_OK;
    }
    if (chain == p->max_chain) return ORC_FAILED;
    *rng = orc_xorshift32(*rng);
    uint32_t s = *rng % B.size;
    uint64_t victim = t[B.first_slot + s];
    t[B.first_slot + s] = cur;
    cur = victim;
    uint32_t j = 0;
    while (j < p->h && !same_bucket(bucket32(p, j, key_of(cur)), B)) j++;
    if (j == p->h) j = p->h - 1;  /* not stored in a candidate: restart at H0 */
    B = bucket32(p, (j + 1) % p->h, key_of(cur));
    chain++;
  }
}

/* Bucketed cuckoo insertion (Section III-A; Section V-B, BCHT insertion).
 * Start at H0.  A bucket with a free slot takes the pair at slot = load
 * (inserts fill each bucket as a prefix).  A full bucket exchanges the
 * carried pair with a random resident; the evicted pair continues at the
 * hash after the one that placed it there, that index being the lowest i
 * with H_i(key) equal to the bucket it left (footnote to Section III-A).
 * Reaching the eviction cap with a full bucket fails the build. */
static int insert_cuckoo32(const orc_params* p, uint64_t* t, uint32_t k, uint32_t v,
                           uint32_t* rng, uint64_t* probes) {
  return cuckoo_walk32(p, t, pack(k, v), bucket32(p, 0, k), 0, rng, probes);
}

/* Load-balanced bucketed cuckoo insertion (Section III-A: the variation
 * that inserts into the least loaded of the h buckets; Section IV,
 * placement strategies).  Read all h candidate buckets and place at slot =
 * load of the least loaded one with a free slot, ties going to the lowest
 * hash index.  When every candidate is full, exchange the carried pair with
 * a random resident of a random candidate bucket and continue with the
 * evicted pair; the bucket it was just evicted from is not chosen again
 * while another candidate differs from it.  The paper names no eviction
 * rule for this variation; this one is the random walk of d-ary cuckoo
 * hashing.  Reaching the eviction cap with every candidate full fails. */
static int insert_lb32(const orc_params* p, uint64_t* t, uint32_t k, uint32_t v,
                       uint32_t* rng, uint64_t* probes) {
  uint64_t cur = pack(k, v);
  uint64_t left = UINT64_MAX;           /* first slot of the bucket just left */
  uint32_t chain = 0;
  for (;;) {
    bucket_ref cand[4];
    uint32_t best = p->h, best_load = 0;
    for (uint32_t i = 0; i < p->h; i++) {
      cand[i] = bucket32(p, i, key_of(cur));
      (*probes)++;
      uint32_t l = load32(t, cand[i]);
      if (l < cand[i].size && (best == p->h || l < best_load)) {
        best = i;
        best_load = l;
      }
    }
    if (best < p->h) {
      t[cand[best].first_slot + best_load] = cur;
      return ORC_OK;
    }
    if (chain == p->max_chain) return ORC_FAILED;
    uint32_t eligible[4], ne = 0;
    for (uint32_t i = 0; i < p->h; i++)
      if (cand[i].first_slot != left) eligible[ne++] = i;
    *rng = orc_xorshift32(*rng);
    uint32_t j = ne ? eligible[*rng % ne] : *rng % p->h;
    *rng = orc_xorshift32(*rng);
    uint32_t s = *rng % cand[j].size;
    uint64_t victim = t[cand[j].first_slot + s];
    t[cand[j].first_slot + s] = cur;
    cur = victim;
    left = cand[j].first_slot;
    chain++;
  }
}

/* Power-of-two-choices insertion (Section III-B; Section V-C, Listing 5 as
 * corrected: the second bucket is H1's).  Read both buckets; if both are
 * full the build fails; otherwise place at slot = load of the less loaded
 * bucket, ties going to H0. */
static int insert_p2_32(const orc_params* p, uint64_t* t, uint32_t k, uint32_t v,
                        uint64_t* probes) {
  bucket_ref B0 = bucket32(p, 0, k), B1 = bucket32(p, 1, k);
  *probes += 2;
  uint32_t l0 = load32(t, B0), l1 = load32(t, B1);
  if (l0 == B0.size && l1 == B1.size) return ORC_FAILED;
  if (l0 <= l1) t[B0.first_slot + l0] = pack(k, v);
  else t[B1.first_slot + l1] = pack(k, v);
  return ORC_OK;
}

/* Iceberg insertion (Section III-C; Section V-D).  Reading taken: the
 * primary bucket is used while it holds fewer than t keys (the prose's
 * "fewer than t"); otherwise the two secondary buckets are read and the pair
 * goes to the less full one (ties to s0) unless both are full, in which case
 * the primary is used if it still has room; with no room anywhere the build
 * fails. */
static int insert_iceberg32(const orc_params* p, uint64_t* t, uint32_t k, uint32_t v,
                            uint64_t* probes) {
  bucket_ref P = bucket32(p, 0, k);
  (*probes)++;
  uint32_t lp = load32(t, P);
  if (lp < p->threshold && lp < P.size) {
    t[P.first_slot + lp] = pack(k, v);
    return ORC_OK;
  }
  bucket_ref S0 = bucket32(p, 1, k), S1 = bucket32(p, 2, k);
  *probes += 2;
  uint32_t l0 = load32(t, S0), l1 = load32(t, S1);
  if (l0 < S0.size || l1 < S1.size) {
    if (l0 <= l1) t[S0.first_slot + l0] = pack(k, v);
    else t[S1.first_slot + l1] = pack(k, v);
    return ORC_OK;
  }
  if (lp < P.size) {
    t[P.first_slot + lp] = pack(k, v);
    return ORC_OK;
  }
  return ORC_FAILED;
}

/* One insertion into an existing layout; rng is the eviction generator's
 * state, advanced once per eviction.  Building a table is filling it with
 * empty slots and inserting every pair in turn (Section III). */
int orc_insert32(const orc_params* p, uint64_t* table, uint32_t key, uint32_t val,
                 uint32_t* rng, uint64_t* probes) {
  uint64_t local_probes = 0;
  if (!probes) probes = &local_probes;
  if (!check_params(p)) return ORC_BADARG;
  if (key == EMPTY32) return ORC_SENTINEL;
  if (p->scheme == ORC_BP2HT) return insert_p2_32(p, table, key, val, probes);
  if (p->scheme == ORC_IHT) return insert_iceberg32(p, table, key, val, probes);
  if (p->scheme == ORC_BCHT_LB) return insert_lb32(p, table, key, val, rng, probes);
  return insert_cuckoo32(p, table, key, val, rng, probes);
}

int orc_exchange32(const orc_params* p, uint64_t* table, uint32_t key, uint32_t val,
                   uint32_t* rng, uint32_t* ev_key, uint32_t* ev_val) {
  if (!check_params(p) || (p->scheme != ORC_BCHT && p->scheme != ORC_CHT1)) return ORC_BADARG;
  bucket_ref B = bucket32(p, 0, key);
  if (load32(table, B) < B.size) return ORC_BADARG;
  *rng = orc_xorshift32(*rng);
  uint32_t s = *rng % B.size;
  uint64_t victim = table[B.first_slot + s];
  table[B.first_slot + s] = pack(key, val);
  *ev_key = key_of(victim);
  *ev_val = (uint32_t)(victim >> 32);
  return ORC_OK;
}

int orc_continue32(const orc_params* p, uint64_t* table, uint32_t key, uint32_t val,
                   uint64_t from_bucket, uint32_t chain, uint32_t* rng, uint64_t* probes) {
  uint64_t local_probes = 0;
  if (!probes) probes = &local_probes;
  if (!check_params(p) || (p->scheme != ORC_BCHT && p->scheme != ORC_CHT1)) return ORC_BADARG;
  if (from_bucket >= p->m) return ORC_BADARG;
  uint32_t j = 0;
  while (j < p->h && bucket32(p, j, key).first_slot != from_bucket * p->b) j++;
  if (j == p->h) return ORC_BADARG;     /* from_bucket is none of the key's candidates */
  return cuckoo_walk32(p, table, pack(key, val), bucket32(p, (j + 1) % p->h, key), chain, rng,
                       probes);
}

int orc_build32(const orc_params* p, const uint32_t* keys, const uint32_t* vals,
                uint64_t n, uint64_t* table, uint64_t* probes) {
  uint64_t local_probes = 0;
  if (!probes) probes = &local_probes;
  *probes = 0;
  if (!check_params(p)) return ORC_BADARG;
  uint64_t words = orc_table_words(p, 0);
  for (uint64_t w = 0; w < words; w++) table[w] = EMPTY_PAIR;
  for (uint64_t i = 0; i < n; i++)
    if (keys[i] == EMPTY32) return ORC_SENTINEL;
  uint32_t rng = p->rng_seed ? p->rng_seed : 0x9E3779B9u;
  for (uint64_t i = 0; i < n; i++) {
    int st = orc_insert32(p, table, keys[i], vals[i], &rng, probes);
    if (st != ORC_OK) return st;
  }
  return ORC_OK;
}

void orc_hash32_many(uint64_t a, uint64_t c, const uint32_t* k, uint64_t n, uint64_t m,
                     uint64_t* out) {
  for (uint64_t i = 0; i < n; i++) out[i] = orc_hash32(a, c, k[i], m);
}

void orc_hash64_many(uint64_t a, uint64_t c, const uint64_t* k, uint64_t n, uint64_t m,
                     uint64_t* out) {
  for (uint64_t i = 0; i < n; i++) out[i] = orc_hash64(a, c, k[i], m);
}

/* 64-bit keys and values: bucketed cuckoo only (16-byte slots). */
int orc_build64(const orc_params* p, const uint64_t* keys, const uint64_t* vals,
                uint64_t n, uint64_t* table, uint64_t* probes) {
  uint64_t local_probes = 0;
  if (!probes) probes = &local_probes;
  *probes = 0;
  if (!check_params(p) || p->scheme != ORC_BCHT || p->mock_n) return ORC_BADARG;
  uint64_t words = orc_table_words(p, 1);
  for (uint64_t w = 0; w < words; w++) table[w] = EMPTY64;
  for (uint64_t i = 0; i < n; i++)
    if (keys[i] == EMPTY64) return ORC_SENTINEL;
  uint32_t rng = p->rng_seed ? p->rng_seed : 0x9E3779B9u;
  for (uint64_t i = 0; i < n; i++) {
    uint64_t ck = keys[i], cv = vals[i];
    bucket_ref B = bucket64(p, 0, ck);
    uint32_t chain = 0;
    for (;;) {
      (*probes)++;
      uint32_t load = load64(table, B);
      if (load < B.size) {
        table[2 * (B.first_slot + load)] = ck;
        table[2 * (B.first_slot + load) + 1] = cv;
        break;
      }
      if (chain == p->max_chain) return ORC_FAILED;
      rng = orc_xorshift32(rng);
      uint64_t s = B.first_slot + rng % B.size;
      uint64_t vk = table[2 * s], vv = table[2 * s + 1];
      table[2 * s] = ck;
      table[2 * s + 1] = cv;
      ck = vk;
      cv = vv;
      uint32_t j = 0;
      while (j < p->h && !same_bucket(bucket64(p, j, ck), B)) j++;
      if (j == p->h) j = p->h - 1;
      B = bucket64(p, (j + 1) % p->h, ck);
      chain++;
    }
  }
  return ORC_OK;
}

/* ---------------------------------------------------------------- query */

/* Listing 2, find_key_value: the first slot holding the key. */
static int find_in32(const uint64_t* t, bucket_ref B, uint32_t q, uint32_t* v) {
  for (uint32_t s = 0; s < B.size; s++) {
    uint64_t e = t[B.first_slot + s];
    if (key_of(e) == q) {
      *v = val_of(e);
      return 1;
    }
  }
  return 0;
}

/* Queries.  Cuckoo (Section V-B, Listing 4 as corrected): probe H0, H1, ...
 * in order; stop on a hit, and stop with a miss after a bucket that lacks
 * the key and is not full (insertion order never skips a bucket with room).
 * Power-of-two (Section V-C), iceberg (Section III-C, V-D) and the
 * load-balanced cuckoo table (Section III-A: placement may skip a bucket
 * with room, so no early exit is valid): probe every candidate in order
 * until a hit, no early exit on room.  Iceberg with
 * iht_early_exit: a key goes to a secondary bucket only when its primary
 * already holds at least t keys (Section III-C), and loads never decrease,
 * so a miss in a primary that holds fewer than t keys proves absence and
 * ends the query after one probe.  A query equal to the sentinel is never a
 * stored key and misses without probing. */
void orc_find32(const orc_params* p, const uint64_t* table, const uint32_t* q,
                uint64_t nq, uint32_t* out_v, uint8_t* out_f, uint64_t* probes,
                uint8_t* per_query_probes) {
  uint64_t total = 0;
  for (uint64_t i = 0; i < nq; i++) {
    uint32_t v = EMPTY32, found = 0, pr = 0;
    if (q[i] != EMPTY32) {
      int early_exit = (p->scheme == ORC_BCHT || p->scheme == ORC_CHT1);
      for (uint32_t j = 0; j < p->h; j++) {
        bucket_ref B = bucket32(p, j, q[i]);
        pr++;
        if (find_in32(table, B, q[i], &v)) {
          found = 1;
          break;
        }
        if (early_exit && load32(table, B) < B.size) break;
        if (p->scheme == ORC_IHT && p->iht_early_exit && j == 0 &&
            load32(table, B) < p->threshold)
          break;
      }
    }
    if (!found) v = EMPTY32;
    out_v[i] = v;
    out_f[i] = (uint8_t)found;
    if (per_query_probes) per_query_probes[i] = (uint8_t)pr;
    total += pr;
  }
  if (probes) *probes = total;
}

void orc_find64(const orc_params* p, const uint64_t* table, const uint64_t* q,
                uint64_t nq, uint64_t* out_v, uint8_t* out_f, uint64_t* probes,
                uint8_t* per_query_probes) {
  uint64_t total = 0;
  for (uint64_t i = 0; i < nq; i++) {
    uint64_t v = EMPTY64;
    uint8_t found = 0, pr = 0;
    if (q[i] != EMPTY64) {
      for (uint32_t j = 0; j < p->h; j++) {
        bucket_ref B = bucket64(p, j, q[i]);
        pr++;
        for (uint32_t s = 0; s < B.size; s++) {
          if (table[2 * (B.first_slot + s)] == q[i]) {
            v = table[2 * (B.first_slot + s) + 1];
            found = 1;
            break;
          }
        }
        if (found || load64(table, B) < B.size) break;
      }
    }
    out_v[i] = found ? v : EMPTY64;
    out_f[i] = found;
    if (per_query_probes) per_query_probes[i] = pr;
    total += pr;
  }
  if (probes) *probes = total;
}

/* ------------------------------------------------------------ brute force */

/* Ascending sort of n uint64 values: least-significant-digit radix sort,
 * four passes over 16-bit digits (linear time keeps full-size checks short). */
static void sort_u64(uint64_t* a, uint64_t n) {
  if (n < 2) return;
  uint64_t* tmp = (uint64_t*)malloc(n * sizeof(uint64_t));
  uint64_t* count = (uint64_t*)malloc(65536 * sizeof(uint64_t));
  uint64_t *src = a, *dst = tmp;
  for (int pass = 0; pass < 4; pass++) {
    int shift = 16 * pass;
    memset(count, 0, 65536 * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; i++) count[(src[i] >> shift) & 0xFFFF]++;
    uint64_t sum = 0;
    for (int d = 0; d < 65536; d++) {
      uint64_t c = count[d];
      count[d] = sum;
      sum += c;
    }
    for (uint64_t i = 0; i < n; i++) dst[count[(src[i] >> shift) & 0xFFFF]++] = src[i];
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  /* four passes: the sorted data is back in a */
  free(tmp);
  free(count);
}

/* Section I: a lookup returns the value stored with the key, or reports the
 * key absent.  Sort the (key, value) pairs by key and binary-search. */
void orc_brute_find32(const uint32_t* keys, const uint32_t* vals, uint64_t n,
                      const uint32_t* q, uint64_t nq, uint32_t* out_v, uint8_t* out_f) {
  uint64_t* s = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  for (uint64_t i = 0; i < n; i++) s[i] = ((uint64_t)keys[i] << 32) | vals[i];
  sort_u64(s, n);
  for (uint64_t i = 0; i < nq; i++) {
    uint64_t lo = 0, hi = n;   /* first index with key >= q */
    while (lo < hi) {
      uint64_t mid = lo + (hi - lo) / 2;
      if ((uint32_t)(s[mid] >> 32) < q[i]) lo = mid + 1;
      else hi = mid;
    }
    if (lo < n && (uint32_t)(s[lo] >> 32) == q[i] && q[i] != EMPTY32) {
      out_v[i] = (uint32_t)s[lo];
      out_f[i] = 1;
    } else {
      out_v[i] = EMPTY32;
      out_f[i] = 0;
    }
  }
  free(s);
}

typedef struct { uint64_t k, v; } kv64;

static int cmp_kv64(const void* x, const void* y) {
  const kv64* a = (const kv64*)x;
  const kv64* b = (const kv64*)y;
  if (a->k != b->k) return (a->k > b->k) - (a->k < b->k);
  return (a->v > b->v) - (a->v < b->v);
}

void orc_brute_find64(const uint64_t* keys, const uint64_t* vals, uint64_t n,
                      const uint64_t* q, uint64_t nq, uint64_t* out_v, uint8_t* out_f) {
  kv64* s = (kv64*)malloc((n ? n : 1) * sizeof(kv64));
  for (uint64_t i = 0; i < n; i++) {
    s[i].k = keys[i];
    s[i].v = vals[i];
  }
  qsort(s, n, sizeof(kv64), cmp_kv64);
  for (uint64_t i = 0; i < nq; i++) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
      uint64_t mid = lo + (hi - lo) / 2;
      if (s[mid].k < q[i]) lo = mid + 1;
      else hi = mid;
    }
    if (lo < n && s[lo].k == q[i] && q[i] != EMPTY64) {
      out_v[i] = s[lo].v;
      out_f[i] = 1;
    } else {
      out_v[i] = EMPTY64;
      out_f[i] = 0;
    }
  }
  free(s);
}

/* Stable ascending sort of n uint64 values by bits [lo, 64):
 * least-significant-digit radix sort over 11-bit digits. */
static void sort_u64_from_bit(uint64_t* a, uint64_t n, int lo) {
  if (n < 2) return;
  uint64_t* tmp = (uint64_t*)malloc(n * sizeof(uint64_t));
  uint64_t count[2048];
  uint64_t *src = a, *dst = tmp;
  for (int shift = lo; shift < 64; shift += 11) {
    memset(count, 0, sizeof(count));
    for (uint64_t i = 0; i < n; i++) count[(src[i] >> shift) & 2047]++;
    uint64_t sum = 0;
    for (int d = 0; d < 2048; d++) {
      uint64_t c = count[d];
      count[d] = sum;
      sum += c;
    }
    for (uint64_t i = 0; i < n; i++) dst[count[(src[i] >> shift) & 2047]++] = src[i];
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  if (src != a) memcpy(a, src, n * sizeof(uint64_t));
  free(tmp);
}

/* Stable ascending sort of n (key, value) records by key: least-significant-
 * digit radix sort over 11-bit digits of the key. */
static void sort_kv64(kv64* a, uint64_t n) {
  if (n < 2) return;
  kv64* tmp = (kv64*)malloc(n * sizeof(kv64));
  uint64_t count[2048];
  kv64 *src = a, *dst = tmp;
  for (int shift = 0; shift < 64; shift += 11) {
    memset(count, 0, sizeof(count));
    for (uint64_t i = 0; i < n; i++) count[(src[i].k >> shift) & 2047]++;
    uint64_t sum = 0;
    for (int d = 0; d < 2048; d++) {
      uint64_t c = count[d];
      count[d] = sum;
      sum += c;
    }
    for (uint64_t i = 0; i < n; i++) dst[count[(src[i].k >> shift) & 2047]++] = src[i];
    kv64* t = src;
    src = dst;
    dst = t;
  }
  if (src != a) memcpy(a, src, n * sizeof(kv64));
  free(tmp);
}

/* The lookup of orc_brute_find32 computed as a sort-merge join: the pairs
 * sorted by key, the queries sorted by value together with their positions,
 * one merge pass matching equal keys, each answer written back to its
 * query's position.  Same results; linear time, so that every query of a
 * 2^28-query batch can be checked.  nq must be below 2^32. */
void orc_join_find32(const uint32_t* keys, const uint32_t* vals, uint64_t n,
                     const uint32_t* q, uint64_t nq, uint32_t* out_v, uint8_t* out_f) {
  uint64_t* s = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  uint64_t* qs = (uint64_t*)malloc((nq ? nq : 1) * sizeof(uint64_t));
  for (uint64_t i = 0; i < n; i++) s[i] = ((uint64_t)keys[i] << 32) | vals[i];
  for (uint64_t i = 0; i < nq; i++) qs[i] = ((uint64_t)q[i] << 32) | i;
  sort_u64_from_bit(s, n, 32);       /* by key */
  sort_u64_from_bit(qs, nq, 32);     /* by query */
  uint64_t j = 0;
  for (uint64_t r = 0; r < nq; r++) {
    const uint32_t qv = (uint32_t)(qs[r] >> 32);
    const uint64_t i = (uint32_t)qs[r];
    while (j < n && (uint32_t)(s[j] >> 32) < qv) j++;
    if (j < n && (uint32_t)(s[j] >> 32) == qv && qv != EMPTY32) {
      out_v[i] = (uint32_t)s[j];
      out_f[i] = 1;
    } else {
      out_v[i] = EMPTY32;
      out_f[i] = 0;
    }
  }
  free(s);
  free(qs);
}

/* orc_brute_find64 as a sort-merge join (see orc_join_find32). */
void orc_join_find64(const uint64_t* keys, const uint64_t* vals, uint64_t n,
                     const uint64_t* q, uint64_t nq, uint64_t* out_v, uint8_t* out_f) {
  kv64* s = (kv64*)malloc((n ? n : 1) * sizeof(kv64));
  kv64* qs = (kv64*)malloc((nq ? nq : 1) * sizeof(kv64));
  for (uint64_t i = 0; i < n; i++) {
    s[i].k = keys[i];
    s[i].v = vals[i];
  }
  for (uint64_t i = 0; i < nq; i++) {
    qs[i].k = q[i];
    qs[i].v = i;
  }
  sort_kv64(s, n);
  sort_kv64(qs, nq);
  uint64_t j = 0;
  for (uint64_t r = 0; r < nq; r++) {
    const uint64_t qv = qs[r].k, i = qs[r].v;
    while (j < n && s[j].k < qv) j++;
    if (j < n && s[j].k == qv && qv != EMPTY64) {
      out_v[i] = s[j].v;
      out_f[i] = 1;
    } else {
      out_v[i] = EMPTY64;
      out_f[i] = 0;
    }
  }
  free(s);
  free(qs);
}

/* ------------------------------------------------------------ invariants */

/*
 * Properties every correct layout has, whichever order concurrent inserts
 * took (layouts themselves legitimately differ between runs):
 *   I6  an empty slot is wholly empty (sentinel key implies sentinel value);
 *   I4  the occupied slots of every bucket form a prefix (inserts write at
 *       slot = load, Listings 3, 5, 6; exchanges only hit full buckets);
 *   I1  the stored pairs are exactly the input pairs, each once;
 *   I2  each stored key sits in one of its candidate buckets (Section III);
 *   I3  cuckoo: for a key in bucket B, every H_i(key) with i below the
 *       lowest index mapping to B is full (what makes the early-exit query
 *       of Section II-A correct);
 *   I5  iceberg: a key outside its primary bucket has a primary holding at
 *       least t keys (Section III-C).
 * Returns the number of the first violated invariant, or 0.
 */
int orc_check32(const orc_params* p, const uint64_t* t, const uint32_t* keys,
                const uint32_t* vals, uint64_t n, char* msg, int msglen) {
  if (!check_params(p)) {
    snprintf(msg, msglen, "bad parameters");
    return -1;
  }
  uint64_t words = orc_table_words(p, 0);
  uint64_t stored = 0;
  for (uint64_t w = 0; w < words; w++) {
    if (key_of(t[w]) == EMPTY32 && t[w] != EMPTY_PAIR) {
      snprintf(msg, msglen, "I6: slot %llu has the empty key with value %u",
               (unsigned long long)w, val_of(t[w]));
      return 6;
    }
    if (key_of(t[w]) != EMPTY32) stored++;
  }
  /* I4 over both levels */
  uint64_t levels = (p->scheme == ORC_IHT && p->b2 > 0) ? 2 : 1;
  for (uint64_t L = 0; L < levels; L++) {
    uint64_t base = L ? p->m * p->b : 0, nb = L ? p->m2 : p->m;
    uint32_t bs = L ? p->b2 : p->b;
    for (uint64_t B = 0; B < nb; B++) {
      int seen_empty = 0;
      for (uint32_t s = 0; s < bs; s++) {
        int empty = key_of(t[base + B * bs + s]) == EMPTY32;
        if (!empty && seen_empty) {
          snprintf(msg, msglen, "I4: level %llu bucket %llu slot %u occupied after a hole",
                   (unsigned long long)L, (unsigned long long)B, s);
          return 4;
        }
        if (empty) seen_empty = 1;
      }
    }
  }
  /* I1: same multiset of pairs */
  if (stored != n) {
    snprintf(msg, msglen, "I1: %llu occupied slots for %llu input pairs",
             (unsigned long long)stored, (unsigned long long)n);
    return 1;
  }
  uint64_t* a = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  uint64_t* b = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  uint64_t j = 0;
  for (uint64_t w = 0; w < words; w++)
    if (key_of(t[w]) != EMPTY32) a[j++] = ((uint64_t)key_of(t[w]) << 32) | val_of(t[w]);
  for (uint64_t i = 0; i < n; i++) b[i] = ((uint64_t)keys[i] << 32) | vals[i];
  sort_u64(a, n);
  sort_u64(b, n);
  for (uint64_t i = 0; i < n; i++) {
    if (a[i] != b[i]) {
      snprintf(msg, msglen, "I1: stored pair (%u,%u) differs from input pair (%u,%u)",
               (uint32_t)(a[i] >> 32), (uint32_t)a[i], (uint32_t)(b[i] >> 32), (uint32_t)b[i]);
      free(a);
      free(b);
      return 1;
    }
  }
  free(a);
  free(b);
  /* I2, I3, I5 per stored key */
  for (uint64_t w = 0; w < words; w++) {
    uint32_t k = key_of(t[w]);
    if (k == EMPTY32) continue;
    int in_secondary = (p->scheme == ORC_IHT && p->b2 > 0 && w >= p->m * p->b);
    uint64_t first = in_secondary ? p->m * p->b + ((w - p->m * p->b) / p->b2) * p->b2
                                  : (w / p->b) * p->b;
    uint32_t lowest = p->h;
    for (uint32_t i = 0; i < p->h; i++) {
      if (bucket32(p, i, k).first_slot == first) {
        lowest = i;
        break;
      }
    }
    if (lowest == p->h) {
      snprintf(msg, msglen, "I2: key %u at slot %llu is not in a candidate bucket", k,
               (unsigned long long)w);
      return 2;
    }
    if (p->scheme == ORC_BCHT || p->scheme == ORC_CHT1) {
      for (uint32_t i = 0; i < lowest; i++) {
        bucket_ref Bi = bucket32(p, i, k);
        if (load32(t, Bi) < Bi.size) {
          snprintf(msg, msglen, "I3: key %u stored via hash %u but bucket of hash %u has room",
                   k, lowest, i);
          return 3;
        }
      }
    }
    if (p->scheme == ORC_IHT && lowest > 0) {
      bucket_ref P = bucket32(p, 0, k);
      if (load32(t, P) < p->threshold && load32(t, P) < P.size) {
        snprintf(msg, msglen, "I5: key %u is in a secondary bucket but its primary is below t",
                 k);
        return 5;
      }
    }
  }
  snprintf(msg, msglen, "ok");
  return 0;
}

int orc_check64(const orc_params* p, const uint64_t* t, const uint64_t* keys,
                const uint64_t* vals, uint64_t n, char* msg, int msglen) {
  if (!check_params(p) || p->scheme != ORC_BCHT) {
    snprintf(msg, msglen, "bad parameters");
    return -1;
  }
  uint64_t slots = p->m * p->b, stored = 0;
  for (uint64_t s = 0; s < slots; s++) {
    if (t[2 * s] == EMPTY64 && t[2 * s + 1] != EMPTY64) {
      snprintf(msg, msglen, "I6: slot %llu has the empty key and a value", (unsigned long long)s);
      return 6;
    }
    if (t[2 * s] != EMPTY64) stored++;
  }
  for (uint64_t B = 0; B < p->m; B++) {
    int seen_empty = 0;
    for (uint32_t s = 0; s < p->b; s++) {
      int empty = t[2 * (B * p->b + s)] == EMPTY64;
      if (!empty && seen_empty) {
        snprintf(msg, msglen, "I4: bucket %llu slot %u occupied after a hole",
                 (unsigned long long)B, s);
        return 4;
      }
      if (empty) seen_empty = 1;
    }
  }
  if (stored != n) {
    snprintf(msg, msglen, "I1: %llu occupied slots for %llu input pairs",
             (unsigned long long)stored, (unsigned long long)n);
    return 1;
  }
  kv64* a = (kv64*)malloc((n ? n : 1) * sizeof(kv64));
  kv64* b = (kv64*)malloc((n ? n : 1) * sizeof(kv64));
  uint64_t j = 0;
  for (uint64_t s = 0; s < slots; s++)
    if (t[2 * s] != EMPTY64) {
      a[j].k = t[2 * s];
      a[j].v = t[2 * s + 1];
      j++;
    }
  for (uint64_t i = 0; i < n; i++) {
    b[i].k = keys[i];
    b[i].v = vals[i];
  }
  qsort(a, n, sizeof(kv64), cmp_kv64);
  qsort(b, n, sizeof(kv64), cmp_kv64);
  for (uint64_t i = 0; i < n; i++) {
    if (a[i].k != b[i].k || a[i].v != b[i].v) {
      snprintf(msg, msglen, "I1: stored pairs differ from input pairs at rank %llu",
               (unsigned long long)i);
      free(a);
      free(b);
      return 1;
    }
  }
  free(a);
  free(b);
  for (uint64_t s = 0; s < slots; s++) {
    uint64_t k = t[2 * s];
    if (k == EMPTY64) continue;
    uint64_t first = (s / p->b) * p->b;
    uint32_t lowest = p->h;
    for (uint32_t i = 0; i < p->h; i++)
      if (bucket64(p, i, k).first_slot == first) {
        lowest = i;
        break;
      }
    if (lowest == p->h) {
      snprintf(msg, msglen, "I2: key at slot %llu is not in a candidate bucket",
               (unsigned long long)s);
      return 2;
    }
    for (uint32_t i = 0; i < lowest; i++) {
      bucket_ref Bi = bucket64(p, i, k);
      if (load64(t, Bi) < Bi.size) {
        snprintf(msg, msglen, "I3: key stored via hash %u but bucket of hash %u has room",
                 lowest, i);
        return 3;
      }
    }
  }
  snprintf(msg, msglen, "ok");
  return 0;
}
