/*
 * CPU oracle for static bucketed hash tables — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, single-threaded, deliberately unoptimised statement of what the
 * method of "Better GPU Hash Tables" (Awad et al., arXiv 2108.07232)
 * computes.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it; the product library never does.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Slot layout (the same layout the GPU library documents, so that a layout
 * built by either side can be checked or queried by the other):
 *   32-bit tables: one uint64 per slot, key in the low 32 bits, value in the
 *                  high 32 bits; an empty slot is all ones.
 *   64-bit tables: two uint64 per slot, key then value; empty is all ones.
 * Bucket i occupies slots [i*b, (i+1)*b).
 */
#ifndef BHT_ORACLE_H
#define BHT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BCHT = 0, ORC_BP2HT = 1, ORC_IHT = 2, ORC_CHT1 = 3, ORC_BCHT_LB = 4 };

enum {
  ORC_OK = 0,
  ORC_FAILED = 1,       /* chain cap reached / every candidate bucket full */
  ORC_SENTINEL = 2,     /* an input key equals the reserved empty key      */
  ORC_BADARG = 3
};

typedef struct {
  int32_t scheme;       /* ORC_BCHT, ORC_BP2HT, ORC_IHT, ORC_CHT1, ORC_BCHT_LB   */
  uint32_t b;           /* slots per (primary) bucket                            */
  uint64_t m;           /* number of (primary) buckets                           */
  uint32_t h;           /* number of hash functions (IHT: 3 = primary, s0, s1)  */
  uint32_t max_chain;   /* cuckoo: maximum evictions per insertion               */
  uint64_t a[4];        /* hash multipliers a_i                                   */
  uint64_t c[4];        /* hash offsets b_i (named c to avoid clashing with b)   */
  uint32_t threshold;   /* IHT: primary used while its load is below this        */
  uint32_t b2;          /* IHT secondary level: slots per bucket (0 = one level) */
  uint64_t m2;          /* IHT secondary level: number of buckets                */
  uint32_t rng_seed;    /* eviction-victim xorshift32 seed (nonzero)             */
  uint32_t mock_n;      /* >0: hash values come from mock_hash instead (tests)   */
  const uint32_t* mock_hash; /* mock_hash[key*h + i] = bucket of hash i, key < mock_n */
  uint32_t iht_early_exit; /* IHT find: a miss in a primary holding fewer than    */
                           /* threshold keys ends the query (see orc_find32)      */
} orc_params;

/* ((a*k + c) mod 4294967291) mod m, Section VII hash family. */
uint64_t orc_hash32(uint64_t a, uint64_t c, uint32_t k, uint64_t m);
/* ((a*k + c) mod (2^61 - 1)) mod m, the same family over 64-bit keys. */
uint64_t orc_hash64(uint64_t a, uint64_t c, uint64_t k, uint64_t m);

/* Element-wise orc_hash32 / orc_hash64 over an array of keys. */
void orc_hash32_many(uint64_t a, uint64_t c, const uint32_t* k, uint64_t n, uint64_t m,
                     uint64_t* out);
void orc_hash64_many(uint64_t a, uint64_t c, const uint64_t* k, uint64_t n, uint64_t m,
                     uint64_t* out);

/* Number of uint64 words the table occupies (both levels). */
uint64_t orc_table_words(const orc_params* p, int wide);

/* Serial bulk build: table must hold orc_table_words() words; it is first
 * filled with empty slots.  probes (may be NULL) receives the number of
 * bucket reads.  Returns ORC_OK, ORC_FAILED, ORC_SENTINEL or ORC_BADARG. */
int orc_build32(const orc_params* p, const uint32_t* keys, const uint32_t* vals,
                uint64_t n, uint64_t* table, uint64_t* probes);
int orc_build64(const orc_params* p, const uint64_t* keys, const uint64_t* vals,
                uint64_t n, uint64_t* table, uint64_t* probes);

/* One insertion into an existing 32-bit layout (rng: eviction generator
 * state).  Returns ORC_OK, ORC_FAILED, ORC_SENTINEL or ORC_BADARG. */
int orc_insert32(const orc_params* p, uint64_t* table, uint32_t key, uint32_t val,
                 uint32_t* rng, uint64_t* probes);

/* Serial bulk find on a built layout.  A miss writes value = all ones and
 * found = 0.  per_query_probes (may be NULL) receives each query's probes. */
void orc_find32(const orc_params* p, const uint64_t* table, const uint32_t* q,
                uint64_t nq, uint32_t* out_v, uint8_t* out_f, uint64_t* probes,
                uint8_t* per_query_probes);
void orc_find64(const orc_params* p, const uint64_t* table, const uint64_t* q,
                uint64_t nq, uint64_t* out_v, uint8_t* out_f, uint64_t* probes,
                uint8_t* per_query_probes);

/* Section III-A's cuckoo insertion split at its first exchange, to replay
 * other schedules of the same steps (BCHT and CHT1 tables):
 * orc_exchange32 makes the first step of inserting (key, val) when its
 * first bucket H_0(key) is full: an exchange with a random slot (the
 * generator advanced once), the evicted pair returned in *ev_key, *ev_val;
 * ORC_BADARG if that bucket has room.  orc_continue32 finishes the
 * insertion of a pair just evicted from bucket from_bucket after `chain`
 * exchanges: it continues at H_{(j+1) mod h}, j the lowest index whose
 * hash names from_bucket (ORC_BADARG if none does). */
int orc_exchange32(const orc_params* p, uint64_t* table, uint32_t key, uint32_t val,
                   uint32_t* rng, uint32_t* ev_key, uint32_t* ev_val);
int orc_continue32(const orc_params* p, uint64_t* table, uint32_t key, uint32_t val,
                   uint64_t from_bucket, uint32_t chain, uint32_t* rng, uint64_t* probes);

/* Plain definition of a lookup over the input pairs: sort + binary search. */
void orc_brute_find32(const uint32_t* keys, const uint32_t* vals, uint64_t n,
                      const uint32_t* q, uint64_t nq, uint32_t* out_v, uint8_t* out_f);
void orc_brute_find64(const uint64_t* keys, const uint64_t* vals, uint64_t n,
                      const uint64_t* q, uint64_t nq, uint64_t* out_v, uint8_t* out_f);

/* The same lookups as a sort-merge join (linear time; nq < 2^32), for
 * checking every query of full-size batches. */
void orc_join_find32(const uint32_t* keys, const uint32_t* vals, uint64_t n,
                     const uint32_t* q, uint64_t nq, uint32_t* out_v, uint8_t* out_f);
void orc_join_find64(const uint64_t* keys, const uint64_t* vals, uint64_t n,
                     const uint64_t* q, uint64_t nq, uint64_t* out_v, uint8_t* out_f);

/* Layout invariants I1..I6 (see orc_check32 in oracle.c).  Returns 0 when
 * all hold, else the number of the first violated invariant, with a message
 * in msg. */
int orc_check32(const orc_params* p, const uint64_t* table, const uint32_t* keys,
                const uint32_t* vals, uint64_t n, char* msg, int msglen);
int orc_check64(const orc_params* p, const uint64_t* table, const uint64_t* keys,
                const uint64_t* vals, uint64_t n, char* msg, int msglen);

/* Marsaglia's xorshift32 (shifts 13, 17, 5): one step from state x. */
uint32_t orc_xorshift32(uint32_t x);

#ifdef __cplusplus
}
#endif
#endif
