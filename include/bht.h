/*
 * bht — static bucketed hash tables on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library libbht.so.  Every entry point is extern "C", takes
 * plain pointers and sizes, and returns a bht_status (no exceptions cross
 * the boundary).  The operations are those of "Better GPU Hash Tables"
 * (Awad, Ashkiani, Porumbescu, Farach-Colton, Owens; arXiv 2108.07232):
 * a table is built once from an unordered list of key-value pairs and then
 * answers positive and negative lookups (Section I; Section III).
 *
 * Schemes (Section III, Section VII):
 *   BHT_BCHT   bucketed cuckoo table, h hash functions (3 by default), keys
 *              cuckoo between buckets, queries stop early at a bucket with
 *              room (Section III-A, Section V-B).
 *   BHT_BP2HT  bucketed power-of-two-choices table: two hashes, a key goes to
 *              the less loaded bucket and never moves (Section III-B, V-C).
 *   BHT_IHT    iceberg table: primary bucket while it holds fewer than t
 *              keys, else the less loaded of two secondary buckets (Section
 *              III-C, V-D); optionally with a separate secondary level.
 *   BHT_CHT1   cuckoo table with one slot per bucket (bucket_size = 1), the
 *              classic GPU cuckoo layout the paper compares against.
 *   BHT_BCHT_LB load-balanced bucketed cuckoo table (Section III-A's
 *              variation): a pair goes to the least loaded of its h buckets
 *              (ties to the lowest hash); when all are full it evicts a random
 *              resident of a random candidate other than the bucket it was
 *              just evicted from; queries probe every candidate (no early
 *              exit is valid).  32-bit keys, h = 2..4, bucket size 8/16/32.
 *
 * Device memory layout (library-owned, 256-byte aligned):
 *   32-bit tables: one 8-byte slot per pair, key in the low 32 bits and value
 *     in the high 32 bits; an empty slot is 0xFFFFFFFFFFFFFFFF.  Bucket i is
 *     slots [i*b, (i+1)*b); with b = 16 a bucket is one 128-byte line.  An
 *     iceberg table with a secondary level stores its m2*b2 secondary slots
 *     right after the m*b primary slots.
 *   64-bit tables: one 16-byte slot per pair (key word, then value word);
 *     empty key word is 0xFFFFFFFFFFFFFFFF; b = 8 makes a 128-byte bucket.
 *
 * Hash family (Section VII): H_i(k) = ((a_i*k + b_i) mod p) mod m with
 * p = 4294967291 for 32-bit keys; for 64-bit keys p = 2^61 - 1.  The caller
 * supplies the constants (a_i in [1, p-1], b_i in [0, p-1]).
 *
 * Keys: unique within one build (duplicates are memory-safe but which value
 * a lookup returns is then unspecified); the all-ones key is reserved as
 * the empty marker and is rejected.  Values are unrestricted: a lookup
 * reports presence separately from the value.
 *
 * Pointers named d_* are device pointers (hipMalloc or a framework's device
 * allocation) owned by the caller; the library reads or writes them only
 * during the call's stream work.  stream is a hipStream_t passed as void*
 * (NULL = the null stream).  Calls on one table are not thread-safe with
 * respect to each other, except concurrent finds on a built table.
 */
#ifndef BHT_H
#define BHT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bht_table bht_table;

typedef enum {
  BHT_BCHT = 0,
  BHT_BP2HT = 1,
  BHT_IHT = 2,
  BHT_CHT1 = 3,
  BHT_BCHT_LB = 4
} bht_scheme;

typedef enum {
  BHT_OK = 0,
  BHT_ERR_INVALID_ARG = 1,   /* null pointer, bad size, bad parameters          */
  BHT_ERR_CAPACITY = 2,      /* more pairs than slots                           */
  BHT_ERR_SENTINEL_KEY = 3,  /* an input key equals the reserved empty key      */
  BHT_ERR_BUILD_FAILED = 4,  /* eviction cap reached or every candidate full;   */
                             /* table contents unspecified: reseed and rebuild  */
  BHT_ERR_NOT_BUILT = 5,     /* find before a successful build                  */
  BHT_ERR_OOM = 6,           /* device allocation failed                        */
  BHT_ERR_HIP = 7,           /* a HIP runtime call failed (see bht_last_error)  */
  BHT_ERR_UNSUPPORTED = 8    /* parameter combination not implemented           */
} bht_status;

typedef struct {
  uint32_t num_hashes;        /* BCHT 1..4 (3 default), BP2HT 2, IHT 3, CHT1 1..4 */
  uint32_t key_bits;          /* 32 or 64 (64: BCHT only)                         */
  uint64_t a[4];              /* hash multipliers a_i                             */
  uint64_t b[4];              /* hash offsets b_i                                 */
  uint32_t rng_seed;          /* eviction victim generator seed (layout only)     */
  uint32_t max_chain;         /* cuckoo: evictions allowed per insertion (128)    */
  uint32_t iht_threshold;     /* IHT: primary used while its load is below this   */
  uint32_t iht_secondary_b;   /* IHT: slots per secondary bucket, 0 = one level   */
  uint64_t iht_secondary_m;   /* IHT: number of secondary buckets                 */
} bht_params;

/* Creates an empty table with m = ceil(capacity_slots / bucket_size)
 * buckets (Section III: capacity C = m*b).  bucket_size: 1 (CHT1), or 8, 16
 * or 32 (32-bit keys; BCHT also 4); 8 for 64-bit keys.  Allocates the slot
 * array with hipMalloc on the current device.  *out receives the table. */
bht_status bht_create(uint64_t capacity_slots, uint32_t bucket_size, bht_scheme scheme,
                      const bht_params* params, bht_table** out);

/* Bytes of device memory a table with these parameters needs (slot array
 * plus 256 bytes of build status), or 0 for invalid parameters. */
uint64_t bht_table_bytes(uint64_t capacity_slots, uint32_t bucket_size, bht_scheme scheme,
                         const bht_params* params);

/* As bht_create, but the table lives in caller-owned device memory
 * d_buffer of buffer_bytes (at least bht_table_bytes, 256-byte aligned),
 * for callers whose allocator owns HBM (e.g. a framework's caching
 * allocator).  The buffer must outlive the table; bht_destroy does not free
 * it. */
bht_status bht_create_in(uint64_t capacity_slots, uint32_t bucket_size, bht_scheme scheme,
                         const bht_params* params, void* d_buffer, uint64_t buffer_bytes,
                         bht_table** out);

/* Frees the table and, unless it was created with bht_create_in, its
 * memory (NULL is accepted). */
void bht_destroy(bht_table* t);

/* Replaces the hash constants and generator seed (after BUILD_FAILED,
 * Section VII: failed builds are retried with new constants).  The table
 * must be built again. */
bht_status bht_reseed(bht_table* t, const bht_params* params);

/* Bulk build from n pairs (d_keys[i], d_values[i]), structure-of-arrays
 * uint32.  Resets every slot to empty and inserts all pairs with the
 * scheme's algorithm (Section III; Section V).  Waits for the stream to read
 * the device status, so the return value reports BUILD_FAILED or
 * SENTINEL_KEY.  n = 0 is valid; n above the slot count is CAPACITY.
 * Placements that compare bucket loads (BP2HT, IHT secondaries) read the
 * candidates with device-scope loads and, when a concurrent placement takes
 * the chosen slot first, read both again and choose again; those re-reads
 * count as bucket reads in bht_build_counted. */
bht_status bht_build(bht_table* t, const uint32_t* d_keys, const uint32_t* d_values,
                     uint64_t n, void* stream);

/* As bht_build but only enqueues the work; bht_build_wait then waits for
 * the stream and returns the build's status.  Lets callers time or overlap
 * the build. */
bht_status bht_build_async(bht_table* t, const uint32_t* d_keys, const uint32_t* d_values,
                           uint64_t n, void* stream);
bht_status bht_build_wait(bht_table* t, void* stream);

/* Fills *out with a parameter set for `scheme` drawn from `seed`: the
 * scheme's default hash count (BP2HT 2, others 3), hash constants a_i
 * uniform in [1, p-1] and b_i uniform in [0, p-1] (Section VII: randomly
 * generated constants; p = 4294967291 for 32-bit keys, 2^61 - 1 for 64-bit
 * keys), a nonzero eviction generator seed and the 128-step eviction cap;
 * IHT threshold and secondary level are left 0 (one level, default
 * threshold).  All four constant pairs are drawn, so num_hashes may be
 * raised afterwards.  Deterministic in seed; key_bits must be 32 or 64. */
bht_status bht_params_from_seed(uint64_t seed, bht_scheme scheme, uint32_t key_bits,
                                bht_params* out);

/* Build with automatic reseeding (Section VII: a build that fails is
 * repeated with new hash constants).  Runs bht_build (32-bit tables) or
 * bht_build64 (64-bit tables; d_keys, d_values then point to uint64) with
 * the table's current parameters; after each BUILD_FAILED it replaces the
 * hash constants and generator seed by the draw of bht_params_from_seed for
 * seed + attempt - 1 (all other parameters kept) and builds again, at most
 * max_attempts builds in total (>= 1).  Returns the last build's status;
 * *attempts_out (may be NULL) receives the number of builds run.  The table
 * keeps the constants of the last attempt.  Synchronous, like bht_build. */
bht_status bht_build_retry(bht_table* t, const void* d_keys, const void* d_values, uint64_t n,
                           uint64_t seed, uint32_t max_attempts, uint32_t* attempts_out,
                           void* stream);

/* Statistics of the last successful build: *partitioned = 1 if it
 * took the partitioned path (see bht_tuning), else 0.  For a partitioned
 * build, *evicted = pairs that met a full first bucket and evicted a
 * resident on chip (iceberg tables: pairs that met a primary holding t
 * pairs and went on to the secondary step), and *overflow_probes = bucket
 * reads made while those pairs were inserted (Section VII-E's probe: one
 * bucket read); both 0 for a concurrent build.  Returns NOT_BUILT before a
 * successful build. */
bht_status bht_build_stats(const bht_table* t, uint32_t* partitioned, uint64_t* evicted,
                           uint64_t* overflow_probes);

/* Padding words of the last successful build's radix passes: a pass with
 * at most 256 digits over 32-bit pairs rounds every (chunk, digit) range
 * of its output up to whole 128-byte lines with the empty key (value 0),
 * which the next step skips; *pass1_words and *pass2_words are the
 * padding pairs the first and the second pass wrote (read back by the next
 * step, so part of the build's traffic), 0 for a pass that did not pad or
 * did not run, and both 0 for a concurrent build.  NOT_BUILT before a
 * successful build. */
bht_status bht_build_padding(const bht_table* t, uint64_t* pass1_words, uint64_t* pass2_words);

/* Bytes of caller-owned workspace a partitioned build of n pairs into this
 * table needs (see bht_tuning's build_mode), or 0 when the table does not
 * take that path (schemes other than BCHT and CHT1, 64-bit keys, n = 0,
 * n >= 2^32, n above the slot count). */
uint64_t bht_build_workspace_bytes(const bht_table* t, uint64_t n);

/* As bht_build_async, but a BCHT or CHT1 build takes the partitioned path
 * with the caller's device workspace d_workspace (workspace_bytes >=
 * bht_build_workspace_bytes(t, n), 256-byte aligned) instead of allocating
 * one, so a serving loop can keep one workspace per stream and never
 * allocate while building.  The workspace must stay untouched until
 * bht_build_wait returns.  Tables the partitioned path does not apply to
 * (or build_mode = BHT_BUILD_CONCURRENT) are built with the concurrent
 * kernel and the workspace is not used.  INVALID_ARG for a null, too small
 * or misaligned workspace. */
bht_status bht_build_async_in(bht_table* t, const uint32_t* d_keys, const uint32_t* d_values,
                              uint64_t n, void* d_workspace, uint64_t workspace_bytes,
                              void* stream);

/* For callers that cannot allocate device memory while they build (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): as bht_build_async_in, but the partitioned path's workspace is
 * a fixed array inside the library (bht_build_noalloc_max_bytes() bytes,
 * 64 MiB: about 8 M pairs), one per GPU, held until the process ends, so
 * the call allocates nothing.  Builds the default would give the concurrent
 * kernel need no workspace and take that kernel.  Finish with
 * bht_build_wait.  The table's device must be current.  CAPACITY when the
 * build needs more workspace than the array holds.  Every call on one GPU
 * shares that GPU's array: builds through this entry point that overlap on
 * one GPU (other streams, other threads) race and must be serialized by the
 * caller; the array keeps the last build's contents, and each build clears
 * what it counts with before use. */
uint64_t bht_build_noalloc_max_bytes(void);
bht_status bht_build_async_noalloc(bht_table* t, const uint32_t* d_keys,
                                   const uint32_t* d_values, uint64_t n, void* stream);

/* Bulk find of n queries (Section III; Section V).  d_out_values[i] is the
 * value stored with d_queries[i], or 0xFFFFFFFF when absent; d_out_found[i]
 * is 1 when present, else 0.  Asynchronous on stream; the table must be
 * built.  Query 0xFFFFFFFF is always absent. */
bht_status bht_find(const bht_table* t, const uint32_t* d_queries, uint64_t n,
                    uint32_t* d_out_values, uint8_t* d_out_found, void* stream);

/* 64-bit keys and values (bucketed cuckoo, 16-byte slots, 8 per bucket;
 * not in the paper, whose pairs fit one 64-bit word).  Keys 2^64 - 1 and
 * 2^64 - 2 are reserved (SENTINEL_KEY).  bht_build64 is synchronous like
 * bht_build and follows the table's build_mode: the partitioned path takes
 * builds of at least 2^18 pairs under BHT_BUILD_AUTO (workspace of about
 * 16 bytes per pair): each bucket's first-choice pairs are placed on chip,
 * the pairs meeting a full first bucket exchange themselves with random
 * residents in rounds ranked by the bucket's load counter, and the evicted
 * pairs then continue their cuckoo chains (Section III-A) concurrently. */
bht_status bht_build64(bht_table* t, const uint64_t* d_keys, const uint64_t* d_values,
                       uint64_t n, void* stream);
bht_status bht_find64(const bht_table* t, const uint64_t* d_queries, uint64_t n,
                      uint64_t* d_out_values, uint8_t* d_out_found, void* stream);

/* Instrumented variants counting probes, a probe being one bucket read
 * (Section VII-E).  bht_build_counted adds the build's bucket reads to
 * *d_probe_total (device uint64) and is synchronous; it always takes the
 * concurrent kernel, on which the paper's insertion probe count is
 * defined.  bht_find_counted writes each query's bucket reads to
 * d_probes[i] (device uint8) and also adds their sum to a counter the table
 * keeps (read by bht_get_probe_stats).  Not meant for timing. */
bht_status bht_build_counted(bht_table* t, const uint32_t* d_keys, const uint32_t* d_values,
                             uint64_t n, uint64_t* d_probe_total, void* stream);
bht_status bht_find_counted(const bht_table* t, const uint32_t* d_queries, uint64_t n,
                            uint32_t* d_out_values, uint8_t* d_out_found, uint8_t* d_probes,
                            void* stream);
/* bht_find64 that also writes each query's bucket reads to d_probes[i]
 * (device uint8).  INVALID_ARG for a null probe array. */
bht_status bht_find64_counted(const bht_table* t, const uint64_t* d_queries, uint64_t n,
                              uint64_t* d_out_values, uint8_t* d_out_found, uint8_t* d_probes,
                              void* stream);
/* Probe totals of a table (Section VII-E): *build_probes = bucket reads of
 * its last build if that build was bht_build_counted, else 0;
 * *find_probes = bucket reads of every instrumented find (32- or 64-bit)
 * on it since the previous bht_get_probe_stats call, or since bht_create.
 * Waits for all work on the device first.  Divide by the keys or queries
 * involved for the paper's per-key averages. */
bht_status bht_get_probe_stats(const bht_table* t, uint64_t* build_probes, uint64_t* find_probes);

/* Tuning (speed only, never results).  tile_width: lanes that read one
 * bucket together (1 for bucket_size 1; 4, 8 or 16 otherwise, at most
 * bucket_size; 0 keeps the default: 4 for BCHT and CHT1 tables of 16-slot
 * buckets, one 16-byte load per lane for the rest).  find_schedule: BHT_FIND_DEFAULT,
 * BHT_FIND_REFILL (a lane that finishes a query takes the next one) or
 * BHT_FIND_CHUNK (a wave answers 64 consecutive queries per chunk and writes
 * their results together) or BHT_FIND_PARALLEL (BCHT and CHT1 only: all h
 * candidate buckets of a query are read at once, Section II-A's parallel
 * query: one memory latency per query instead of up to h, at h probes per
 * query; results are identical).  grid_blocks: blocks of 256 threads per launch,
 * 0 = as many as the device keeps resident.  build_mode (BCHT, CHT1, IHT
 * and the 64-bit table; 64-bit tables take tile_width 8 and ignore the
 * rest):
 * BHT_BUILD_CONCURRENT inserts every pair with the concurrent cuckoo
 * kernel (Section V-B); BHT_BUILD_PARTITIONED first groups the pairs by the
 * region of their first bucket (two streaming radix passes), places each
 * region's pairs in their first bucket in on-chip memory, writes the
 * buckets whole, lets each pair that met a full first bucket exchange
 * itself with a random resident there (Section III-A's eviction step, on
 * chip), and runs the concurrent cuckoo kernel only on the pairs evicted:
 * their chains continue concurrently, as in the concurrent build, and
 * since no bucket ever loses a pair the layout obeys the same invariants
 * (every key in a candidate bucket, the early-exit property).  It allocates a
 * library-owned workspace of about 8-9 bytes per pair on first use (kept
 * until bht_destroy).  Iceberg tables (Section III-C) take the same path
 * with primaries filled on chip up to iht_threshold pairs and the rest
 * inserted at their secondary choices afterwards, concurrently (a pair
 * reaches the secondary level only once its primary holds iht_threshold
 * pairs, as the threshold rule requires).  BHT_BUILD_AUTO partitions builds of at least 2^18 pairs (2^26
 * for two-level iceberg tables, never one-level ones) into tables whose
 * memory the library owns (bht_create).
 * iht_early_exit (iceberg tables only, else UNSUPPORTED): 1 makes a find
 * stop after a miss in a primary bucket that holds fewer than
 * iht_threshold keys, which proves absence because a key goes to a
 * secondary bucket only once its primary holds that many (Section III-C);
 * such a negative query costs one probe instead of three.  0 (default)
 * probes every candidate, as Section V-D describes.  query_unroll (chunk
 * schedule, single-table and batched queries): queries per lane per chunk,
 * 1 or 2 (0 = the default: 2 for BCHT and CHT1 tables of 16-slot buckets,
 * else 1); the autotuner of the batched mode chooses it. */
typedef enum {
  BHT_FIND_DEFAULT = 0,
  BHT_FIND_REFILL = 1,
  BHT_FIND_CHUNK = 2,
  BHT_FIND_PARALLEL = 3
} bht_find_schedule;
typedef enum {
  BHT_BUILD_AUTO = 0,
  BHT_BUILD_CONCURRENT = 1,
  BHT_BUILD_PARTITIONED = 2
} bht_build_mode;
typedef struct {
  uint32_t tile_width;
  uint32_t find_schedule;
  uint32_t grid_blocks;
  uint32_t build_mode;
  uint32_t iht_early_exit;
  uint32_t query_unroll;
} bht_tuning;
bht_status bht_set_tuning(bht_table* t, const bht_tuning* tuning);
bht_status bht_get_tuning(const bht_table* t, bht_tuning* tuning);

/* Profiling: when enabled, HIP events are recorded on the call's stream
 * right before and after the main kernel of each build (the insertion
 * kernel, not the table reset) and each find.  bht_kernel_ms waits for the
 * events and returns the last build's and last find's kernel time in
 * milliseconds (-1 when none was recorded). */
bht_status bht_enable_timing(bht_table* t, int on);
bht_status bht_kernel_ms(const bht_table* t, float* build_ms, float* find_ms);

/* Geometry: number of (primary) buckets, slots per bucket, pairs stored by
 * the last successful build, and total bytes of the slot array. */
bht_status bht_info(const bht_table* t, uint64_t* num_buckets, uint32_t* bucket_size,
                    uint64_t* n_stored, uint64_t* table_bytes);

/* Copies the raw slot array (table_bytes from bht_info) to host memory, for
 * layout checks.  Synchronous. */
bht_status bht_download(const bht_table* t, void* host_slots);

/* Replaces the slot array with a host layout (table_bytes bytes) holding
 * n_stored pairs and marks the table built (tests: query a layout built
 * elsewhere).  Synchronous. */
bht_status bht_upload(bht_table* t, const void* host_slots, uint64_t n_stored);

/* Device address of the slot array (for callers that query several tables
 * in one launch). */
bht_status bht_device_slots(const bht_table* t, void** d_slots);

/* Diagnostics (ceilings for the roofline).  bht_diag_gather reads n_reads
 * random aligned blocks of line_bytes (32, 64, 128 or 256) from d_buf
 * (bytes long), line_bytes/16 lanes x 16 bytes per block, no table logic;
 * with 128 it is the access pattern of one bucket probe.  bht_diag_cas issues
 * n_ops random 8-byte compare-and-swaps on d_buf that never change it (the
 * new value equals the expected one).  bht_diag_stream reads the first
 * bytes of d_src in order (16-byte words, bytes rounded down to a multiple
 * of 16) and, when d_dst is not NULL, writes them to d_dst (a device copy;
 * the ranges must not overlap), else only reads them: the streaming
 * ceilings.  Both buffers 16-byte aligned.  d_sink is a device uint64 the
 * kernels may write.  All are asynchronous on stream. */
bht_status bht_diag_gather(const void* d_buf, uint64_t bytes, uint64_t n_reads, uint32_t line_bytes,
                           uint64_t seed, uint64_t* d_sink, void* stream);
bht_status bht_diag_cas(void* d_buf, uint64_t bytes, uint64_t n_ops, uint64_t seed,
                        uint64_t* d_sink, void* stream);
bht_status bht_diag_stream(const void* d_src, void* d_dst, uint64_t bytes, uint64_t* d_sink,
                           void* stream);

/* Batched mode (not in the paper): many bucketed cuckoo tables of uneven
 * sizes built and then queried together.  Every table of a batch is a
 * 32-bit BHT_BCHT table with the same bucket size, tile width and query
 * unroll (bht_tuning).  Entry i
 * names its table, its n_keys input pairs and its n_queries queries with
 * their output arrays (all caller-owned device memory, as for bht_build and
 * bht_find).  bht_batch_create copies the table descriptors and the work
 * items (ranges of item_size pairs or queries; 0 = 8192) to the device.
 * bht_batch_run enqueues a reset of the batch's queues and statuses, the
 * build of every table and one persistent query kernel pulling (table,
 * range) items from a device-side queue.  The build is the partitioned
 * build of all tables at once (counting, scan and scatter kernels over
 * (table, chunk) items, one on-chip placement per bin of any table, one
 * overflow insertion kernel); when a table asks for BHT_BUILD_CONCURRENT or
 * needs more than 1,024 bins it is instead a fill and one persistent
 * concurrent build kernel pulling (table, range) items.  These are
 * separate kernels because a kernel boundary is what makes one phase's
 * writes visible to the next phase's plain loads on every XCD.  On a
 * non-null stream the sequence is captured once into a HIP graph and
 * replayed by later runs on that stream.
 * bht_batch_wait waits for the stream and writes each table's build status
 * to status_out[i] (may be NULL); it returns BHT_OK when every table built.
 * A table whose build failed holds unspecified contents and unspecified
 * query outputs: reseed it and run it again (alone or in a new batch). */
typedef struct bht_batch bht_batch;
typedef struct {
  bht_table* table;
  const uint32_t* d_keys;
  const uint32_t* d_values;
  uint64_t n_keys;
  const uint32_t* d_queries;
  uint64_t n_queries;
  uint32_t* d_out_values;
  uint8_t* d_out_found;
} bht_batch_entry;
bht_status bht_batch_create(const bht_batch_entry* entries, uint32_t count, uint32_t item_size,
                            bht_batch** out);
bht_status bht_batch_run(bht_batch* b, void* stream);
bht_status bht_batch_wait(bht_batch* b, void* stream, bht_status* status_out);
void bht_batch_destroy(bht_batch* b);
/* The batch in one synchronous call: create, run once (launched directly
 * on stream, no graph), wait, destroy.  status_out[i] (may be NULL) gets
 * table i's build status; returns BHT_OK when every table built.  The
 * descriptors are a host array: the library reads every table's size on
 * the host to plan the partitioning anyway. */
bht_status bht_batch_build_find(const bht_batch_entry* entries, uint32_t count, uint32_t item_size,
                                bht_status* status_out, void* stream);

/* Coalesced lookups (serving): one launch answers many query batches on
 * many built 32-bit BCHT tables that share bucket size and tile width.  A
 * context holds device and pinned host space for up to max_requests
 * requests and max_items work items (one item = item_size queries of one
 * request; 0 = 8192).  bht_multi_find stages the request descriptors,
 * copies them asynchronously and launches one persistent query kernel on
 * stream; outputs are as for bht_find.  A call first waits until the
 * context's previous copies have completed, so one context serves one
 * stream at a time (use one context per stream for overlap). */
typedef struct bht_find_ctx bht_find_ctx;
typedef struct {
  const bht_table* table;
  const uint32_t* d_queries;
  uint64_t n;
  uint32_t* d_out_values;
  uint8_t* d_out_found;
} bht_find_request;
bht_status bht_find_ctx_create(uint32_t max_requests, uint64_t max_items, bht_find_ctx** out);
bht_status bht_multi_find(bht_find_ctx* ctx, const bht_find_request* reqs, uint32_t count,
                          uint32_t item_size, void* stream);
void bht_find_ctx_destroy(bht_find_ctx* ctx);

/* Host copy of the library's hash, for checking its arithmetic without a
 * GPU: ((a*k + b) mod p) mod m with the 32-bit family, and with the 64-bit
 * family. */
uint64_t bht_hash32(uint64_t a, uint64_t b, uint32_t k, uint64_t m);
uint64_t bht_hash64(uint64_t a, uint64_t b, uint64_t k, uint64_t m);

/* Human-readable status name, and the calling thread's last error detail. */
const char* bht_status_string(bht_status s);
const char* bht_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
