/*
 * slash.h - C ABI of the MI355X (gfx950) SLASH hot-path library, libslash.so.
 *
 * SLASH (Meisburger & Shrivastava, "Distributed Tera-Scale Similarity Search
 * with MPI") finds near neighbours of very sparse binary vectors with (K, L)
 * LSH tables and frequency aggregation, without distance computations.  This
 * library holds one node's shard on one GPU:
 *   - hash:   densified one-permutation MinHash, K values per table, L tables
 *             (Section 2.2, Section 2.3);
 *   - build:  every vector into its bucket of every table (Algorithm 1), each
 *             bucket a fixed-capacity reservoir (Section 3, "Avoid Skewed
 *             buckets") that keeps the R ids of smallest seeded priority;
 *   - insert: streaming insertion into the same fixed-size buckets
 *             (Section 3.1);
 *   - query:  probe the L buckets, aggregate candidate frequencies in a
 *             count-min sketch and report the top-k identities (Section 2.3
 *             "Cheap Frequency based Filtering", Algorithm 2, Section 2.4).
 *
 * Conventions for every call:
 *   - Every pointer argument named *_dev, and every pointer inside slash_csr,
 *     is a device pointer on the current HIP device; host pointers are named
 *     *_host.  `stream` is a hipStream_t (NULL = the default stream).
 *   - The caller owns every input and output buffer; they must stay valid
 *     until the work enqueued by the call has completed on `stream`.  The
 *     library owns the index memory until slash_free.
 *   - Calls return a slash_status; no C++ exception or abort crosses the ABI.
 *     On error, slash_last_error() describes it (thread-local string).
 *   - Results are bit-exact functions of (params, data, insert history):
 *     integer arithmetic only, every order total.
 *   - Ids are 0..N-1 in row order of slash_build, then sequential per insert.
 *     The id 0xFFFFFFFF marks an empty slot and is never assigned.
 */
#ifndef SLASH_H_
#define SLASH_H_

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SLASH_API __attribute__((visibility("default")))
#else
#define SLASH_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SLASH_OK = 0,
  SLASH_E_INVAL = -1,       /* bad parameter, index outside [0, dim), empty row, k > k_max */
  SLASH_E_NOMEM = -2,       /* device memory (or the serve HBM budget) exhausted */
  SLASH_E_DEVICE = -3,      /* HIP runtime error; text in slash_last_error() */
  SLASH_E_CAPACITY = -4,    /* ids would exceed 0xFFFFFFFE */
  SLASH_E_BUSY = -5,        /* serve queue full; retry later */
  SLASH_E_CLOSED = -6,      /* server stopped */
  SLASH_E_UNSUPPORTED = -7  /* parameters outside what the kernels implement */
} slash_status;

#define SLASH_EMPTY 0xFFFFFFFFu

/* Flags for calls that take a `flags` argument. */
#define SLASH_FLAG_TRUSTED 1u /* skip device-side input validation (no host sync) */
#define SLASH_FLAG_EXACT 2u   /* queries: rank candidates by their exact multiplicity among the probed
                                 slots instead of the count-min estimate (scores are the multiplicities) */

/* Index parameters (Section 4 "Initialization"; Section 6 "Values of K and
 * L").  Constraints checked by every call:
 *   dim >= 1; 1 <= K; 1 <= L; K * L <= 4096; 1 <= log2_buckets <= 30;
 *   1 <= R <= 256; 1 <= cm_rows <= 16; log2_cm_width <= 16 (0 means one
 *   counter); 1 <= k_max <= 1024; bucket 0 or 1; hash_mode:
 *   0 - one densified one-permutation pass (Section 2.2) over K*L equal range
 *       bins of one nonzero hash; table t takes bins [tK, tK + K);
 *   1 - a DOPH pass of K bins per table, each table with its own nonzero
 *       hash;
 *   2 - classic MinHash with K*L independent hash functions (Section 2.2;
 *       the L x K seeds of Section 4 "Initialization"): value j is the
 *       minimum over the row of its own nonzero hash, no densification;
 *       K*L times the hashing work of mode 0.
 *
 * bucket selects what a bucket holds:
 *   0 - the R ids of smallest priority (bottom-R reservoir, Section 3 "Avoid
 *       Skewed buckets"); queries aggregate with the count-min sketch of
 *       cm_rows x 2^log2_cm_width counters.
 *   1 - a Topkapi sketch (Section 3.1, Appendix 2) of cm_rows rows of
 *       2^log2_cm_width (heavy hitter, count) cells, row r sending id x to
 *       cell (a_r * x + b_r) >> (64 - log2_cm_width) (the count-min row
 *       hash); R is not used.  Ids enter a bucket in ascending order; on
 *       insertion a cell takes the id with count 1 when its count is 0,
 *       counts up on a match and down otherwise.  A query folds its L bucket
 *       sketches in table order (equal heavy hitters add; otherwise the
 *       larger count wins and keeps the difference; equal counts give the
 *       smaller id and count 0) and reports heavy hitters of count >= 1 by
 *       (count desc, id asc), an id held by several rows scoring its largest
 *       count.  Needs log2_cm_width <= 8 and cm_rows * 2^log2_cm_width <= 256. */
typedef struct {
  uint32_t dim;           /* number of features D */
  uint32_t K;             /* hashes per table */
  uint32_t L;             /* tables */
  uint32_t log2_buckets;  /* B: 2^B buckets per table */
  uint32_t R;             /* reservoir capacity per bucket */
  uint32_t cm_rows;       /* d: count-min rows */
  uint32_t log2_cm_width; /* log2 w: counters per count-min row */
  uint32_t k_max;         /* output row stride of queries */
  uint32_t hash_mode;     /* 0, 1 or 2, see above */
  uint32_t bucket;        /* 0: bottom-R reservoir, 1: Topkapi sketch (see above) */
  uint64_t seed;          /* every hash constant derives from this (Section 3 "Design") */
} slash_params;

/* Sparse binary rows in CSR form, device memory: row i holds the feature
 * indices indices[indptr[i] .. indptr[i+1]); indptr has n_rows + 1 entries
 * (indptr[0] need not be 0).  Order and repeats inside a row do not change
 * any result.  A row must be non-empty and its indices in [0, dim). */
typedef struct {
  const int64_t* indptr;
  const int32_t* indices;
  uint64_t n_rows;
} slash_csr;

typedef struct slash_index slash_index;
typedef struct slash_server slash_server;

typedef struct {
  slash_params params;
  uint64_t n_items;          /* ids assigned so far */
  uint64_t table_bytes;      /* device bytes held by the tables */
  uint32_t n_buckets;        /* 2^B */
  uint32_t reserved;
} slash_index_info;

/* Schedule of the batched query path (waves per query, queries per ticket,
 * resident work-groups per CU).  Any schedule gives identical results. */
typedef struct {
  uint32_t waves_per_query;  /* 1, 2, 4, 8 or 16 */
  uint32_t queries_per_ticket; /* 0 = one work-group per query (no work counter) */
  uint32_t groups_per_cu;    /* persistent form: 0 = as many as fit */
  uint32_t reserved;
} slash_schedule;

/* ------------------------------------------------------------------ core */

/* Build an index over `data` (Algorithm 1): hash every row into its L bucket
 * ids, group (table, bucket, id) triples with a device radix sort, and keep
 * per bucket the R ids of smallest priority p_t(id) in ascending priority,
 * plus seen = the number of ids hashed there.  Row i gets id i.  Tables live
 * in device memory: ids [L][2^B][R] (uint32, 0xFFFFFFFF-padded), seen
 * [L][2^B] (uint32).  Rows are checked (non-empty, indptr increasing)
 * before any work; indices are checked against [0, dim) by the hash kernel
 * itself, and the build stops with E_INVAL after the hash pass when one is
 * outside.  Synchronises `stream` before returning (validation flags,
 * work-list sizes; the tables are sorted and selected two at a time, on
 * `stream` and on a second stream of the library's, each with its own
 * scratch).  Errors: E_INVAL (params, rows, indices), E_NOMEM,
 * E_CAPACITY (n_rows > 0xFFFFFFFE), E_UNSUPPORTED (among others: a shape no
 * query kernel answers, i.e. more than 16384 reservoir slots L * R per query
 * or a count-min / id set larger than LDS; slash_import_tables and
 * slash_load refuse such shapes too), E_DEVICE.  *out is set only on
 * success. */
SLASH_API slash_status slash_build(const slash_params* params, slash_csr data, void* stream, slash_index** out);

/* Insert rows (Section 3.1 streaming insert): ids n_items, n_items+1, ... in
 * row order; each touched bucket keeps the R smallest-priority ids of its old
 * content and the new ids (Topkapi buckets: the new ids enter the bucket's
 * sketch in ascending order), seen += number of new ids.  The result equals a
 * bulk build over all rows inserted so far.  new_ids_dev (nullable) receives
 * the n_rows assigned ids.  Needs exclusive access to the index (no
 * concurrent query on another stream).  Validation (unless TRUSTED) happens
 * before any table changes; on error the index is unchanged. */
SLASH_API slash_status slash_insert(slash_index* index, slash_csr rows, uint32_t flags, uint32_t* new_ids_dev,
                          void* stream);

/* Query (Section 2.3 query phase; Algorithm 2 on one node): hash each query
 * row, gather the ids of its L buckets (with multiplicity), estimate each
 * candidate's frequency with the count-min sketch (cm_rows x 2^log2_cm_width
 * counters; est(c) = min over rows of the counter c hashes to) and write the
 * top-k distinct candidates by (estimate desc, id asc).  Output row q is
 * ids_dev[q * k_max .. q * k_max + k_max) and scores_dev likewise; slots past
 * min(k, #distinct candidates) hold (0xFFFFFFFF, 0).  k_per_query_dev
 * (nullable) gives each query its own k; else `k` applies to all.  k and each
 * k_per_query must be <= k_max (checked on the device unless TRUSTED; under
 * TRUSTED larger values are clamped to k_max).  With SLASH_FLAG_EXACT the
 * candidates are ranked by their exact multiplicity among the probed slots
 * (at most L) instead of the estimate (the sketch-versus-exact comparison of
 * Section 6.2); scores are then the multiplicities.  One work-group per query,
 * no device allocation, asynchronous under TRUSTED.  Topkapi buckets: one
 * wave per query folds the L bucket sketches and reports as described at
 * slash_params (scores are merged counts; EXACT is E_UNSUPPORTED). */
SLASH_API slash_status slash_query(const slash_index* index, slash_csr queries, const uint32_t* k_per_query_dev,
                         uint32_t k, uint32_t flags, uint32_t* ids_dev, uint32_t* scores_dev, void* stream);

/* Same results as slash_query (bit-exact) through the batched path: every
 * query is first hashed by the row-parallel hash kernel into an index-owned
 * bucket-id buffer (grown on demand), then one launch answers them: a
 * persistent one whose resident work-groups take queries from a device work
 * counter, or (queries_per_ticket = 0) one work-group per query, with the
 * schedule `sched` (NULL = the tuned schedule for this index, see
 * slash_autotune; when schedules of several query-size classes are tuned,
 * the batch's mean row size picks the nearest class, which reads its first
 * and last row offsets with a copy that synchronises `stream`).  Both launches are recorded once into a HIP graph and
 * replayed.  Batched calls on one index share that buffer: issue them on one
 * stream (or otherwise order them). */
SLASH_API slash_status slash_query_batched(const slash_index* index, slash_csr queries, const uint32_t* k_per_query_dev,
                                 uint32_t k, uint32_t flags, uint32_t* ids_dev, uint32_t* scores_dev,
                                 const slash_schedule* sched, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * results as slash_query_batched (bit-exact), with the same arguments, but
 * the call allocates nothing.  Its kernels (row-parallel hash, then the
 * query kernel in the schedule's form, launched directly rather than
 * through a HIP graph) keep the batch's bucket ids and work counter in a
 * statically sized device array of the library, 16 MiB per GPU (a work
 * counter in a 256-byte head, then n_rows * L bucket ids), which each GPU
 * the library runs on holds until the process ends.  A batch needing more
 * (n_rows * L > 4,194,240) is refused with E_INVAL before anything is
 * launched.  Every call on one GPU shares that GPU's array and keeps the
 * last call's contents (the counter is cleared by each call with a fill
 * kernel): calls that overlap on one GPU race, so issue them on one stream
 * or otherwise order them.  Topkapi-bucket indexes use no scratch.  The
 * caller still provides every input and output buffer.  Other errors as
 * slash_query_batched. */
SLASH_API slash_status slash_query_batched_static(const slash_index* index, slash_csr queries,
                                                  const uint32_t* k_per_query_dev, uint32_t k, uint32_t flags,
                                                  uint32_t* ids_dev, uint32_t* scores_dev,
                                                  const slash_schedule* sched, void* stream);

/* Time every candidate schedule on `sample` (device CSR of representative
 * queries, k as given) and keep the fastest per query-size class for
 * slash_query_batched.  Candidates that disagree with slash_query are
 * rejected (E_DEVICE).  best_out (nullable) receives the schedule chosen for
 * the sample's dominant class.  Synchronises `stream`. */
SLASH_API slash_status slash_autotune(slash_index* index, slash_csr sample, uint32_t k, slash_schedule* best_out,
                            void* stream);

/* Bucket ids [n_rows][L] of each row (the hash step alone, Section 2.2-2.3). */
SLASH_API slash_status slash_hash(const slash_index* index, slash_csr rows, uint32_t flags, uint32_t* buckets_dev,
                        void* stream);

/* Copy the tables into caller device buffers: ids [L][2^B][R] (Topkapi
 * buckets: cells [L][2^B][cm_rows][2^log2_cm_width][2] as heavy hitter,
 * count), seen [L][2^B] (either may be NULL).  Asynchronous on `stream`. */
SLASH_API slash_status slash_export_tables(const slash_index* index, uint32_t* ids_dev, uint32_t* seen_dev,
                                 void* stream);

/* Create an index from tables exported earlier (with the same params):
 * ids [L][2^B][R] and seen [L][2^B] device buffers are copied in; n_items is
 * the number of ids assigned so far (the next insert continues from it).
 * Together with slash_export_tables this saves and restores an index (the
 * caller moves the buffers to storage).  Reservoir tables are checked: the
 * first min(R, seen) slots of every bucket must hold ids below n_items and
 * the slots past them EMPTY, as a build or insert leaves them (Topkapi cells
 * are taken as they are).  Errors: E_INVAL (params, NULL buffers, tables
 * failing the check), E_CAPACITY (n_items > 0xFFFFFFFE), E_NOMEM, E_DEVICE.
 * Synchronises `stream`. */
SLASH_API slash_status slash_import_tables(const slash_params* params, const uint32_t* ids_dev, const uint32_t* seen_dev,
                                 uint64_t n_items, void* stream, slash_index** out);

/* Save an index to a file (the index stays valid): a 128-byte header
 * (magic "SLASHIDX", format version 1, every slash_params field, n_items,
 * the byte sizes of the two arrays and a 64-bit FNV-1a checksum of them),
 * then the table array and the seen array exactly as slash_export_tables
 * lays them out, little endian.  Copies the tables through 64 MiB of pinned
 * host memory on `stream` and synchronises it.  Errors: E_INVAL (NULL
 * arguments, file not writable), E_DEVICE. */
SLASH_API slash_status slash_save(const slash_index* index, const char* path, void* stream);

/* Load an index saved by slash_save: the parameters come from the file, the
 * tables are copied to the device and checked as by slash_import_tables, and
 * the next insert continues from the saved n_items.  Errors: E_INVAL (not a
 * saved index, another format version, parameters that fail the checks of
 * slash_build, a file whose size or checksum does not match its header,
 * tables that fail the check), E_NOMEM, E_DEVICE.  Synchronises `stream`. */
SLASH_API slash_status slash_load(const char* path, void* stream, slash_index** out);

SLASH_API slash_status slash_index_info_get(const slash_index* index, slash_index_info* info);

/* Per-phase timing of the build that made `index`, measured with HIP events
 * recorded around every launch of the phase on the stream it ran on; the
 * build runs its tables alternately on the caller's stream and on a second
 * stream of its own (created once per device, kept until the process ends),
 * so launches of two tables overlap and the phase totals of a build add up
 * to more than its duration.  Phases:
 * validate, hash, sort_upsweep, sort_scan, sort_downsweep, segment_bounds,
 * select, heavy.  alg_bytes is the phase's algorithmic HBM traffic (bytes the
 * phase must read and write, counted once).  Writes up to max entries to out
 * (host memory), *n receives the number written. */
typedef struct {
  char name[32];
  uint32_t launches;
  uint32_t reserved;
  double total_ms;
  double alg_bytes;
} slash_phase_stat;
SLASH_API slash_status slash_build_profile(const slash_index* index, slash_phase_stat* out, uint32_t max, uint32_t* n);

/* Free the index (waits for the device to finish with it). */
SLASH_API void slash_free(slash_index* index);

/* Thread-local description of the last error ("" if none). */
SLASH_API const char* slash_last_error(void);

/* Route the library's device allocations through caller functions (e.g. a
 * framework's caching allocator).  alloc_fn returns NULL on failure.  Pass
 * NULLs to restore hipMalloc/hipFree.  Set it before any index exists (a
 * block is always freed through the allocator that made it only while the
 * setting is unchanged).  Not thread-safe against concurrent allocation.
 *
 * With the default allocator the library keeps the device blocks it frees
 * (build scratch, the tables of freed indexes) and reuses them for later
 * allocations of up to their size, since allocating and freeing tens of GB
 * costs more than a build's kernels.  An allocation that fails releases the
 * cache of its device and is retried; slash_release_cache() returns every
 * cached block to the device now (also done by slash_set_allocator). */
typedef void* (*slash_alloc_fn)(size_t bytes, void* ctx);
typedef void (*slash_free_fn)(void* ptr, void* ctx);
SLASH_API slash_status slash_set_allocator(slash_alloc_fn alloc_fn, slash_free_fn free_fn, void* ctx);
SLASH_API void slash_release_cache(void);

/* -------------------------------------------------------------- serving */

/* Continuous-batching server over a resident index (the query process is
 * online, Section 2.3).  A scheduler thread admits pending requests into
 * device batches as staging slots free up and launches them on one device
 * stream in submission order, so a query admitted in epoch e sees exactly
 * the inserts submitted before it; inserts queued back to back are applied
 * in one launch (each still closes its own epoch).  Inserts are prepared
 * ahead in submission order (copied in, hashed and grouped on a second
 * stream into per-slot scratch, up to eight at a time), so only their table
 * writes sit in the ordered stream, and those run inside the launch of the
 * query batch before them when it is small (see insert_fusion).  Batch
 * slots (device and pinned host staging for one batch) are allocated at
 * start, up to max_inflight, as far as the HBM budget and the device's free
 * memory (leaving 1 GiB free) allow; one that did not fit then is added
 * later, while requests wait for a slot, if memory has freed up. */
#define SLASH_SERVE_MAX_K 128u /* largest k a served query may ask for */

typedef struct {
  uint64_t hbm_budget_bytes;  /* device bytes the server may hold for request data */
  uint32_t max_batch;         /* queries per device batch */
  uint32_t max_inflight;      /* batch slots at most (>= 1): batches launched and not yet harvested */
  uint32_t queue_capacity;    /* pending requests accepted before E_BUSY */
  uint32_t max_wait_us;       /* 0: a batch launches as soon as a slot is free; else a batch that is
                                 neither full nor followed by an insert waits until its oldest
                                 query has waited this long */
  uint32_t max_query_nnz;     /* largest query row accepted */
  uint32_t max_insert_nnz;    /* indices one insert request may carry (0: max(4096 * 64, 8 * max_query_nnz)) */
  uint32_t insert_fusion;     /* 0: a query batch of at most (compute units / 2) queries that is followed
                                 by an insert already prepared shares a launch with that insert: the
                                 batch reads its slots, the insert's tables are written after every
                                 query of the batch has, and the batch is ranked in the next launch;
                                 1: never; 2: always, waiting for the insert's preparation.  Results
                                 are the same */
  uint32_t reserved;          /* 0 */
} slash_serve_config;

typedef struct {
  uint64_t ticket;
  uint64_t epoch;        /* index epoch the request saw (queries) or created (inserts) */
  int32_t status;        /* slash_status of this request */
  uint32_t kind;         /* 0 = query, 1 = insert */
  uint32_t k;            /* queries: requested k */
  uint32_t n_ids;        /* inserts: number of ids assigned */
  uint32_t first_id;     /* inserts: first assigned id */
  uint32_t reserved;
  uint32_t ids[SLASH_SERVE_MAX_K];    /* queries: top-k ids (k entries valid) */
  uint32_t scores[SLASH_SERVE_MAX_K]; /* queries: their estimates */
  double t_submit_s;     /* host clock (seconds, steady) at submission */
  double t_done_s;       /* host clock when the result became available */
} slash_completion;

typedef struct {
  uint64_t queries_done, inserts_done, rows_inserted, batches, rejected_busy, rejected_nomem;
  uint64_t peak_inflight, peak_hbm_bytes;
  double busy_s;   /* seconds with device work in flight (host clock) */
  double launch_s; /* scheduler seconds in launch calls (query batches, insert preparations and commits) */
  double wait_s;   /* of which waiting for a prepared insert's word before its commit */
  double pack_s;   /* scheduler seconds copying request data into staging */
  uint64_t fused_commits; /* insert commits (each of one or more merged inserts) whose table writes ran
                             in a query batch's launch */
  uint64_t split_batches; /* query batches gathered in one launch and ranked in a later one */
} slash_serve_stats;

SLASH_API slash_status slash_serve_start(slash_index* index, const slash_serve_config* cfg, slash_server** out);

/* Submit one query (host indices, copied before return).  Checked on the
 * host: nnz in [1, max_query_nnz], indices in [0, dim), k <= min(k_max,
 * SLASH_SERVE_MAX_K); E_BUSY when the queue is full, E_CLOSED after stop. */
SLASH_API slash_status slash_serve_submit_query(slash_server* srv, const int32_t* indices_host, uint32_t nnz, uint32_t k,
                                      uint64_t* ticket);

/* Submit one insert of n_rows host CSR rows (indptr_host has n_rows + 1
 * entries, indptr_host[0] == 0; copied and checked before return).  Ids are
 * assigned when the insert is applied, in submission order. */
SLASH_API slash_status slash_serve_submit_insert(slash_server* srv, const int64_t* indptr_host, const int32_t* indices_host,
                                       uint32_t n_rows, uint64_t* ticket);

/* Take up to max finished requests (any order); *n receives the count. */
SLASH_API slash_status slash_serve_poll(slash_server* srv, slash_completion* out, uint32_t max, uint32_t* n);

/* Stop: drain every accepted request, join the scheduler, free the server. */
SLASH_API slash_status slash_serve_stop(slash_server* srv, slash_serve_stats* stats);

/* Open-loop replay for measurement: submit requests at the given arrival
 * times (seconds from the call) from a native client thread, poll every
 * completion and write per-request latency (done - scheduled arrival, s).
 * Queries are rows of q_indptr/q_indices (host), inserts take consecutive
 * rows of ins_indptr/ins_indices (host).  Returns when all have completed. */
SLASH_API slash_status slash_serve_replay(slash_server* srv, uint64_t n, const double* t_arrival, const uint8_t* is_insert,
                                const uint32_t* ins_rows, const int64_t* q_indptr, const int32_t* q_indices,
                                const uint32_t* q_k, const int64_t* ins_indptr, const int32_t* ins_indices,
                                double* latency_s, uint32_t* out_ids, uint32_t out_stride);

#ifdef __cplusplus
}
#endif
#endif /* SLASH_H_ */
