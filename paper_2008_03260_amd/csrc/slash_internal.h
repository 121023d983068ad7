// Internal declarations of libslash: constant layout, device helpers and the
// kernel launchers shared by the host orchestration files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "slash.h"

#define SL_EMPTY 0xFFFFFFFFu
#define SL_WAVE 64

namespace slash {

// ------------------------------------------------------------ constants
// Device-resident constant table of one index.  Everything derives from the
// seed (Section 3 "Design": one shared seed gives every worker the same hash
// functions).  Offsets are in elements of the named type.
struct ConstView {
  const uint64_t* a_h;   // [n_h]  nonzero-hash multipliers (odd)
  const uint64_t* b_h;   // [n_h]
  const uint32_t* dirw;  // [ceil(M/32)] densification direction bits (1 = right)
  const uint64_t* a_tj;  // [L*K] bucket multipliers (odd)
  const uint64_t* b_t;   // [L]
  const uint32_t* key_t; // [L] priority keys
  const uint32_t* m1_t;  // [L] odd
  const uint32_t* m2_t;  // [L] odd
  const uint64_t* a_r;   // [d] count-min multipliers (odd)
  const uint64_t* b_r;   // [d]
  uint32_t* bad = nullptr;  // when set, hashing ORs 2 here on an index outside [0, dim)
};

struct HostConsts {
  std::vector<uint64_t> a_h, b_h, a_tj, b_t, a_r, b_r;
  std::vector<uint32_t> dirw, key_t, m1_t, m2_t;
};

// Shape of an index as the kernels see it.
struct Shape {
  uint32_t dim, K, L, M, B, R, d, lw, k_max, mode;
  uint32_t bucket;  // 0: bottom-R reservoir of R ids; 1: Topkapi sketch of d x 2^lw cells
  uint32_t nb;     // 2^B
  uint32_t mshift; // M = 2^mshift when pow2, else 0xFF
};

struct TablesView {
  uint32_t* ids;   // [L][nb][R]
  uint32_t* seen;  // [L][nb]
};

// ------------------------------------------------------- device helpers

__device__ __forceinline__ uint32_t hi32(uint64_t z) { return (uint32_t)(z >> 32); }

// Nonzero hash u(i) = hi32(a * i + b) (mod 2^64), a 2-universal stand-in for
// the random permutation of MinHash (Section 2.2).
__device__ __forceinline__ uint32_t nz_hash(uint64_t a, uint64_t b, uint32_t i) {
  return hi32(a * (uint64_t)i + b);
}

// Range bin of u among n equal bins: hi32(u * n).
__device__ __forceinline__ uint32_t range_bin(uint32_t u, uint32_t n) {
  return (uint32_t)(((uint64_t)u * n) >> 32);
}

// Reservoir priority: xor-multiply-xorshift bijection of uint32.
__device__ __forceinline__ uint32_t priority(uint32_t id, uint32_t key, uint32_t m1, uint32_t m2) {
  uint32_t x = (id ^ key) * m1;
  x ^= x >> 16;
  x *= m2;
  x ^= x >> 15;
  return x;
}

// Count-min row hash (a * c + b) >> (64 - lw); lw = 0 means one counter.
__device__ __forceinline__ uint32_t cm_hash(uint64_t a, uint64_t b, uint32_t c, uint32_t lw) {
  return lw ? (uint32_t)((a * (uint64_t)c + b) >> (64 - lw)) : 0u;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  uint32_t l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// Lanes of the wave whose `nbits`-bit digit equals this lane's digit,
// restricted to `active`.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int nbits, uint64_t active) {
  uint64_t m = active;
  for (int b = 0; b < nbits; ++b) {
    bool bit = (d >> b) & 1u;
    uint64_t v = ballot64(bit);
    m &= bit ? v : ~v;
  }
  return m;
}

// Work-groups are dealt round-robin to the 8 XCDs (each with its own L2).
// Map block b to a tile so that every XCD works through one contiguous range
// of tiles; a bijection on [0, n) for any n.  Neighbouring tiles then share
// an L2, so their partial-line writes to the same output run merge there.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
  const uint32_t x = b % kXcds, i = b / kXcds, q = n / kXcds, r = n % kXcds;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Record the thread-local error text and return s.
slash_status fail(slash_status s, const char* fmt, ...);

// ------------------------------------------------------------ launchers
// Every launcher enqueues on `st` and returns hipSuccess or the launch error.

hipError_t launch_validate(slash_csr rows, uint32_t dim, const uint32_t* kq, uint32_t k_max,
                           uint32_t* flag, hipStream_t st);
// Hash rows into keys: keys[t * key_stride + r] = bucket id (combined with t
// when `combine`: t * nb + bucket).
hipError_t launch_hash_rows(const Shape& s, const ConstView& c, slash_csr rows, uint32_t* keys,
                            uint64_t key_stride, int combine, hipStream_t st);
// Bucket ids in row-major [n][L].
hipError_t launch_hash_rowmajor(const Shape& s, const ConstView& c, slash_csr rows, uint32_t* out,
                                hipStream_t st);

// Key-value radix sort of n uint32 keys on bits [0, nbits).  vals_in may be
// NULL: values are then the positions 0..n-1.  Results land in
// (keys_out, vals_out); the tmp buffers hold n entries each.
// Optional event marks around kernel launches (build profiling).
struct PhaseTimer {
  virtual void begin(int phase, hipStream_t st) = 0;
  virtual void end(int phase, hipStream_t st) = 0;
  virtual ~PhaseTimer() {}
};
enum { PH_VALIDATE, PH_HASH, PH_UPSWEEP, PH_SCAN, PH_DOWNSWEEP, PH_BOUNDS, PH_SELECT, PH_HEAVY, PH_COUNT };

struct SortBuffers {
  uint32_t *k0, *v0, *k1, *v1;  // ping-pong, n each
  uint32_t* hist;               // >= hist_entries(n)
  uint32_t* part;               // scan partials
};
size_t sort_hist_entries(uint64_t n);
size_t sort_part_entries(uint64_t n);
hipError_t radix_sort(const uint32_t* keys_in, const uint32_t* vals_in, uint64_t n, int nbits,
                      SortBuffers& b, uint32_t** keys_out, uint32_t** vals_out, hipStream_t st,
                      PhaseTimer* timer = nullptr);

// The build's sort: n ids (the positions 0..n-1) by their keys' bits
// [0, nbits), carried as 6 bytes per item; needs packed_sort_ok(n, nbits).
// Writes the ids in key order to *ids_out (one of b.k0 / b.k1) and each key's
// run [start[key], end[key]); keys with no items keep what start and end held
// (fill both with 0).
bool packed_sort_ok(uint64_t n, int nbits);
hipError_t radix_sort_runs(const uint32_t* keys_in, uint64_t n, int nbits, SortBuffers& b, uint32_t* start,
                           uint32_t* end, uint32_t** ids_out, hipStream_t st, PhaseTimer* timer = nullptr);

// Bounds [s0, e0) of a bucket's run as the build wrote them (an empty run as
// (0, 0); any e0 <= s0 is taken as empty).
__device__ __forceinline__ void bucket_run(const uint32_t* start, const uint32_t* end, uint32_t b, uint32_t& s0,
                                           uint32_t& e0) {
  s0 = start[b];
  e0 = end[b];
  if (e0 <= s0) s0 = e0 = 0;
}

// Exclusive scan of n uint32 (in place), scratch `part` of sort_part_entries(n).
hipError_t exclusive_scan(uint32_t* data, uint64_t n, uint32_t* part, hipStream_t st);

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st);
// Kernel entry of the fill kernel (for HIP graph nodes): (uint32_t* p, uint32_t v, uint64_t n).
void* fill_kernel_ptr();
// Kernel entry of the persistent query kernel for `waves` waves per query.
void* persistent_query_kernel(const Shape& s, uint32_t waves, bool exact = false);
// The grid-stride form (one work-group per query, no work counter), with
// arguments (Shape, ConstView, TablesView, QueryArgs).
void* plain_query_kernel(const Shape& s, uint32_t waves, bool exact = false);
hipError_t launch_validate_indices(const int32_t* idx, uint64_t n, uint32_t dim, uint32_t* flag, hipStream_t st);
hipError_t launch_item_ids(uint32_t* vals, uint32_t first_id, uint64_t n_rows, uint64_t items, hipStream_t st);
hipError_t launch_iota_u32(uint32_t* p, uint32_t first, uint64_t n, hipStream_t st);
// Check imported reservoir tables ([n_buckets][R] ids, [n_buckets] seen):
// ORs 8 into *flag unless every bucket's first min(R, seen) slots hold ids
// below n_items and the rest are EMPTY.
hipError_t launch_check_tables(const uint32_t* ids, const uint32_t* seen, uint64_t n_buckets, uint32_t R,
                               uint64_t n_items, uint32_t* flag, hipStream_t st);

// Per-bucket [start, end) of a sorted key array (start/end pre-zeroed, nb entries).
hipError_t launch_segment_bounds(const uint32_t* skeys, uint64_t n, uint32_t* start, uint32_t* end,
                                 hipStream_t st);

// Bottom-R selection for table t: buckets with <= heavy_t items are finished
// in place; heavier ones are appended to heavy_list (count in *heavy_n).
hipError_t launch_select_light(const Shape& s, const ConstView& c, uint32_t t, const uint32_t* svals,
                               const uint32_t* start, const uint32_t* end, TablesView tab,
                               uint32_t heavy_t, uint32_t* heavy_list, uint32_t* heavy_n, hipStream_t st);
// Chunk work: items [off, off+len) of `src` -> bottom-R candidates written to
// dst[w * R ..] (padded with EMPTY), for table t.
struct ChunkWork {
  uint64_t off;
  uint32_t len;
  uint32_t dst;  // output slot (in units of R)
};
struct FinalWork {
  uint64_t off;
  uint32_t len;
  uint32_t bucket;
  uint32_t seen;
  uint32_t pad;
};
// Finish the heavy buckets listed by launch_select_light entirely on the
// device: plan chunks of chunk_len ids, reduce each chunk to a bottom-R
// candidate list (cand: heavy_chunk_capacity(n) * R ids), merge each bucket's
// candidates into its reservoir.  No host synchronisation.
size_t heavy_chunk_capacity(uint64_t n, uint32_t chunk_len);
hipError_t launch_heavy(const Shape& s, const ConstView& c, uint32_t t, const uint32_t* svals, uint64_t n,
                        const uint32_t* heavy_list, const uint32_t* heavy_n, uint32_t chunk_len, ChunkWork* chunks,
                        FinalWork* finals, uint32_t* n_chunks, uint32_t* cand, TablesView tab, hipStream_t st);


// Small insert (n rows, keys [L][n] as written by launch_hash_rows without
// combining): one block per table groups the (bucket, id) pairs in LDS
// (launch_insert_group: reads only the keys, writes only the scratch), then
// one kernel merges every touched bucket's run into its reservoir
// (launch_insert_runs: the only kernel that writes the tables).
bool small_insert_ok(const Shape& s, uint64_t n);
size_t small_insert_scratch(const Shape& s, uint64_t n);
// Optional completion signal of the grouping kernel: when flag is set, the
// last block to finish sets *flag = value (host-visible) once every block's
// writes are visible device-wide; counter is a device word that holds 0
// before the launch (the last block returns it to 0).
struct GroupSignal {
  uint32_t* counter = nullptr;
  uint64_t* flag = nullptr;
  uint64_t value = 0;
};
hipError_t launch_insert_group(const Shape& s, const uint32_t* keys, uint32_t n, uint32_t first_id, void* scratch,
                               hipStream_t st, const GroupSignal& sig = {});
hipError_t launch_insert_runs(const Shape& s, const ConstView& c, void* scratch, uint32_t n, TablesView tab,
                              hipStream_t st);
hipError_t launch_insert_small(const Shape& s, const ConstView& c, const uint32_t* keys, uint32_t n, uint32_t first_id,
                               void* scratch, TablesView tab, hipStream_t st);
// The run records ([L][n] uint2) and ids ([L][n]) inside a small insert's
// scratch; false when n does not take the small path.
bool insert_run_arrays(const Shape& s, void* scratch, uint32_t n, const uint2** recs, const uint32_t** items);
// Insert merge: sorted combined keys (t*nb+b) with new ids -> merged reservoirs.
hipError_t launch_insert_merge(const Shape& s, const ConstView& c, const uint32_t* skeys,
                               const uint32_t* svals, uint64_t n, uint32_t* seg_scratch,
                               uint32_t* part, TablesView tab, hipStream_t st);

// Query kernels.
struct QueryArgs {
  slash_csr q;
  const uint32_t* kq;
  uint32_t k;
  uint32_t clamp;  // 1: clamp k to k_max
  uint32_t* out_ids;
  uint32_t* out_scores;
  const uint32_t* qbk;  // bucket ids [n][L] hashed beforehand, or NULL (hash in the query kernel)
  uint32_t exact = 0;   // 1: rank by exact multiplicity instead of the count-min estimate
  uint32_t* slot_ids = nullptr;  // serving: the gathered slot ids [n][L * R] between the two halves
};
// Kernel entry of the row-major hash kernel for this shape and its launch
// geometry (for HIP graph nodes): (Shape, ConstView, slash_csr, uint32_t* out).
void* hash_rowmajor_kernel(const Shape& s, uint32_t* threads, size_t* lds);
uint32_t hash_rowmajor_grid(const Shape& s, uint64_t n_rows);
int query_block_threads(const Shape& s, uint32_t waves);
size_t query_lds_bytes(const Shape& s, uint32_t waves, bool exact = false);
bool query_supported(const Shape& s);
bool query_supported(const Shape& s, uint32_t waves, bool exact = false);
uint32_t query_default_waves(const Shape& s);
hipError_t query_occupancy(const Shape& s, uint32_t waves, int* per_cu, bool exact = false);
hipError_t launch_query_waves(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& a,
                              uint32_t waves, hipStream_t st);
hipError_t launch_query(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& a,
                        hipStream_t st);
// Serving: one launch that ranks the previous batch's queries from the
// slot ids their gather stored (prev, may be empty), answers this batch's
// queries whole or only gathers them (cur, may be empty; count-min, hashing
// in the kernel; cur_host_ip, when not null, is cur's row offsets in host
// memory, whose first entries go in the launch so the kernel need not read
// them), and then applies a prepared small insert's runs to the
// tables (n_ins rows, none when 0) after every query of this batch has read
// them.  `dev` holds two device words that start at zero and only grow;
// tickets/gathered are their values after the last launch (updated here;
// launches using one FuseSync must be ordered on one stream).  gave_up is a
// host-coherent word a launch sets when its bounded wait ends without the
// queries' count.  hipErrorNotSupported when the shape has no such kernel.
struct FuseSync {
  unsigned long long* dev = nullptr;
  uint32_t* gave_up = nullptr;
  unsigned long long tickets = 0, gathered = 0;
};
bool serve_step_supported(const Shape& s);
hipError_t launch_serve_step(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& prev,
                             const QueryArgs& cur, bool gather_only, void* ins_scratch, uint32_t n_ins, int n_cu,
                             FuseSync& fs, hipStream_t st, const int64_t* cur_host_ip = nullptr);
hipError_t launch_query_persistent(const Shape& s, const ConstView& c, const TablesView& tab,
                                   const QueryArgs& a, uint32_t waves, uint32_t per_ticket, uint32_t grid,
                                   uint32_t* ticket, hipStream_t st);

// Topkapi buckets (bucket == 1): each bucket is d x 2^lw (heavy hitter,
// count) cells, stored as uint2 in the table array.
bool tk_supported(const Shape& s);
// Build of one table from its sorted ids: buckets of at most heavy_t ids
// (light), then the listed heavier ones.  heavy_t must be the heavy kernels'
// chunk length (16384); scratch holds tk_heavy_scratch_words(s, n / 16384 + 1)
// words; hpar is its start.
size_t tk_heavy_scratch_words(const Shape& s, uint64_t max_heavy);
hipError_t launch_tk_light(const Shape& s, const ConstView& c, uint32_t t, const uint32_t* sv, const uint32_t* start,
                           const uint32_t* end, TablesView tab, uint32_t heavy_t, uint32_t* heavy_list,
                           uint32_t* heavy_n, uint32_t* hpar, hipStream_t st);
hipError_t launch_tk_heavy(const Shape& s, const ConstView& c, uint32_t t, const uint32_t* sv, const uint32_t* start,
                           const uint32_t* end, TablesView tab, const uint32_t* heavy_list, const uint32_t* heavy_n,
                           uint64_t n, uint32_t* scratch, hipStream_t st);
hipError_t launch_tk_clear(const Shape& s, TablesView tab, hipStream_t st);
hipError_t launch_tk_segments(const Shape& s, const ConstView& c, const uint32_t* sk, const uint32_t* sv, uint64_t n,
                              const uint32_t* seg_start, const uint32_t* nseg, TablesView tab, hipStream_t st);
hipError_t launch_tk_runs(const Shape& s, const ConstView& c, const uint2* recs, const uint32_t* items, uint32_t n,
                          TablesView tab, hipStream_t st);
hipError_t launch_tk_query(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& a,
                           hipStream_t st);

// Size the index's insert scratch for batches of up to `rows` rows now, so
// that later inserts of at most that many rows allocate nothing.
slash_status reserve_insert_scratch(slash_index* ix, uint64_t rows);

// slash_insert's body (rows on `st`, in order after earlier work on it).
slash_status insert_rows(slash_index* ix, slash_csr rows, uint32_t flags, uint32_t* new_ids_dev, hipStream_t st);

// A small insert split in two for a caller that prepares inserts beside
// other work and orders the table writes itself (the server):
// insert_prepare hashes and groups `rows` (trusted) into the caller's scratch
// on `st` and takes the next ids (*first_id); insert_commit writes the tables
// from that scratch on `st`, which the caller must order after the prepare's
// kernels and after every query that must not see the rows.  Prepares take
// ids in call order.  insert_scratch_bytes gives the scratch sizes for
// inserts of up to `rows` rows, or returns false when such inserts cannot
// take this path.
// With sig.flag set, the grouping kernel sets *sig.flag = sig.value when the
// prepare's kernels are done (see GroupSignal).
struct InsertScratch {
  uint32_t* keys = nullptr;  // [L][rows] bucket ids
  void* runs = nullptr;      // run records and ids
  uint32_t rows = 0;
};
bool insert_scratch_bytes(const slash_index* ix, uint32_t rows, size_t* keys_bytes, size_t* runs_bytes);
slash_status insert_prepare(slash_index* ix, slash_csr rows, const InsertScratch& sc, hipStream_t st,
                            uint32_t* first_id, const GroupSignal& sig = {});
slash_status insert_commit(slash_index* ix, const InsertScratch& sc, uint32_t n, hipStream_t st);
// One serving step on `st` (see launch_serve_step): rank the queries of
// `prev` (their k in prev_kq, results to prev_ids/prev_scores, slot ids in
// prev_slots; none when prev.n_rows == 0), answer or gather (into cur_slots)
// the queries of `cur`, and commit the prepared insert sc (n rows; none when
// n == 0).  SLASH_E_UNSUPPORTED when no step kernel fits: nothing was
// launched.
struct ServeBatch {
  slash_csr q{};
  const int64_t* host_indptr = nullptr;  // q's row offsets in host memory (the first ones go in the launch)
  const uint32_t* kq = nullptr;
  uint32_t* ids = nullptr;
  uint32_t* scores = nullptr;
  uint32_t* slot_ids = nullptr;
};
bool serve_step_ok(const slash_index* ix, uint64_t n_queries);
slash_status serve_step(slash_index* ix, const ServeBatch& prev, const ServeBatch& cur, bool gather_only,
                        const InsertScratch* sc, uint32_t n, FuseSync& fs, hipStream_t st);

}  // namespace slash
