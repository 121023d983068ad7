// Host side of the C ABI: parameter checks, constant derivation, device
// memory, and the orchestration of the hash / sort / select / query kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "slash_internal.h"

using namespace slash;

// ----------------------------------------------------------------- errors

static thread_local std::string g_err;

slash_status slash::fail(slash_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                             \
  do {                                                                                            \
    hipError_t e__ = (expr);                                                                      \
    if (e__ != hipSuccess) return fail(SLASH_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e__)); \
  } while (0)

extern "C" const char* slash_last_error(void) { return g_err.c_str(); }

// -------------------------------------------------------------- allocator

static slash_alloc_fn g_alloc = nullptr;
static slash_free_fn g_free = nullptr;
static void* g_alloc_ctx = nullptr;

static void* dalloc_raw(size_t bytes) {
  if (bytes == 0) bytes = 4;
  if (g_alloc) return g_alloc(bytes, g_alloc_ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

static void dfree_raw(void* p) {
  if (!p) return;
  if (g_free)
    g_free(p, g_alloc_ctx);
  else
    (void)hipFree(p);
}

// Cache of freed device blocks (default allocator only).  A 200M-row build
// needs about 38 GB of scratch and 8.6 GB of tables; hipMalloc and hipFree of
// that much take longer than the build's kernels, so freed blocks are kept
// and handed to later allocations of up to their size (best fit, at most
// twice the request).  Every block is idle when it enters the cache: scratch
// is returned after its stream has synchronised, index memory after the
// device has drained.  When an allocation fails, the cache of that device is
// released and the allocation retried.  slash_release_cache() frees it.
namespace {
struct CachedBlock {
  void* p;
  size_t bytes;
  int device;
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;
std::map<void*, std::pair<size_t, int>> g_live;  // blocks handed out by the cache path

void release_cache(int device, bool all_devices) {
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (size_t i = 0; i < g_cache.size();) {
      if (all_devices || g_cache[i].device == device) {
        drop.push_back(g_cache[i].p);
        g_cache[i] = g_cache.back();
        g_cache.pop_back();
      } else {
        ++i;
      }
    }
  }
  for (void* p : drop) (void)hipFree(p);
}
}  // namespace

static void* dalloc(size_t bytes) {
  if (bytes == 0) bytes = 4;
  if (g_alloc) return dalloc_raw(bytes);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    size_t best = g_cache.size();
    for (size_t i = 0; i < g_cache.size(); ++i) {
      const CachedBlock& b = g_cache[i];
      if (b.device == dev && b.bytes >= bytes && b.bytes / 2 <= bytes &&
          (best == g_cache.size() || b.bytes < g_cache[best].bytes))
        best = i;
    }
    if (best != g_cache.size()) {
      CachedBlock b = g_cache[best];
      g_cache[best] = g_cache.back();
      g_cache.pop_back();
      g_live[b.p] = {b.bytes, b.device};
      return b.p;
    }
  }
  void* p = dalloc_raw(bytes);
  if (!p) {
    release_cache(dev, false);
    p = dalloc_raw(bytes);
  }
  if (p) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_live[p] = {bytes, dev};
  }
  return p;
}

static void dfree(void* p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_live.find(p);
    if (it != g_live.end()) {
      g_cache.push_back(CachedBlock{p, it->second.first, it->second.second});
      g_live.erase(it);
      return;
    }
  }
  dfree_raw(p);
}

extern "C" void slash_release_cache(void) { release_cache(0, true); }

extern "C" slash_status slash_set_allocator(slash_alloc_fn a, slash_free_fn f, void* ctx) {
  if ((a == nullptr) != (f == nullptr)) return fail(SLASH_E_INVAL, "allocator and free must both be set or both NULL");
  release_cache(0, true);
  g_alloc = a;
  g_free = f;
  g_alloc_ctx = ctx;
  return SLASH_OK;
}

// RAII device buffer for scratch.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { dfree(p); }
  bool get(size_t b) {
    if (b <= bytes && p) return true;
    dfree(p);
    p = dalloc(b);
    bytes = p ? b : 0;
    return p != nullptr;
  }
  template <class T>
  T* as() const { return (T*)p; }
};

// The build's second stream on a device (tables alternate between it and
// the caller's stream): created on first use, default priority, kept until
// the process ends.
static hipStream_t build_stream(int device) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(device);
  if (it != streams.end()) return it->second;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
  streams[device] = st;
  return st;
}

// Synchronises a stream when it goes out of scope.  Declared after the
// scratch buffers of a call, it runs before they return to the cache, so no
// block re-enters the cache while queued work may still use it (error paths
// included).
struct SyncOnExit {
  hipStream_t st;
  ~SyncOnExit() { (void)hipStreamSynchronize(st); }
};

// Grow index-owned scratch.  Work queued earlier on another stream may still
// read the old buffer, so the device is drained before it is replaced (sizes
// only grow, so this happens a few times per index).
static bool grow(DBuf& b, size_t bytes) {
  if (b.p && bytes <= b.bytes) return true;
  if (b.p && hipDeviceSynchronize() != hipSuccess) return false;
  return b.get(bytes);
}

// ------------------------------------------------------------- constants

// SplitMix64 (Steele, Lea, Flood 2014).
static uint64_t sm64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One seed gives every hash function (Section 3 "Design", Section 4
// "Initialization").  Draw order: nonzero-hash pair(s) (one, one per table,
// or one per MinHash function, by hash mode); one direction bit per
// bin; per table K odd multipliers then an offset; per table priority key and
// two odd 32-bit multipliers; per count-min row an odd multiplier and an
// offset.
static HostConsts derive_consts(const slash_params& p) {
  HostConsts h;
  uint64_t s = p.seed;
  const uint32_t M = p.K * p.L;
  const uint32_t n_h = p.hash_mode == 2 ? M : (p.hash_mode ? p.L : 1);
  for (uint32_t t = 0; t < n_h; ++t) {
    h.a_h.push_back(sm64(s) | 1u);
    h.b_h.push_back(sm64(s));
  }
  h.dirw.assign((M + 31) / 32 + 1, 0u);
  for (uint32_t b = 0; b < M; ++b)
    if (sm64(s) >> 63) h.dirw[b >> 5] |= 1u << (b & 31);
  for (uint32_t t = 0; t < p.L; ++t) {
    for (uint32_t j = 0; j < p.K; ++j) h.a_tj.push_back(sm64(s) | 1u);
    h.b_t.push_back(sm64(s));
  }
  for (uint32_t t = 0; t < p.L; ++t) {
    h.key_t.push_back((uint32_t)sm64(s));
    h.m1_t.push_back((uint32_t)sm64(s) | 1u);
    h.m2_t.push_back((uint32_t)sm64(s) | 1u);
  }
  for (uint32_t r = 0; r < p.cm_rows; ++r) {
    h.a_r.push_back(sm64(s) | 1u);
    h.b_r.push_back(sm64(s));
  }
  return h;
}

static Shape make_shape(const slash_params& p);

// Whether a query form exists for the shape: Topkapi buckets need the fold
// kernel's cells to fit; reservoir buckets need some work-group width whose
// threads hold the L * R slots (at most 16 per thread, 16 waves) and whose
// sketch or id set fits in LDS, with count-min or exact counting.
static bool queryable(const Shape& s) {
  if (s.bucket) return tk_supported(s);
  for (uint32_t w : {16u, 8u, 4u, 2u, 1u})
    if (query_supported(s, w, false) || query_supported(s, w, true)) return true;
  return false;
}

static slash_status check_params(const slash_params* p) {
  if (!p) return fail(SLASH_E_INVAL, "params is NULL");
  if (p->dim == 0) return fail(SLASH_E_INVAL, "dim must be >= 1");
  if (p->K == 0 || p->L == 0) return fail(SLASH_E_INVAL, "K and L must be >= 1");
  if ((uint64_t)p->K * p->L > 4096) return fail(SLASH_E_UNSUPPORTED, "K * L must be <= 4096");
  if (p->log2_buckets < 1 || p->log2_buckets > 30) return fail(SLASH_E_INVAL, "log2_buckets must be in [1, 30]");
  if (p->R < 1 || p->R > 256) return fail(SLASH_E_INVAL, "R must be in [1, 256]");
  if (p->cm_rows < 1 || p->cm_rows > 16) return fail(SLASH_E_INVAL, "cm_rows must be in [1, 16]");
  if (p->log2_cm_width > 16) return fail(SLASH_E_INVAL, "log2_cm_width must be <= 16");
  if (p->k_max < 1 || p->k_max > 1024) return fail(SLASH_E_INVAL, "k_max must be in [1, 1024]");
  if (p->hash_mode > 2) return fail(SLASH_E_INVAL, "hash_mode must be 0, 1 or 2");
  if (p->bucket > 1) return fail(SLASH_E_INVAL, "bucket must be 0 or 1");
  if (p->bucket == 1 && (p->log2_cm_width > 8 || (p->cm_rows << p->log2_cm_width) > 256))
    return fail(SLASH_E_UNSUPPORTED, "Topkapi buckets need log2_cm_width <= 8 and cm_rows * 2^log2_cm_width <= 256");
  if (((uint64_t)p->L << p->log2_buckets) > (1ull << 32)) return fail(SLASH_E_UNSUPPORTED, "L * 2^B must be <= 2^32");
  if ((uint64_t)p->L * p->R > 65535) return fail(SLASH_E_UNSUPPORTED, "L * R must be <= 65535");
  // an index is built only if it can be queried
  if (!queryable(make_shape(*p)))
    return fail(SLASH_E_UNSUPPORTED,
                p->bucket ? "Topkapi cells per bucket too many for the query kernel"
                          : "no query form fits: L * R above 16384 slots, or the count-min (cm_rows x 2^log2_cm_width "
                            "8-bit counters) too large for LDS");
  return SLASH_OK;
}

// -------------------------------------------------------------- the index

struct GraphSlot {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t fill = nullptr, hash = nullptr, run = nullptr;
  uint32_t waves = 0, per_ticket = 0, grid = 0;
};

// Event pairs around every launch of a phase; read after the stream syncs.
struct EventTimer : PhaseTimer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[PH_COUNT];
  hipEvent_t open[PH_COUNT] = {};
  void begin(int ph, hipStream_t st) override {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    open[ph] = e;
  }
  void end(int ph, hipStream_t st) override {
    if (!open[ph]) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    ev[ph].emplace_back(open[ph], e);
    open[ph] = nullptr;
  }
  // total ms and launches per phase (events must have completed)
  void collect(double* ms, uint32_t* n) {
    for (int p = 0; p < PH_COUNT; ++p) {
      ms[p] = 0;
      n[p] = (uint32_t)ev[p].size();
      for (auto& pr : ev[p]) {
        float t = 0;
        if (hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) ms[p] += t;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
      }
      ev[p].clear();
    }
  }
  ~EventTimer() override {
    double ms[PH_COUNT];
    uint32_t n[PH_COUNT];
    collect(ms, n);
  }
};

static const char* kPhaseNames[PH_COUNT] = {"validate", "hash", "sort_upsweep", "sort_scan", "sort_downsweep",
                                            "segment_bounds", "select", "heavy"};

struct slash_index {
  slash_params p{};
  double phase_ms[PH_COUNT] = {};
  uint32_t phase_n[PH_COUNT] = {};
  double phase_bytes[PH_COUNT] = {};
  Shape shape{};
  HostConsts hc;
  int device = 0;
  int n_cu = 0;
  uint64_t n_items = 0;
  void* d_consts = nullptr;
  ConstView cv{};
  uint32_t* ids = nullptr;
  uint32_t* seen = nullptr;
  uint32_t* flag = nullptr;     // validation flag
  uint32_t* tickets = nullptr;  // ring of work counters for the batched path
  uint32_t ticket_next = 0;
  DBuf ins_keys, ins_vals, ins_k0, ins_v0, ins_k1, ins_v1, ins_hist, ins_part, ins_seg;
  DBuf qbk;  // bucket ids of the batched path's queries [n][L]
  std::mutex mu;
  std::map<uint64_t, GraphSlot> graphs;
  // tuned schedule per query-size class (0: nnz < 64, 1: < 256, 2: < 1024, 3: larger)
  slash_schedule tuned[4];
  bool has_tuned[4] = {false, false, false, false};
};

static const uint32_t kTicketRing = 256;

static TablesView tables(const slash_index* ix) { return TablesView{ix->ids, ix->seen}; }

// 32-bit words a bucket occupies in the table array: R ids, or the Topkapi
// sketch's cells of two words each.
static uint64_t bucket_words(const Shape& s) { return s.bucket ? 2ull * (s.d << s.lw) : s.R; }

static Shape make_shape(const slash_params& p) {
  Shape s;
  s.dim = p.dim;
  s.K = p.K;
  s.L = p.L;
  s.M = p.K * p.L;
  s.B = p.log2_buckets;
  s.R = p.R;
  s.d = p.cm_rows;
  s.lw = p.log2_cm_width;
  s.k_max = p.k_max;
  s.mode = p.hash_mode;
  s.bucket = p.bucket;
  s.nb = 1u << p.log2_buckets;
  s.mshift = 0xFFu;
  if ((s.M & (s.M - 1)) == 0) {
    uint32_t m = 0;
    while ((1u << m) < s.M) ++m;
    s.mshift = m;
  }
  return s;
}

// One contiguous table; kernels stage its leading part (the u64 arrays, then
// the direction words) into LDS as a flat copy, so this order is fixed.
static slash_status upload_consts(slash_index* ix, hipStream_t st) {
  const HostConsts& h = ix->hc;
  std::vector<uint64_t> u64;
  size_t o_ah = u64.size();
  u64.insert(u64.end(), h.a_h.begin(), h.a_h.end());
  size_t o_bh = u64.size();
  u64.insert(u64.end(), h.b_h.begin(), h.b_h.end());
  size_t o_atj = u64.size();
  u64.insert(u64.end(), h.a_tj.begin(), h.a_tj.end());
  size_t o_bt = u64.size();
  u64.insert(u64.end(), h.b_t.begin(), h.b_t.end());
  size_t o_ar = u64.size();
  u64.insert(u64.end(), h.a_r.begin(), h.a_r.end());
  size_t o_br = u64.size();
  u64.insert(u64.end(), h.b_r.begin(), h.b_r.end());
  std::vector<uint32_t> u32;
  size_t o_dir = u32.size();
  u32.insert(u32.end(), h.dirw.begin(), h.dirw.end());
  size_t o_key = u32.size();
  u32.insert(u32.end(), h.key_t.begin(), h.key_t.end());
  size_t o_m1 = u32.size();
  u32.insert(u32.end(), h.m1_t.begin(), h.m1_t.end());
  size_t o_m2 = u32.size();
  u32.insert(u32.end(), h.m2_t.begin(), h.m2_t.end());
  size_t bytes = u64.size() * 8 + u32.size() * 4;
  ix->d_consts = dalloc(bytes);
  if (!ix->d_consts) return fail(SLASH_E_NOMEM, "constant table allocation failed");
  uint8_t* base = (uint8_t*)ix->d_consts;
  HIP_TRY(hipMemcpy(base, u64.data(), u64.size() * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(base + u64.size() * 8, u32.data(), u32.size() * 4, hipMemcpyHostToDevice));
  const uint64_t* d64 = (const uint64_t*)base;
  const uint32_t* d32 = (const uint32_t*)(base + u64.size() * 8);
  ix->cv.a_h = d64 + o_ah;
  ix->cv.b_h = d64 + o_bh;
  ix->cv.a_tj = d64 + o_atj;
  ix->cv.b_t = d64 + o_bt;
  ix->cv.a_r = d64 + o_ar;
  ix->cv.b_r = d64 + o_br;
  ix->cv.dirw = d32 + o_dir;
  ix->cv.key_t = d32 + o_key;
  ix->cv.m1_t = d32 + o_m1;
  ix->cv.m2_t = d32 + o_m2;
  (void)st;
  return SLASH_OK;
}

static void destroy_index(slash_index* ix) {
  if (!ix) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : ix->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  dfree(ix->d_consts);
  dfree(ix->ids);
  dfree(ix->seen);
  dfree(ix->flag);
  dfree(ix->tickets);
  delete ix;
}

extern "C" void slash_free(slash_index* ix) { destroy_index(ix); }

// Device-side validation of rows (and per-query k); reads back one flag.
// Checks rows (non-empty, indptr increasing), per-query k and, unless
// check_indices is false (the build checks indices while hashing them), that
// every index is in [0, dim).
static slash_status validate_rows(slash_index* ix, slash_csr rows, const uint32_t* kq, hipStream_t st,
                                  PhaseTimer* timer = nullptr, int64_t* nnz_out = nullptr,
                                  bool check_indices = true) {
  if (rows.n_rows == 0) return SLASH_OK;
  if (!rows.indptr || !rows.indices) return fail(SLASH_E_INVAL, "CSR pointers are NULL");
  int64_t ends[2];
  HIP_TRY(hipMemcpyAsync(&ends[0], rows.indptr, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&ends[1], rows.indptr + rows.n_rows, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ends[1] < ends[0]) return fail(SLASH_E_INVAL, "indptr is decreasing");
  if (nnz_out) *nnz_out = ends[1] - ends[0];
  HIP_TRY(launch_fill_u32(ix->flag, 0u, 1, st));
  if (timer) timer->begin(PH_VALIDATE, st);
  HIP_TRY(launch_validate(rows, ix->p.dim, kq, ix->p.k_max, ix->flag, st));
  if (check_indices)
    HIP_TRY(launch_validate_indices(rows.indices + ends[0], (uint64_t)(ends[1] - ends[0]), ix->p.dim, ix->flag, st));
  if (timer) timer->end(PH_VALIDATE, st);
  uint32_t f = 0;
  HIP_TRY(hipMemcpyAsync(&f, ix->flag, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (f & 1u) return fail(SLASH_E_INVAL, "a row is empty (or indptr decreases)");
  if (f & 2u) return fail(SLASH_E_INVAL, "a feature index is outside [0, dim)");
  if (f & 4u) return fail(SLASH_E_INVAL, "a per-query k exceeds k_max");
  return SLASH_OK;
}

static int ceil_log2(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

// ------------------------------------------------------------------ build

// Ids one wave reduces per bucket or chunk: reservoir buckets above kHeavy go
// to the chunked heavy path (4096, 8192 and 32768 measured slower on the
// 200M-row shard); the Topkapi heavy kernels work in chunks of kHeavyTk ids
// and take the buckets above it.
static const uint32_t kHeavy = 16384;
static const uint32_t kHeavyTk = 16384;

static slash_status reserve_small_inserts(slash_index* ix);

static slash_status alloc_tables(slash_index* ix) {
  const Shape& s = ix->shape;
  size_t n_ids = (size_t)s.L * s.nb * bucket_words(s);
  ix->ids = (uint32_t*)dalloc(n_ids * 4);
  ix->seen = (uint32_t*)dalloc((size_t)s.L * s.nb * 4);
  ix->flag = (uint32_t*)dalloc(64);
  ix->tickets = (uint32_t*)dalloc(kTicketRing * 4);
  if (!ix->ids || !ix->seen || !ix->flag || !ix->tickets) return fail(SLASH_E_NOMEM, "table allocation failed (%zu bytes)", n_ids * 4);
  return SLASH_OK;
}

extern "C" slash_status slash_build(const slash_params* params, slash_csr data, void* stream, slash_index** out) {
  if (!out) return fail(SLASH_E_INVAL, "out is NULL");
  slash_status rs = check_params(params);
  if (rs != SLASH_OK) return rs;
  if (data.n_rows > 0xFFFFFFFEull) return fail(SLASH_E_CAPACITY, "more than 2^32-2 rows");
  hipStream_t st = (hipStream_t)stream;
  slash_index* ix = new (std::nothrow) slash_index();
  if (!ix) return fail(SLASH_E_NOMEM, "host allocation failed");
  ix->p = *params;
  ix->shape = make_shape(*params);
  ix->hc = derive_consts(*params);
  HIP_TRY(hipGetDevice(&ix->device));
  HIP_TRY(hipDeviceGetAttribute(&ix->n_cu, hipDeviceAttributeMultiprocessorCount, ix->device));
  auto bail = [&](slash_status s) {
    destroy_index(ix);
    return s;
  };
  if ((rs = upload_consts(ix, st)) != SLASH_OK) return bail(rs);
  if ((rs = alloc_tables(ix)) != SLASH_OK) return bail(rs);
  EventTimer timer;
  int64_t nnz = 0;
  if ((rs = validate_rows(ix, data, nullptr, st, &timer, &nnz, false)) != SLASH_OK) return bail(rs);
  const Shape& s = ix->shape;
  const uint64_t n = data.n_rows;
  if (n == 0) {
    // a non-empty build writes every bucket's slots (or cells) and seen
    // count in its select pass, so only an empty one clears the tables
    hipError_t e = s.bucket ? launch_tk_clear(s, tables(ix), st)
                            : launch_fill_u32(ix->ids, SL_EMPTY, (uint64_t)s.L * s.nb * s.R, st);
    if (e == hipSuccess) e = launch_fill_u32(ix->seen, 0u, (uint64_t)s.L * s.nb, st);
    if (e != hipSuccess) return bail(fail(SLASH_E_DEVICE, "table init: %s", hipGetErrorString(e)));
  }
  if (n > 0) {
    // Tables alternate between the caller's stream and a second stream, each
    // with its own sort and select scratch, so the phases of one table that
    // leave most of the GPU idle (single-block planning and scans, launch
    // gaps, the tail of a heavy bucket's merge) overlap another table's
    // kernels.  The tables are independent; the host waits for both streams.
    struct TableScratch {
      DBuf k0, v0, k1, v1, hist, part, start, end, heavy, heavy_n, hchunks, hfinals, hcount, hcand, tkh;
    };
    DBuf keys;
    TableScratch ts[2];
    hipStream_t st2 = build_stream(ix->device);
    if (!st2) return bail(fail(SLASH_E_DEVICE, "build stream creation failed"));
    SyncOnExit drain{st}, drain2{st2};
    size_t hist_n = sort_hist_entries(n);
    size_t part_n = std::max(sort_part_entries(hist_n), sort_part_entries(n)) + 16;
    const size_t hcap = heavy_chunk_capacity(n, kHeavy);
    if (!keys.get((size_t)s.L * n * 4)) return bail(fail(SLASH_E_NOMEM, "build scratch allocation failed"));
    for (TableScratch& x : ts)
      if (!x.k0.get(n * 4) || !x.v0.get(n * 4) || !x.k1.get(n * 4) || !x.v1.get(n * 4) || !x.hist.get(hist_n * 4) ||
          !x.part.get(part_n * 4) || !x.start.get((size_t)s.nb * 4) || !x.end.get((size_t)s.nb * 4) ||
          !x.heavy.get((size_t)s.nb * 12) || !x.heavy_n.get(4) || !x.hchunks.get(hcap * sizeof(ChunkWork)) ||
          !x.hfinals.get((n / kHeavy + 1) * sizeof(FinalWork)) || !x.hcount.get(4) ||
          !x.hcand.get(hcap * s.R * 4) || (s.bucket && !x.tkh.get(tk_heavy_scratch_words(s, n / kHeavyTk + 1) * 4)))
        return bail(fail(SLASH_E_NOMEM, "build scratch allocation failed"));
    // the hash kernel also checks every index against [0, dim) (flag bit 2)
    ConstView cvb = ix->cv;
    cvb.bad = ix->flag;
    timer.begin(PH_HASH, st);
    hipError_t e = launch_hash_rows(s, cvb, data, keys.as<uint32_t>(), n, 0, st);
    timer.end(PH_HASH, st);
    if (e != hipSuccess) return bail(fail(SLASH_E_DEVICE, "hash: %s", hipGetErrorString(e)));
    {
      uint32_t f = 0;
      e = hipMemcpyAsync(&f, ix->flag, 4, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return bail(fail(SLASH_E_DEVICE, "hash: %s", hipGetErrorString(e)));
      if (f & 2u) return bail(fail(SLASH_E_INVAL, "a feature index is outside [0, dim)"));
    }
    // every table is enqueued back to back: heavy buckets are planned and
    // finished on the device, so the host never waits between tables
    // the packed sort (ids below 2^28, keys below 2^20) writes the bucket
    // runs itself; otherwise the sorted keys are scanned for them
    const bool packed = packed_sort_ok(n, (int)s.B);
    for (uint32_t t = 0; t < s.L; ++t) {
      TableScratch& x = ts[t & 1];
      const hipStream_t tst = (t & 1) ? st2 : st;
      SortBuffers sb{x.k0.as<uint32_t>(), x.v0.as<uint32_t>(), x.k1.as<uint32_t>(), x.v1.as<uint32_t>(),
                     x.hist.as<uint32_t>(), x.part.as<uint32_t>()};
      DBuf &start = x.start, &end = x.end, &heavy = x.heavy, &heavy_n = x.heavy_n, &hchunks = x.hchunks,
           &hfinals = x.hfinals, &hcount = x.hcount, &hcand = x.hcand, &tkh = x.tkh;
      uint32_t *sk = nullptr, *sv = nullptr;
      const uint32_t* tkeys = keys.as<uint32_t>() + (uint64_t)t * n;
      e = launch_fill_u32(start.as<uint32_t>(), 0u, s.nb, tst);
      if (e == hipSuccess) e = launch_fill_u32(end.as<uint32_t>(), 0u, s.nb, tst);
      if (e == hipSuccess) e = launch_fill_u32(heavy_n.as<uint32_t>(), 0u, 1, tst);
      if (e == hipSuccess && packed) {
        e = radix_sort_runs(tkeys, n, (int)s.B, sb, start.as<uint32_t>(), end.as<uint32_t>(), &sv, tst, &timer);
      } else if (e == hipSuccess) {
        e = radix_sort(tkeys, nullptr, n, (int)s.B, sb, &sk, &sv, tst, &timer);
        timer.begin(PH_BOUNDS, tst);
        if (e == hipSuccess) e = launch_segment_bounds(sk, n, start.as<uint32_t>(), end.as<uint32_t>(), tst);
        timer.end(PH_BOUNDS, tst);
      }
      timer.begin(PH_SELECT, tst);
      if (e == hipSuccess && s.bucket)
        e = launch_tk_light(s, ix->cv, t, sv, start.as<uint32_t>(), end.as<uint32_t>(), tables(ix), kHeavyTk,
                            heavy.as<uint32_t>(), heavy_n.as<uint32_t>(), tkh.as<uint32_t>(), tst);
      else if (e == hipSuccess)
        e = launch_select_light(s, ix->cv, t, sv, start.as<uint32_t>(), end.as<uint32_t>(), tables(ix), kHeavy,
                                heavy.as<uint32_t>(), heavy_n.as<uint32_t>(), tst);
      timer.end(PH_SELECT, tst);
      timer.begin(PH_HEAVY, tst);
      if (e == hipSuccess && s.bucket)
        e = launch_tk_heavy(s, ix->cv, t, sv, start.as<uint32_t>(), end.as<uint32_t>(), tables(ix),
                            heavy.as<uint32_t>(), heavy_n.as<uint32_t>(), n, tkh.as<uint32_t>(), tst);
      else if (e == hipSuccess)
        e = launch_heavy(s, ix->cv, t, sv, n, heavy.as<uint32_t>(), heavy_n.as<uint32_t>(), kHeavy,
                         hchunks.as<ChunkWork>(), hfinals.as<FinalWork>(), hcount.as<uint32_t>(), hcand.as<uint32_t>(),
                         tables(ix), tst);
      timer.end(PH_HEAVY, tst);
      if (e != hipSuccess) return bail(fail(SLASH_E_DEVICE, "build table %u: %s", t, hipGetErrorString(e)));
    }
    e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipStreamSynchronize(st2);
    if (e != hipSuccess) return bail(fail(SLASH_E_DEVICE, "build: %s", hipGetErrorString(e)));
  }
  HIP_TRY(hipStreamSynchronize(st));
  timer.collect(ix->phase_ms, ix->phase_n);
  {
    // algorithmic bytes: what each phase must read and write once
    const double N = (double)n, L = s.L, NB = s.nb;
    const int passes = (int)(s.B + 7) / 8;
    ix->phase_bytes[PH_VALIDATE] = 4.0 * nnz + 8.0 * (N + 1);
    ix->phase_bytes[PH_HASH] = 4.0 * nnz + 8.0 * (N + 1) + 4.0 * L * N;
    if (packed_sort_ok(n, (int)s.B)) {
      // counts read 4 B keys, then 2 B low halves (digits below bit 16) or
      // 4 B words; a scatter reads 4 B keys (first pass) or 6 B packed items
      // and writes 6 B packed items, or 4 B ids (last pass) and the runs
      double up = 0, down = 0;
      for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p, bits = std::min(8, (int)s.B - shift);
        up += p == 0 ? 4.0 : (shift + bits <= 16 ? 2.0 : 4.0);
        down += (p == 0 ? 4.0 : 6.0) + (p + 1 == passes ? 4.0 : 6.0);
      }
      ix->phase_bytes[PH_UPSWEEP] = up * N * L;
      ix->phase_bytes[PH_DOWNSWEEP] = down * N * L;
      ix->phase_bytes[PH_BOUNDS] = 8.0 * NB * L;  // the runs, written once
    } else {
      ix->phase_bytes[PH_UPSWEEP] = 4.0 * N * L * passes;
      ix->phase_bytes[PH_DOWNSWEEP] = L * (12.0 * N + (passes - 1) * 16.0 * N);
      ix->phase_bytes[PH_BOUNDS] = 4.0 * N * L + 8.0 * NB * L;
    }
    ix->phase_bytes[PH_SELECT] = L * (4.0 * N + 8.0 * NB + NB * (4.0 * (double)bucket_words(s) + 4.0));
  }
  ix->n_items = n;
  // scratch for insert batches of up to 4096 rows, so that the first insert
  // allocates nothing
  if ((rs = reserve_small_inserts(ix)) != SLASH_OK) return bail(rs);
  *out = ix;
  return SLASH_OK;
}

// ----------------------------------------------------------------- insert

static slash_status reserve_small_inserts(slash_index* ix) {
  uint64_t rows = 4096;
  while (rows > 1 && !small_insert_ok(ix->shape, rows)) rows /= 2;
  return slash::reserve_insert_scratch(ix, rows);
}

slash_status slash::reserve_insert_scratch(slash_index* ix, uint64_t rows) {
  if (!ix) return fail(SLASH_E_INVAL, "index is NULL");
  if (!small_insert_ok(ix->shape, rows)) return SLASH_OK;
  std::lock_guard<std::mutex> lk(ix->mu);
  if (!grow(ix->ins_keys, (size_t)rows * ix->shape.L * 4) || !grow(ix->ins_seg, small_insert_scratch(ix->shape, rows)))
    return fail(SLASH_E_NOMEM, "insert scratch allocation failed");
  return SLASH_OK;
}

extern "C" slash_status slash_insert(slash_index* ix, slash_csr rows, uint32_t flags, uint32_t* new_ids_dev,
                                     void* stream) {
  return slash::insert_rows(ix, rows, flags, new_ids_dev, (hipStream_t)stream);
}

bool slash::insert_scratch_bytes(const slash_index* ix, uint32_t rows, size_t* keys_bytes, size_t* runs_bytes) {
  if (!ix || !small_insert_ok(ix->shape, rows)) return false;
  *keys_bytes = (size_t)rows * ix->shape.L * 4;
  *runs_bytes = small_insert_scratch(ix->shape, rows);
  return true;
}

slash_status slash::insert_prepare(slash_index* ix, slash_csr rows, const InsertScratch& sc, hipStream_t st,
                                   uint32_t* first_id, const GroupSignal& sig) {
  if (!ix || !first_id) return fail(SLASH_E_INVAL, "NULL argument");
  const uint64_t n = rows.n_rows;
  if (n == 0 || n > sc.rows || !small_insert_ok(ix->shape, n))
    return fail(SLASH_E_INVAL, "insert of %llu rows does not fit the scratch", (unsigned long long)n);
  std::lock_guard<std::mutex> lk(ix->mu);
  if (ix->n_items + n > 0xFFFFFFFFull) return fail(SLASH_E_CAPACITY, "ids would exceed 0xFFFFFFFE");
  const uint32_t first = (uint32_t)ix->n_items;
  HIP_TRY(launch_hash_rows(ix->shape, ix->cv, rows, sc.keys, n, 0, st));
  HIP_TRY(launch_insert_group(ix->shape, sc.keys, (uint32_t)n, first, sc.runs, st, sig));
  ix->n_items += n;
  *first_id = first;
  return SLASH_OK;
}

slash_status slash::insert_commit(slash_index* ix, const InsertScratch& sc, uint32_t n, hipStream_t st) {
  if (!ix || n == 0 || n > sc.rows) return fail(SLASH_E_INVAL, "bad insert commit");
  HIP_TRY(launch_insert_runs(ix->shape, ix->cv, sc.runs, n, tables(ix), st));
  return SLASH_OK;
}

bool slash::serve_step_ok(const slash_index* ix, uint64_t n_queries) {
  // one 16-wave work-group per query: the batches slash_query runs that way
  return ix && n_queries * 2 <= (uint64_t)ix->n_cu && serve_step_supported(ix->shape);
}

slash_status slash::serve_step(slash_index* ix, const ServeBatch& prev, const ServeBatch& cur, bool gather_only,
                               const InsertScratch* sc, uint32_t n, FuseSync& fs, hipStream_t st) {
  if (!ix || (n && (!sc || n > sc->rows))) return fail(SLASH_E_INVAL, "bad serving step");
  for (const ServeBatch* b : {&prev, &cur})
    if (b->q.n_rows && (!b->kq || !b->ids || !b->scores)) return fail(SLASH_E_INVAL, "bad serving step batch");
  if (!serve_step_ok(ix, prev.q.n_rows) || !serve_step_ok(ix, cur.q.n_rows))
    return fail(SLASH_E_UNSUPPORTED, "no serving step kernel fits");
  QueryArgs pa{prev.q, prev.kq, 0, 1, prev.ids, prev.scores, nullptr};
  pa.slot_ids = prev.slot_ids;
  QueryArgs ca{cur.q, cur.kq, 0, 1, cur.ids, cur.scores, nullptr};
  ca.slot_ids = cur.slot_ids;
  const hipError_t e = launch_serve_step(ix->shape, ix->cv, tables(ix), pa, ca, gather_only, n ? sc->runs : nullptr, n,
                                         ix->n_cu, fs, st, cur.host_indptr);
  if (e == hipErrorNotSupported) return fail(SLASH_E_UNSUPPORTED, "no serving step kernel fits");
  if (e == hipErrorInvalidValue) return fail(SLASH_E_INVAL, "malformed serving step");
  HIP_TRY(e);
  return SLASH_OK;
}

slash_status slash::insert_rows(slash_index* ix, slash_csr rows, uint32_t flags, uint32_t* new_ids_dev,
                                hipStream_t st) {
  if (!ix) return fail(SLASH_E_INVAL, "index is NULL");
  const uint64_t n = rows.n_rows;
  if (n == 0) return SLASH_OK;
  if (ix->n_items + n > 0xFFFFFFFFull) return fail(SLASH_E_CAPACITY, "ids would exceed 0xFFFFFFFE");
  std::lock_guard<std::mutex> lk(ix->mu);
  slash_status rs;
  if (!(flags & SLASH_FLAG_TRUSTED) && (rs = validate_rows(ix, rows, nullptr, st)) != SLASH_OK) return rs;
  const Shape& s = ix->shape;
  const uint32_t first = (uint32_t)ix->n_items;
  if (small_insert_ok(s, n)) {
    // three launches: hash the rows, sort per table in LDS, merge every run
    if (!grow(ix->ins_keys, (size_t)n * s.L * 4) || !grow(ix->ins_seg, small_insert_scratch(s, n)))
      return fail(SLASH_E_NOMEM, "insert scratch allocation failed");
    HIP_TRY(launch_hash_rows(s, ix->cv, rows, ix->ins_keys.as<uint32_t>(), n, 0, st));
    HIP_TRY(launch_insert_small(s, ix->cv, ix->ins_keys.as<uint32_t>(), (uint32_t)n, first, ix->ins_seg.p, tables(ix),
                                st));
    if (new_ids_dev) HIP_TRY(launch_iota_u32(new_ids_dev, first, n, st));
    ix->n_items += n;
    return SLASH_OK;
  }
  const uint64_t items = n * s.L;
  if (items >= 0xFFFFFFFFull) return fail(SLASH_E_UNSUPPORTED, "insert batch too large");
  size_t hist_n = sort_hist_entries(items);
  size_t part_n = std::max(sort_part_entries(hist_n), sort_part_entries(items)) + 16;
  if (!grow(ix->ins_keys, items * 4) || !grow(ix->ins_vals, items * 4) || !grow(ix->ins_k0, items * 4) ||
      !grow(ix->ins_v0, items * 4) || !grow(ix->ins_k1, items * 4) || !grow(ix->ins_v1, items * 4) ||
      !grow(ix->ins_hist, hist_n * 4) || !grow(ix->ins_part, part_n * 4) || !grow(ix->ins_seg, (2 * items + 4) * 4))
    return fail(SLASH_E_NOMEM, "insert scratch allocation failed");
  HIP_TRY(launch_hash_rows(s, ix->cv, rows, ix->ins_keys.as<uint32_t>(), n, 1, st));
  HIP_TRY(launch_item_ids(ix->ins_vals.as<uint32_t>(), first, n, items, st));
  SortBuffers sb{ix->ins_k0.as<uint32_t>(), ix->ins_v0.as<uint32_t>(), ix->ins_k1.as<uint32_t>(),
                 ix->ins_v1.as<uint32_t>(), ix->ins_hist.as<uint32_t>(), ix->ins_part.as<uint32_t>()};
  uint32_t *sk = nullptr, *sv = nullptr;
  int bits = (int)s.B + ceil_log2(s.L);
  HIP_TRY(radix_sort(ix->ins_keys.as<uint32_t>(), ix->ins_vals.as<uint32_t>(), items, bits, sb, &sk, &sv, st));
  HIP_TRY(launch_insert_merge(s, ix->cv, sk, sv, items, ix->ins_seg.as<uint32_t>(), ix->ins_part.as<uint32_t>(),
                              tables(ix), st));
  if (new_ids_dev) HIP_TRY(launch_iota_u32(new_ids_dev, first, n, st));
  ix->n_items += n;
  return SLASH_OK;
}

// ------------------------------------------------------------------ query

static slash_status query_prelude(const slash_index* ix, slash_csr q, const uint32_t* kq, uint32_t k, uint32_t flags,
                                  uint32_t* ids, uint32_t* scores, hipStream_t st) {
  if (!ix) return fail(SLASH_E_INVAL, "index is NULL");
  if (q.n_rows && (!ids || !scores)) return fail(SLASH_E_INVAL, "output pointers are NULL");
  if (!kq && k > ix->p.k_max) return fail(SLASH_E_INVAL, "k (%u) exceeds k_max (%u)", k, ix->p.k_max);
  if (ix->shape.bucket && (flags & SLASH_FLAG_EXACT))
    return fail(SLASH_E_UNSUPPORTED, "exact counting needs reservoir buckets");
  if (ix->shape.bucket ? !tk_supported(ix->shape)
                       : !query_supported(ix->shape, query_default_waves(ix->shape), (flags & SLASH_FLAG_EXACT) != 0))
    return fail(SLASH_E_UNSUPPORTED, "query shape not supported (count-min or id set too large for LDS)");
  if (!(flags & SLASH_FLAG_TRUSTED))
    return validate_rows(const_cast<slash_index*>(ix), q, kq, st);
  return SLASH_OK;
}

extern "C" slash_status slash_query(const slash_index* ix, slash_csr q, const uint32_t* kq, uint32_t k, uint32_t flags,
                                    uint32_t* ids, uint32_t* scores, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  slash_status rs = query_prelude(ix, q, kq, k, flags, ids, scores, st);
  if (rs != SLASH_OK) return rs;
  if (q.n_rows == 0) return SLASH_OK;
  QueryArgs a{q, kq, k, 1, ids, scores, nullptr};
  a.exact = (flags & SLASH_FLAG_EXACT) ? 1u : 0u;
  if (ix->shape.bucket) {
    HIP_TRY(launch_tk_query(ix->shape, ix->cv, tables(ix), a, st));
    return SLASH_OK;
  }
  // A batch too small to occupy the GPU runs each query with 16 waves
  // (shorter per-query latency); larger batches use the default width.
  uint32_t waves = query_default_waves(ix->shape);
  if (q.n_rows * 2 <= (uint64_t)ix->n_cu && query_supported(ix->shape, 16u, a.exact != 0)) waves = 16;
  HIP_TRY(launch_query_waves(ix->shape, ix->cv, tables(ix), a, waves, st));
  return SLASH_OK;
}

static uint32_t size_class(double mean_nnz) {
  if (mean_nnz < 64) return 0;
  if (mean_nnz < 256) return 1;
  if (mean_nnz < 1024) return 2;
  return 3;
}

static slash_schedule default_schedule(const slash_index* ix) {
  slash_schedule sc{query_default_waves(ix->shape), 1, 0, 0};
  return sc;
}

// Graph = [reset work counter, hash all queries (row-parallel), persistent
// query kernel reading the bucket ids]; node arguments are updated per call.
static slash_status run_batched(slash_index* ix, const QueryArgs& a0, const slash_schedule& sc, hipStream_t st) {
  QueryArgs a = a0;
  const Shape& s = ix->shape;
  uint32_t waves = sc.waves_per_query;
  if (!query_supported(s, waves, a.exact != 0))
    return fail(SLASH_E_UNSUPPORTED, "schedule with %u waves/query not supported", waves);
  int occ = 0;
  HIP_TRY(query_occupancy(s, waves, &occ, a.exact != 0));
  if (occ < 1) occ = 1;
  // queries_per_ticket 0: the grid-stride kernel, one work-group per query
  const bool plain = sc.queries_per_ticket == 0;
  uint32_t per_cu = sc.groups_per_cu ? std::min<uint32_t>(sc.groups_per_cu, (uint32_t)occ) : (uint32_t)occ;
  uint32_t grid = per_cu * (uint32_t)ix->n_cu;
  uint64_t max_grid = (a.q.n_rows + std::max(1u, sc.queries_per_ticket) - 1) / std::max(1u, sc.queries_per_ticket);
  if (grid > max_grid) grid = (uint32_t)std::max<uint64_t>(1, max_grid);
  uint32_t per_ticket = plain ? 0u : std::max(1u, sc.queries_per_ticket);
  if (plain) grid = (uint32_t)std::min<uint64_t>(a.q.n_rows, 1u << 30);
  std::lock_guard<std::mutex> lk(ix->mu);
  const size_t need = (size_t)a.q.n_rows * s.L * 4;
  if (!grow(ix->qbk, need)) return fail(SLASH_E_NOMEM, "batched bucket-id buffer");
  a.qbk = ix->qbk.as<uint32_t>();
  uint32_t* ticket = ix->tickets + (ix->ticket_next++ % kTicketRing);
  uint32_t hash_threads = 0;
  size_t hash_lds = 0;
  void* hash_fn = hash_rowmajor_kernel(s, &hash_threads, &hash_lds);
  if (!hash_fn) return fail(SLASH_E_DEVICE, "hash kernel attributes");
  const uint32_t hash_grid = hash_rowmajor_grid(s, a.q.n_rows);
  // the plain form's grid follows the batch size and is updated in place (its
  // grid-stride loop is correct for any grid)
  uint64_t gkey = ((uint64_t)a.exact << 63) | ((uint64_t)waves << 48) | ((uint64_t)per_ticket << 32) | (plain ? 0u : grid);
  GraphSlot& g = ix->graphs[gkey];
  Shape sh = s;
  ConstView cv = ix->cv;
  TablesView tv = tables(ix);
  QueryArgs qa = a;
  uint32_t zero = 0;
  uint64_t one = 1;
  void* run_args[] = {&sh, &cv, &tv, &qa, &per_ticket, &ticket};
  void* plain_args[] = {&sh, &cv, &tv, &qa};
  uint32_t* tk = ticket;
  void* fill_args[] = {&tk, &zero, &one};
  slash_csr hq = a.q;
  uint32_t* hout = const_cast<uint32_t*>(a.qbk);
  void* hash_args[] = {&sh, &cv, &hq, &hout};
  hipKernelNodeParams hp{};
  hp.func = hash_fn;
  hp.gridDim = dim3(hash_grid);
  hp.blockDim = dim3(hash_threads);
  hp.sharedMemBytes = (unsigned)hash_lds;
  hp.kernelParams = hash_args;
  hipKernelNodeParams rp{};
  rp.func = plain ? plain_query_kernel(s, waves, a.exact != 0) : persistent_query_kernel(s, waves, a.exact != 0);
  rp.gridDim = dim3(grid);
  rp.blockDim = dim3(waves * SL_WAVE);
  rp.sharedMemBytes = (unsigned)query_lds_bytes(s, waves, a.exact != 0);
  rp.kernelParams = plain ? plain_args : run_args;
  hipKernelNodeParams fp{};
  fp.func = fill_kernel_ptr();
  fp.gridDim = dim3(1);
  fp.blockDim = dim3(64);
  fp.sharedMemBytes = 0;
  fp.kernelParams = fill_args;
  if (!g.exec) {
    HIP_TRY(hipGraphCreate(&g.graph, 0));
    HIP_TRY(hipGraphAddKernelNode(&g.fill, g.graph, nullptr, 0, &fp));
    HIP_TRY(hipGraphAddKernelNode(&g.hash, g.graph, &g.fill, 1, &hp));
    HIP_TRY(hipGraphAddKernelNode(&g.run, g.graph, &g.hash, 1, &rp));
    HIP_TRY(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
  } else {
    HIP_TRY(hipGraphExecKernelNodeSetParams(g.exec, g.fill, &fp));
    HIP_TRY(hipGraphExecKernelNodeSetParams(g.exec, g.hash, &hp));
    HIP_TRY(hipGraphExecKernelNodeSetParams(g.exec, g.run, &rp));
  }
  HIP_TRY(hipGraphLaunch(g.exec, st));
  return SLASH_OK;
}

// Schedule of a batched call: the caller's, else the tuned one (several
// tuned size classes: the batch's mean row size picks the nearest), else the
// default.
static slash_status batched_schedule(const slash_index* ix, slash_csr q, const slash_schedule* sched, hipStream_t st,
                                     slash_schedule* out) {
  slash_schedule sc = default_schedule(ix);
  if (sched) {
    sc = *sched;
  } else {
    int n_tuned = 0, only = -1;
    for (int c = 0; c < 4; ++c)
      if (ix->has_tuned[c]) {
        ++n_tuned;
        only = c;
      }
    if (n_tuned == 1) {
      sc = ix->tuned[only];
    } else if (n_tuned > 1) {
      // several size classes tuned: the batch's mean row size picks one (the
      // nearest tuned class)
      int64_t ends[2];
      HIP_TRY(hipMemcpyAsync(&ends[0], q.indptr, 8, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(&ends[1], q.indptr + q.n_rows, 8, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      const int cls = (int)size_class((double)(ends[1] - ends[0]) / (double)q.n_rows);
      int best = -1;
      for (int c = 0; c < 4; ++c)
        if (ix->has_tuned[c] && (best < 0 || std::abs(c - cls) < std::abs(best - cls))) best = c;
      sc = ix->tuned[best];
    }
  }
  *out = sc;
  return SLASH_OK;
}

extern "C" slash_status slash_query_batched(const slash_index* cix, slash_csr q, const uint32_t* kq, uint32_t k,
                                            uint32_t flags, uint32_t* ids, uint32_t* scores,
                                            const slash_schedule* sched, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  slash_status rs = query_prelude(cix, q, kq, k, flags, ids, scores, st);
  if (rs != SLASH_OK) return rs;
  if (q.n_rows == 0) return SLASH_OK;
  slash_index* ix = const_cast<slash_index*>(cix);
  if (ix->shape.bucket) {
    // Topkapi buckets: one wave per query, hashing in the kernel
    QueryArgs ta{q, kq, k, 1, ids, scores, nullptr};
    HIP_TRY(launch_tk_query(ix->shape, ix->cv, tables(ix), ta, st));
    return SLASH_OK;
  }
  slash_schedule sc;
  if ((rs = batched_schedule(ix, q, sched, st, &sc)) != SLASH_OK) return rs;
  QueryArgs a{q, kq, k, 1, ids, scores, nullptr};
  a.exact = (flags & SLASH_FLAG_EXACT) ? 1u : 0u;
  return run_batched(ix, a, sc, st);
}

// ------------------------------------------------ allocation-free batched

// Scratch of slash_query_batched_static: a work counter (word 0, padded to
// 256 bytes) and the batch's bucket ids [n][L].  One copy per device, held
// until the process ends.  Host code never uses this name as an address
// (on the host it stands for the symbol, not device memory): the device
// address comes from hipGetSymbolAddress, once per device.
static constexpr size_t kStaticScratchWords = size_t(4) << 20;  // 16 MiB
static constexpr uint32_t kStaticTicketWords = 64;
static __device__ __align__(256) uint32_t scratch[kStaticScratchWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
uint32_t* g_static_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current device's scratch array (set up on the first
// call on that device, with that device current).
static slash_status static_scratch(uint32_t** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SLASH_E_UNSUPPORTED, "device %d beyond the static scratch table", dev);
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(SLASH_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_static_ptr[dev] = (uint32_t*)p;
  }
  *out = g_static_ptr[dev];
  return SLASH_OK;
}

extern "C" slash_status slash_query_batched_static(const slash_index* cix, slash_csr q, const uint32_t* kq, uint32_t k,
                                                   uint32_t flags, uint32_t* ids, uint32_t* scores,
                                                   const slash_schedule* sched, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  slash_status rs = query_prelude(cix, q, kq, k, flags, ids, scores, st);
  if (rs != SLASH_OK) return rs;
  if (q.n_rows == 0) return SLASH_OK;
  QueryArgs a{q, kq, k, 1, ids, scores, nullptr};
  a.exact = (flags & SLASH_FLAG_EXACT) ? 1u : 0u;
  const Shape& s = cix->shape;
  if (s.bucket) {
    // Topkapi buckets hash inside their query kernel: no scratch
    HIP_TRY(launch_tk_query(s, cix->cv, tables(cix), a, st));
    return SLASH_OK;
  }
  const uint64_t need = kStaticTicketWords + q.n_rows * (uint64_t)s.L;
  if (need > kStaticScratchWords)
    return fail(SLASH_E_INVAL, "batch of %llu queries needs %llu scratch words; the static scratch holds %llu "
                               "(at most %llu queries of %u tables)",
                (unsigned long long)q.n_rows, (unsigned long long)need, (unsigned long long)kStaticScratchWords,
                (unsigned long long)((kStaticScratchWords - kStaticTicketWords) / s.L), s.L);
  slash_schedule sc;
  if ((rs = batched_schedule(cix, q, sched, st, &sc)) != SLASH_OK) return rs;
  const uint32_t waves = sc.waves_per_query;
  if (!query_supported(s, waves, a.exact != 0))
    return fail(SLASH_E_UNSUPPORTED, "schedule with %u waves/query not supported", waves);
  uint32_t* sp = nullptr;
  if ((rs = static_scratch(&sp)) != SLASH_OK) return rs;
  uint32_t* ticket = sp;
  a.qbk = sp + kStaticTicketWords;
  HIP_TRY(launch_hash_rowmajor(s, cix->cv, q, sp + kStaticTicketWords, st));
  if (sc.queries_per_ticket == 0) {
    HIP_TRY(launch_query_waves(s, cix->cv, tables(cix), a, waves, st));
    return SLASH_OK;
  }
  int occ = 0;
  HIP_TRY(query_occupancy(s, waves, &occ, a.exact != 0));
  if (occ < 1) occ = 1;
  const uint32_t per_ticket = sc.queries_per_ticket;
  const uint32_t per_cu = sc.groups_per_cu ? std::min<uint32_t>(sc.groups_per_cu, (uint32_t)occ) : (uint32_t)occ;
  uint64_t grid = (uint64_t)per_cu * (uint32_t)cix->n_cu;
  grid = std::min<uint64_t>(grid, (q.n_rows + per_ticket - 1) / per_ticket);
  // the work counter starts at zero (a fill kernel, not a memset)
  HIP_TRY(launch_fill_u32(ticket, 0u, 1, st));
  HIP_TRY(launch_query_persistent(s, cix->cv, tables(cix), a, waves, per_ticket, (uint32_t)std::max<uint64_t>(1, grid),
                                  ticket, st));
  return SLASH_OK;
}

extern "C" slash_status slash_autotune(slash_index* ix, slash_csr sample, uint32_t k, slash_schedule* best_out,
                                       void* stream) {
  hipStream_t st = (hipStream_t)stream;
  slash_status rs = query_prelude(ix, sample, nullptr, k, 0, (uint32_t*)1, (uint32_t*)1, st);
  if (rs != SLASH_OK) return rs;
  if (sample.n_rows == 0) return fail(SLASH_E_INVAL, "empty tuning sample");
  if (ix->shape.bucket) {
    // one launch form only for Topkapi buckets: nothing to tune
    if (best_out) *best_out = default_schedule(ix);
    return SLASH_OK;
  }
  const uint64_t n = sample.n_rows;
  const uint32_t km = ix->p.k_max;
  DBuf ref_i, ref_s, got_i, got_s;
  SyncOnExit drain{st};
  if (!ref_i.get(n * km * 4) || !ref_s.get(n * km * 4) || !got_i.get(n * km * 4) || !got_s.get(n * km * 4))
    return fail(SLASH_E_NOMEM, "autotune buffers");
  QueryArgs ra{sample, nullptr, k, 1, ref_i.as<uint32_t>(), ref_s.as<uint32_t>(), nullptr};
  HIP_TRY(launch_query(ix->shape, ix->cv, tables(ix), ra, st));
  std::vector<uint32_t> h_ref(n * km * 2), h_got(n * km * 2);
  HIP_TRY(hipMemcpyAsync(h_ref.data(), ref_i.p, n * km * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(h_ref.data() + n * km, ref_s.p, n * km * 4, hipMemcpyDeviceToHost, st));
  int64_t ends[2];
  HIP_TRY(hipMemcpyAsync(&ends[0], sample.indptr, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&ends[1], sample.indptr + n, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  uint32_t cls = size_class((double)(ends[1] - ends[0]) / (double)n);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best_ms = 1e30f;
  slash_schedule best = default_schedule(ix);
  const uint32_t wv[] = {1, 2, 4, 8, 16};
  const uint32_t tk[] = {0, 1, 2, 8};  // 0: one work-group per query, no work counter
  const uint32_t gpc[] = {0, 2};
  for (uint32_t w : wv) {
    if (!query_supported(ix->shape, w)) continue;
    for (uint32_t t : tk)
      for (uint32_t g : gpc) {
        if (t == 0 && g != 0) continue;  // the plain form has no resident-group count
        slash_schedule sc{w, t, g, 0};
        QueryArgs ga{sample, nullptr, k, 1, got_i.as<uint32_t>(), got_s.as<uint32_t>(), nullptr};
        rs = run_batched(ix, ga, sc, st);  // warm-up + correctness
        if (rs != SLASH_OK) continue;
        HIP_TRY(hipMemcpyAsync(h_got.data(), got_i.p, n * km * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(h_got.data() + n * km, got_s.p, n * km * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (h_got != h_ref) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          return fail(SLASH_E_DEVICE, "schedule (%u waves, %u per ticket, %u per CU) disagrees with the plain path", w, t, g);
        }
        HIP_TRY(hipEventRecord(e0, st));
        for (int rep = 0; rep < 3; ++rep) {
          rs = run_batched(ix, ga, sc, st);
          if (rs != SLASH_OK) return rs;
        }
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
          best_ms = ms;
          best = sc;
        }
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ix->tuned[cls] = best;
  ix->has_tuned[cls] = true;
  if (best_out) *best_out = best;
  return SLASH_OK;
}

// ----------------------------------------------------------- small calls

extern "C" slash_status slash_hash(const slash_index* ix, slash_csr rows, uint32_t flags, uint32_t* buckets,
                                   void* stream) {
  if (!ix) return fail(SLASH_E_INVAL, "index is NULL");
  hipStream_t st = (hipStream_t)stream;
  if (rows.n_rows == 0) return SLASH_OK;
  if (!buckets) return fail(SLASH_E_INVAL, "output is NULL");
  slash_status rs;
  if (!(flags & SLASH_FLAG_TRUSTED) && (rs = validate_rows(const_cast<slash_index*>(ix), rows, nullptr, st)) != SLASH_OK)
    return rs;
  HIP_TRY(launch_hash_rowmajor(ix->shape, ix->cv, rows, buckets, st));
  return SLASH_OK;
}

extern "C" slash_status slash_export_tables(const slash_index* ix, uint32_t* ids, uint32_t* seen, void* stream) {
  if (!ix) return fail(SLASH_E_INVAL, "index is NULL");
  hipStream_t st = (hipStream_t)stream;
  const Shape& s = ix->shape;
  if (ids) HIP_TRY(hipMemcpyAsync(ids, ix->ids, (size_t)s.L * s.nb * bucket_words(s) * 4, hipMemcpyDeviceToDevice, st));
  if (seen) HIP_TRY(hipMemcpyAsync(seen, ix->seen, (size_t)s.L * s.nb * 4, hipMemcpyDeviceToDevice, st));
  return SLASH_OK;
}

// An index with derived constants and allocated (unfilled) tables, for the
// import and load paths.
static slash_status new_index(const slash_params* params, uint64_t n_items, hipStream_t st, slash_index** out) {
  slash_status rs = check_params(params);
  if (rs != SLASH_OK) return rs;
  if (n_items > 0xFFFFFFFEull) return fail(SLASH_E_CAPACITY, "more than 2^32-2 ids");
  slash_index* ix = new (std::nothrow) slash_index();
  if (!ix) return fail(SLASH_E_NOMEM, "host allocation failed");
  ix->p = *params;
  ix->shape = make_shape(*params);
  ix->hc = derive_consts(*params);
  if (hipGetDevice(&ix->device) != hipSuccess ||
      hipDeviceGetAttribute(&ix->n_cu, hipDeviceAttributeMultiprocessorCount, ix->device) != hipSuccess) {
    destroy_index(ix);
    return fail(SLASH_E_DEVICE, "device query failed");
  }
  if ((rs = upload_consts(ix, st)) != SLASH_OK || (rs = alloc_tables(ix)) != SLASH_OK) {
    destroy_index(ix);
    return rs;
  }
  ix->n_items = n_items;
  *out = ix;
  return SLASH_OK;
}

// After the tables of an imported or loaded index are in place: check
// reservoir tables (a bucket's first min(R, seen) slots hold assigned ids,
// the rest are EMPTY, which queries rely on: they read every non-EMPTY slot)
// and reserve the insert scratch.  Frees the index on error.
static slash_status finish_index(slash_index* ix, hipStream_t st) {
  const Shape& s = ix->shape;
  uint32_t f = 0;
  hipError_t e = hipSuccess;
  if (!s.bucket) e = launch_fill_u32(ix->flag, 0u, 1, st);
  if (e == hipSuccess && !s.bucket)
    e = launch_check_tables(ix->ids, ix->seen, (uint64_t)s.L * s.nb, s.R, ix->n_items, ix->flag, st);
  if (e == hipSuccess && !s.bucket) e = hipMemcpyAsync(&f, ix->flag, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  slash_status rs = SLASH_OK;
  if (e != hipSuccess)
    rs = fail(SLASH_E_DEVICE, "table copy: %s", hipGetErrorString(e));
  else if (f & 8u)
    rs = fail(SLASH_E_INVAL, "tables: a bucket holds an EMPTY or unassigned id in its first min(R, seen) slots, or "
                             "an id past them");
  else
    rs = reserve_small_inserts(ix);
  if (rs != SLASH_OK) destroy_index(ix);
  return rs;
}

extern "C" slash_status slash_import_tables(const slash_params* params, const uint32_t* ids, const uint32_t* seen,
                                           uint64_t n_items, void* stream, slash_index** out) {
  if (!out) return fail(SLASH_E_INVAL, "out is NULL");
  if (!ids || !seen) return fail(SLASH_E_INVAL, "table buffers are NULL");
  hipStream_t st = (hipStream_t)stream;
  slash_index* ix = nullptr;
  slash_status rs = new_index(params, n_items, st, &ix);
  if (rs != SLASH_OK) return rs;
  const Shape& s = ix->shape;
  hipError_t e = hipMemcpyAsync(ix->ids, ids, (size_t)s.L * s.nb * bucket_words(s) * 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(ix->seen, seen, (size_t)s.L * s.nb * 4, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    destroy_index(ix);
    return fail(SLASH_E_DEVICE, "table copy: %s", hipGetErrorString(e));
  }
  if ((rs = finish_index(ix, st)) != SLASH_OK) return rs;
  *out = ix;
  return SLASH_OK;
}

// ------------------------------------------------------------ save / load

// File layout (little endian): a 128-byte header, then the table array
// ([L][2^B][R] ids, or [L][2^B][cm_rows][2^lw][2] Topkapi cells, uint32),
// then seen [L][2^B] (uint32).  Header: magic "SLASHIDX", format version,
// header bytes, the slash_params fields one by one (uint32 each, then the
// uint64 seed), n_items, the byte sizes of the two arrays, and a 64-bit
// FNV-1a checksum of both arrays.
namespace {
constexpr char kMagic[8] = {'S', 'L', 'A', 'S', 'H', 'I', 'D', 'X'};
constexpr uint32_t kFormat = 1;
constexpr size_t kHeaderBytes = 128;
constexpr size_t kChunk = size_t(64) << 20;  // staging chunk (pinned host memory)

struct FileHeader {
  char magic[8];
  uint32_t format, header_bytes;
  uint32_t dim, K, L, log2_buckets, R, cm_rows, log2_cm_width, k_max, hash_mode, bucket;
  uint64_t seed, n_items, table_bytes, seen_bytes, checksum;
};
static_assert(sizeof(FileHeader) <= kHeaderBytes, "header fits its 128 bytes");

uint64_t fnv1a(uint64_t h, const uint8_t* p, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001B3ull;
  }
  return h;
}
constexpr uint64_t kFnvBasis = 0xCBF29CE484222325ull;

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) fclose(f);
  }
};
struct Pinned {
  void* p = nullptr;
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};
}  // namespace

extern "C" slash_status slash_save(const slash_index* ix, const char* path, void* stream) {
  if (!ix || !path) return fail(SLASH_E_INVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const Shape& s = ix->shape;
  FileHeader h;
  memset(&h, 0, sizeof h);
  memcpy(h.magic, kMagic, 8);
  h.format = kFormat;
  h.header_bytes = (uint32_t)kHeaderBytes;
  const slash_params& p = ix->p;
  h.dim = p.dim, h.K = p.K, h.L = p.L, h.log2_buckets = p.log2_buckets, h.R = p.R, h.cm_rows = p.cm_rows;
  h.log2_cm_width = p.log2_cm_width, h.k_max = p.k_max, h.hash_mode = p.hash_mode, h.bucket = p.bucket;
  h.seed = p.seed;
  h.n_items = ix->n_items;
  h.table_bytes = (uint64_t)s.L * s.nb * bucket_words(s) * 4;
  h.seen_bytes = (uint64_t)s.L * s.nb * 4;
  File out;
  out.f = fopen(path, "wb");
  if (!out.f) return fail(SLASH_E_INVAL, "cannot open %s for writing", path);
  uint8_t head[kHeaderBytes] = {};
  if (fwrite(head, 1, kHeaderBytes, out.f) != kHeaderBytes) return fail(SLASH_E_INVAL, "write to %s failed", path);
  Pinned buf;
  HIP_TRY(hipHostMalloc(&buf.p, kChunk));
  uint64_t sum = kFnvBasis;
  const struct {
    const uint32_t* src;
    uint64_t bytes;
  } parts[2] = {{ix->ids, h.table_bytes}, {ix->seen, h.seen_bytes}};
  for (const auto& part : parts)
    for (uint64_t off = 0; off < part.bytes; off += kChunk) {
      const size_t n = (size_t)std::min<uint64_t>(kChunk, part.bytes - off);
      HIP_TRY(hipMemcpyAsync(buf.p, (const uint8_t*)part.src + off, n, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      sum = fnv1a(sum, (const uint8_t*)buf.p, n);
      if (fwrite(buf.p, 1, n, out.f) != n) return fail(SLASH_E_INVAL, "write to %s failed", path);
    }
  h.checksum = sum;
  memcpy(head, &h, sizeof h);
  if (fseek(out.f, 0, SEEK_SET) != 0 || fwrite(head, 1, kHeaderBytes, out.f) != kHeaderBytes || fflush(out.f) != 0)
    return fail(SLASH_E_INVAL, "write to %s failed", path);
  return SLASH_OK;
}

extern "C" slash_status slash_load(const char* path, void* stream, slash_index** out) {
  if (!path || !out) return fail(SLASH_E_INVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  File in;
  in.f = fopen(path, "rb");
  if (!in.f) return fail(SLASH_E_INVAL, "cannot open %s", path);
  uint8_t head[kHeaderBytes];
  FileHeader h;
  if (fread(head, 1, kHeaderBytes, in.f) != kHeaderBytes) return fail(SLASH_E_INVAL, "%s: short header", path);
  memcpy(&h, head, sizeof h);
  if (memcmp(h.magic, kMagic, 8) != 0) return fail(SLASH_E_INVAL, "%s: not a saved index", path);
  if (h.format != kFormat || h.header_bytes != kHeaderBytes)
    return fail(SLASH_E_INVAL, "%s: format %u (header %u bytes) is not %u", path, h.format, h.header_bytes, kFormat);
  slash_params p{};
  p.dim = h.dim, p.K = h.K, p.L = h.L, p.log2_buckets = h.log2_buckets, p.R = h.R, p.cm_rows = h.cm_rows;
  p.log2_cm_width = h.log2_cm_width, p.k_max = h.k_max, p.hash_mode = h.hash_mode, p.bucket = h.bucket;
  p.seed = h.seed;
  slash_status rs = check_params(&p);
  if (rs != SLASH_OK) return fail(SLASH_E_INVAL, "%s: saved parameters: %s", path, slash_last_error());
  const Shape s = make_shape(p);
  if (h.table_bytes != (uint64_t)s.L * s.nb * bucket_words(s) * 4 || h.seen_bytes != (uint64_t)s.L * s.nb * 4)
    return fail(SLASH_E_INVAL, "%s: array sizes do not match the saved parameters", path);
  if (fseek(in.f, 0, SEEK_END) != 0) return fail(SLASH_E_INVAL, "%s: cannot seek", path);
  const long long size = ftell(in.f);
  if (size < 0 || (uint64_t)size != kHeaderBytes + h.table_bytes + h.seen_bytes)
    return fail(SLASH_E_INVAL, "%s: %lld bytes, expected %llu", path, size,
                (unsigned long long)(kHeaderBytes + h.table_bytes + h.seen_bytes));
  if (fseek(in.f, (long)kHeaderBytes, SEEK_SET) != 0) return fail(SLASH_E_INVAL, "%s: cannot seek", path);
  slash_index* ix = nullptr;
  if ((rs = new_index(&p, h.n_items, st, &ix)) != SLASH_OK) return rs;
  auto bail = [&](slash_status r) {
    (void)hipStreamSynchronize(st);
    destroy_index(ix);
    return r;
  };
  Pinned buf;
  if (hipHostMalloc(&buf.p, kChunk) != hipSuccess) return bail(fail(SLASH_E_NOMEM, "pinned staging buffer"));
  uint64_t sum = kFnvBasis;
  const struct {
    uint32_t* dst;
    uint64_t bytes;
  } parts[2] = {{ix->ids, h.table_bytes}, {ix->seen, h.seen_bytes}};
  for (const auto& part : parts)
    for (uint64_t off = 0; off < part.bytes; off += kChunk) {
      const size_t n = (size_t)std::min<uint64_t>(kChunk, part.bytes - off);
      // the previous chunk's copy reads the staging buffer until it is done
      if (hipStreamSynchronize(st) != hipSuccess) return bail(fail(SLASH_E_DEVICE, "load: stream"));
      if (fread(buf.p, 1, n, in.f) != n) return bail(fail(SLASH_E_INVAL, "%s: short read", path));
      sum = fnv1a(sum, (const uint8_t*)buf.p, n);
      if (hipMemcpyAsync((uint8_t*)part.dst + off, buf.p, n, hipMemcpyHostToDevice, st) != hipSuccess)
        return bail(fail(SLASH_E_DEVICE, "load: copy"));
    }
  if (hipStreamSynchronize(st) != hipSuccess) return bail(fail(SLASH_E_DEVICE, "load: stream"));
  if (sum != h.checksum) return bail(fail(SLASH_E_INVAL, "%s: checksum mismatch", path));
  if ((rs = finish_index(ix, st)) != SLASH_OK) return rs;
  *out = ix;
  return SLASH_OK;
}

extern "C" slash_status slash_build_profile(const slash_index* ix, slash_phase_stat* out, uint32_t max, uint32_t* n) {
  if (!ix || !n || (!out && max)) return fail(SLASH_E_INVAL, "NULL argument");
  uint32_t c = 0;
  for (int p = 0; p < PH_COUNT && c < max; ++p) {
    memset(&out[c], 0, sizeof out[c]);
    snprintf(out[c].name, sizeof out[c].name, "%s", kPhaseNames[p]);
    out[c].launches = ix->phase_n[p];
    out[c].total_ms = ix->phase_ms[p];
    out[c].alg_bytes = ix->phase_bytes[p];
    ++c;
  }
  *n = c;
  return SLASH_OK;
}

extern "C" slash_status slash_index_info_get(const slash_index* ix, slash_index_info* info) {
  if (!ix || !info) return fail(SLASH_E_INVAL, "NULL argument");
  memset(info, 0, sizeof *info);
  info->params = ix->p;
  info->n_items = ix->n_items;
  info->n_buckets = ix->shape.nb;
  info->table_bytes = (uint64_t)ix->shape.L * ix->shape.nb * (bucket_words(ix->shape) + 1) * 4;
  return SLASH_OK;
}
