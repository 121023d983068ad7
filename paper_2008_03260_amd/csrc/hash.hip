// Hash kernels (Section 2.2 DOPH, Section 2.3 table addresses), input
// validation and small utility kernels.
#include <algorithm>

#include "doph.h"

namespace slash {

namespace {

constexpr int kMaxHashWaves = 4;

__host__ __device__ inline bool const_staged(const Shape& s) { return const_words(s) <= kConstCapWords; }

// LDS words of one group's DOPH scratch: the register form needs only the
// minima.
__host__ __device__ inline uint32_t group_lds_words(const Shape& s, int P) {
  return P ? s.M : doph_lds_words(s.M);
}

// Hash one row with a group of G lanes and call emit(t, bucket) for its L
// tables (P > 0: register densification with P bins per lane, else the
// generic LDS walk).  With PRE the row's first 4·G indices are already in x0
// (register form only).  Every lane of the wave calls.
template <int G, int P, bool CL, bool PRE = false, class Emit>
__device__ __forceinline__ void hash_row(const Shape& s, const ConstView& c, const int32_t* idx, uint32_t nnz,
                                         bool live, uint32_t* my, Emit emit, const uint32_t* x0 = nullptr) {
  const uint32_t gl = threadIdx.x & (G - 1);
  if constexpr (P > 0) {
    uint32_t h[P];
    doph_regs<G, P, CL, PRE>(s, c, idx, nnz, my, h, x0);
    if (live) table_buckets_regs<P, CL>(s, c, h, gl, emit);
  } else {
    const uint32_t* h = doph_group<G, CL>(s, c, idx, nnz, my);
    if (live)
      for (uint32_t t = gl; t < s.L; t += G) emit(t, table_bucket<CL>(s, c, h, t));
  }
  wave_sync();
}

// Each block takes chunks of `rpc` consecutive rows; a group of G lanes
// hashes one row at a time (64 / G rows per wave at once) and stages its L
// bucket ids in LDS; the block then writes every table's rpc ids as one
// contiguous run (keys are table-major).
// Waves per SIMD the register budget is held to: the 8-bins-per-lane form
// (M = 128) is cut from 108 to 96 VGPRs, one more wave per SIMD (the block's
// LDS allows five); the others keep what they need.
template <int P>
constexpr int hash_min_waves() { return P == 8 ? 5 : 1; }

template <int G, int P, bool CL>
__global__ void __launch_bounds__(kMaxHashWaves * SL_WAVE, hash_min_waves<P>())
    k_hash_rows(Shape s, ConstView c, slash_csr rows, uint32_t* __restrict__ keys, uint64_t key_stride,
                int combine, uint32_t rpc) {
  extern __shared__ uint32_t lds[];
  constexpr uint32_t GPW = SL_WAVE / G;  // groups per wave
  const uint32_t ng = (blockDim.x / SL_WAVE) * GPW;
  const uint32_t grp = threadIdx.x / G;
  const uint32_t per_grp = group_lds_words(s, P);
  const uint32_t cw = CL ? (const_words(s) + 3) & ~3u : 0u;  // 16-byte aligned scratch after it
  const ConstView cl = CL ? stage_consts(s, c, lds, blockDim.x) : c;
  uint32_t* my = lds + cw + grp * per_grp;
  uint32_t* stage = lds + cw + ng * per_grp;  // [L][rpc + 1]: the pad spreads one row's tables over banks
  const uint32_t sst = rpc + 1;
  __syncthreads();
  const uint64_t n = rows.n_rows;
  const uint64_t n_chunks = (n + rpc - 1) / rpc;
  for (uint64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
    const uint64_t r0 = ch * rpc;
    // Every group runs the same number of rounds (wave-wide syncs inside).
    // Software pipeline over the group's rows of this chunk: while row j is
    // hashed, the first indices of row j+1 and the bounds of row j+2 are in
    // flight.
    auto bounds = [&](uint32_t rl, int64_t& b, int64_t& e) {
      if (rl < rpc && r0 + rl < n) {
        b = rows.indptr[r0 + rl];
        e = rows.indptr[r0 + rl + 1];
      } else {
        b = e = 0;
      }
    };
    const uint32_t gl = threadIdx.x & (G - 1);
    int64_t b0, e0, b1, e1;
    bounds(grp, b0, e0);
    bounds(grp + ng, b1, e1);
    uint32_t x[4];
    if constexpr (P > 0) load_batch<G>(rows.indices + b0, 0, (uint32_t)(e0 - b0), gl, x);
    for (uint32_t rb = 0; rb < rpc; rb += ng) {
      const uint32_t rl = rb + grp;
      const bool live = rl < rpc && r0 + rl < n;
      const int64_t beg = b0;
      const uint32_t nnz = (uint32_t)(e0 - b0);
      uint32_t xc[4] = {x[0], x[1], x[2], x[3]};
      if constexpr (P > 0) load_batch<G>(rows.indices + b1, 0, (uint32_t)(e1 - b1), gl, x);
      b0 = b1;
      e0 = e1;
      bounds(rl + 2 * ng, b1, e1);
      auto emit = [&](uint32_t t, uint32_t b) { stage[t * sst + rl] = combine ? t * s.nb + b : b; };
      if constexpr (P > 0)
        hash_row<G, P, CL, true>(s, cl, rows.indices + beg, live ? nnz : 0u, live, my, emit, xc);
      else
        hash_row<G, P, CL>(s, cl, rows.indices + beg, live ? nnz : 0u, live, my, emit);
    }
    __syncthreads();
    const uint32_t tot = s.L * rpc;
    for (uint32_t e = threadIdx.x; e < tot; e += blockDim.x) {
      uint32_t t = e / rpc, rl = e - t * rpc;
      if (r0 + rl < n) keys[t * key_stride + r0 + rl] = stage[t * sst + rl];
    }
    __syncthreads();
  }
}

template <int G, int P, bool CL>
__global__ void __launch_bounds__(kMaxHashWaves * SL_WAVE)
    k_hash_rowmajor(Shape s, ConstView c, slash_csr rows, uint32_t* __restrict__ out) {
  extern __shared__ uint32_t lds[];
  constexpr uint32_t GPW = SL_WAVE / G;
  const uint32_t ng = (blockDim.x / SL_WAVE) * GPW;
  const uint32_t grp = threadIdx.x / G;
  const uint32_t cw = CL ? (const_words(s) + 3) & ~3u : 0u;  // 16-byte aligned scratch after it
  const ConstView cl = CL ? stage_consts(s, c, lds, blockDim.x) : c;
  uint32_t* my = lds + cw + grp * group_lds_words(s, P);
  __syncthreads();
  const uint64_t n = rows.n_rows;
  const uint64_t stride = (uint64_t)gridDim.x * ng;
  const uint64_t rounds = (n + stride - 1) / stride;
  for (uint64_t k = 0; k < rounds; ++k) {
    const uint64_t r = k * stride + (uint64_t)blockIdx.x * ng + grp;
    const bool live = r < n;
    int64_t beg = 0, end = 0;
    if (live) {
      beg = rows.indptr[r];
      end = rows.indptr[r + 1];
    }
    hash_row<G, P, CL>(s, cl, rows.indices + beg, (uint32_t)(end - beg), live, my,
                       [&](uint32_t t, uint32_t b) { out[r * s.L + t] = b; });
  }
}

constexpr size_t kLdsCap = 160 * 1024;

// LDS words ahead of the per-wave DOPH scratch.
uint32_t const_lds_words(const Shape& s) { return const_staged(s) ? (const_words(s) + 3) & ~3u : 0u; }

// Rows staged per chunk: at most 128 (64 and 256 measured slower on the
// 200M-row shard), and the stage stays within 32 KB.
uint32_t hash_rpc(const Shape& s) {
  uint32_t r = 8192u / s.L;
  if (r < 1) r = 1;
  if (r > 128) r = 128;
  return r;
}

// Lanes per row.
uint32_t row_group(const Shape& s) { return hash_group(s.M); }

// Bins per lane of the register DOPH form for this shape, or 0 (generic).
int hash_p(const Shape& s) { return (int)doph_regs_p(s, row_group(s)); }

// Host check that the chosen kernel fits the shape: the register form needs
// M = G * P bins with K dividing P (its lanes own whole tables); the generic
// form needs a group size it is instantiated for.
bool hash_shape_ok(const Shape& s) {
  const uint32_t G = row_group(s);
  const int P = hash_p(s);
  if (P) return s.mode == 0 && s.M == G * (uint32_t)P && (uint32_t)P % s.K == 0;
  return G == 16 || G == 32 || G == 64;
}

// Waves per block such that the block's LDS fits (64 / G rows per wave).
uint32_t hash_waves(const Shape& s, size_t fixed) {
  const size_t per_wave = (size_t)(SL_WAVE / row_group(s)) * group_lds_words(s, hash_p(s)) * 4;
  for (uint32_t w = kMaxHashWaves; w > 1; w >>= 1)
    if (w * per_wave + fixed <= kLdsCap) return w;
  return 1;
}

// LDS bytes of a hash block with nw waves and `fixed` bytes ahead of the
// per-group scratch.
size_t hash_lds(const Shape& s, uint32_t nw, size_t fixed) {
  return (size_t)nw * (SL_WAVE / row_group(s)) * group_lds_words(s, hash_p(s)) * 4 + fixed;
}

template <int G, bool CL>
const void* rows_fn_p(int P) {
  switch (P) {
    case 4: return (const void*)k_hash_rows<G, 4, CL>;
    case 8: return (const void*)k_hash_rows<G, 8, CL>;
    case 16: return (const void*)k_hash_rows<G, 16, CL>;
    default: return (const void*)k_hash_rows<G, 0, CL>;
  }
}

template <int G, bool CL>
const void* rowmajor_fn_p(int P) {
  switch (P) {
    case 4: return (const void*)k_hash_rowmajor<G, 4, CL>;
    case 8: return (const void*)k_hash_rowmajor<G, 8, CL>;
    case 16: return (const void*)k_hash_rowmajor<G, 16, CL>;
    default: return (const void*)k_hash_rowmajor<G, 0, CL>;
  }
}

const void* hash_rows_fn(const Shape& s) {
  const bool cl = const_staged(s);
  const int P = hash_p(s);
  switch (row_group(s)) {
    case 16: return cl ? rows_fn_p<16, true>(P) : rows_fn_p<16, false>(P);
    case 32: return cl ? rows_fn_p<32, true>(P) : rows_fn_p<32, false>(P);
    default: return cl ? rows_fn_p<64, true>(P) : rows_fn_p<64, false>(P);
  }
}

const void* hash_rowmajor_fn(const Shape& s) {
  const bool cl = const_staged(s);
  const int P = hash_p(s);
  switch (row_group(s)) {
    case 16: return cl ? rowmajor_fn_p<16, true>(P) : rowmajor_fn_p<16, false>(P);
    case 32: return cl ? rowmajor_fn_p<32, true>(P) : rowmajor_fn_p<32, false>(P);
    default: return cl ? rowmajor_fn_p<64, true>(P) : rowmajor_fn_p<64, false>(P);
  }
}

hipError_t allow_lds(const void* f, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// flag bits: 1 = empty row or decreasing indptr, 2 = index outside [0, dim),
// 4 = per-query k above k_max.
__global__ void k_validate_rows(slash_csr rows, const uint32_t* kq, uint32_t k_max, uint32_t* flag) {
  uint32_t f = 0;
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < rows.n_rows;
       r += (uint64_t)gridDim.x * blockDim.x) {
    if (rows.indptr[r + 1] <= rows.indptr[r]) f |= 1u;
    if (kq && kq[r] > k_max) f |= 4u;
  }
  if (f) atomicOr(flag, f);
}

__global__ void k_validate_idx(const int32_t* idx, uint64_t n, uint32_t dim, uint32_t* flag) {
  uint32_t f = 0;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < n; e += (uint64_t)gridDim.x * blockDim.x) {
    int32_t v = idx[e];
    if (v < 0 || (uint32_t)v >= dim) f |= 2u;
  }
  if (__ballot(f != 0) && f) atomicOr(flag, f);
}

__global__ void k_fill(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_iota(uint32_t* p, uint32_t first, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = first + (uint32_t)i;
}

// Start and end of every key's run in the sorted keys.  A thread takes 8
// consecutive keys (all loads issued before any compare) plus the neighbours
// on either side.
__global__ void k_segment_bounds(const uint32_t* __restrict__ sk, uint64_t n, uint32_t* start, uint32_t* end) {
  constexpr uint32_t kPer = 8;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * kPer;
  for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kPer; i0 < n; i0 += stride) {
    uint32_t k[kPer];
    if (i0 + kPer <= n) {
#pragma unroll
      for (uint32_t j = 0; j < kPer; ++j) k[j] = sk[i0 + j];
    } else {
#pragma unroll
      for (uint32_t j = 0; j < kPer; ++j) k[j] = i0 + j < n ? sk[i0 + j] : 0u;
    }
    const uint32_t prev = i0 > 0 ? sk[i0 - 1] : ~k[0];
    const uint32_t next = i0 + kPer < n ? sk[i0 + kPer] : 0u;
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      const uint64_t i = i0 + j;
      if (i >= n) break;
      const uint32_t before = j ? k[j - 1] : prev;
      if (i == 0 || before != k[j]) start[k[j]] = (uint32_t)i;
      const bool last = i + 1 == n;
      const uint32_t after = j + 1 < kPer ? k[j + 1] : next;
      if (last || after != k[j]) end[k[j]] = (uint32_t)(i + 1);
    }
  }
}

// Sort values of an insert batch: item i = t * n_rows + r belongs to row r.
__global__ void k_item_ids(uint32_t* v, uint32_t first, uint64_t n_rows, uint64_t items) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < items; i += (uint64_t)gridDim.x * blockDim.x)
    v[i] = first + (uint32_t)(i % n_rows);
}

// Imported reservoir tables: the first min(R, seen) slots of a bucket hold
// ids below n_items, the rest are EMPTY (what a build or insert leaves, and
// what a query relies on: it reads every non-EMPTY slot).  ORs 8 into *flag
// on a violation.
__global__ void k_check_tables(const uint32_t* __restrict__ ids, const uint32_t* __restrict__ seen, uint64_t n_buckets,
                               uint32_t R, uint64_t n_items, uint32_t* flag) {
  const uint64_t total = n_buckets * R;
  bool bad = false;
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total; x += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t b = x / R;
    const uint32_t j = (uint32_t)(x - b * R);
    const uint32_t fill = min(R, seen[b]);
    const uint32_t v = ids[x];
    bad |= j < fill ? (v == SL_EMPTY || (uint64_t)v >= n_items) : v != SL_EMPTY;
  }
  if (bad) atomicOr(flag, 8u);
}

uint32_t grid_for(uint64_t work, uint32_t block, uint32_t cap = 65536) {
  uint64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

}  // namespace

hipError_t launch_hash_rows(const Shape& s, const ConstView& c, slash_csr rows, uint32_t* keys, uint64_t key_stride,
                            int combine, hipStream_t st) {
  if (rows.n_rows == 0) return hipSuccess;
  if (!hash_shape_ok(s)) return hipErrorInvalidValue;
  // a small batch (an insert) takes shorter chunks so that it spreads over
  // about a thousand blocks instead of a few dozen
  uint32_t rpc = hash_rpc(s);
  const uint64_t want = (rows.n_rows + 1023) / 1024;
  if (want < rpc) rpc = (uint32_t)std::max<uint64_t>(std::min<uint64_t>(16, rpc), want);
  const size_t stage = (size_t)s.L * (rpc + 1) * 4 + (size_t)const_lds_words(s) * 4;
  const uint32_t nw = hash_waves(s, stage);
  const size_t lds = hash_lds(s, nw, stage);
  const void* fn = hash_rows_fn(s);
  hipError_t e = allow_lds(fn, lds);
  if (e != hipSuccess) return e;
  uint64_t chunks = (rows.n_rows + rpc - 1) / rpc;
  uint32_t grid = (uint32_t)(chunks < 16384 ? chunks : 16384);
  Shape sh = s;
  ConstView cv = c;
  void* args[] = {&sh, &cv, &rows, &keys, &key_stride, &combine, const_cast<uint32_t*>(&rpc)};
  e = hipLaunchKernel(fn, dim3(grid), dim3(nw * SL_WAVE), args, lds, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_hash_rowmajor(const Shape& s, const ConstView& c, slash_csr rows, uint32_t* out, hipStream_t st) {
  if (rows.n_rows == 0) return hipSuccess;
  if (!hash_shape_ok(s)) return hipErrorInvalidValue;
  const size_t fixed = (size_t)const_lds_words(s) * 4;
  const uint32_t nw = hash_waves(s, fixed);
  const size_t lds = hash_lds(s, nw, fixed);
  const void* fn = hash_rowmajor_fn(s);
  hipError_t e = allow_lds(fn, lds);
  if (e != hipSuccess) return e;
  uint32_t grid = grid_for(rows.n_rows, nw * (SL_WAVE / row_group(s)), 8192);
  Shape sh = s;
  ConstView cv = c;
  void* args[] = {&sh, &cv, &rows, &out};
  e = hipLaunchKernel(fn, dim3(grid), dim3(nw * SL_WAVE), args, lds, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

void* hash_rowmajor_kernel(const Shape& s, uint32_t* threads, size_t* lds) {
  if (!hash_shape_ok(s)) return nullptr;
  const size_t fixed = (size_t)const_lds_words(s) * 4;
  const uint32_t nw = hash_waves(s, fixed);
  *threads = nw * SL_WAVE;
  *lds = hash_lds(s, nw, fixed);
  const void* fn = hash_rowmajor_fn(s);
  if (allow_lds(fn, *lds) != hipSuccess) return nullptr;
  return const_cast<void*>(fn);
}

uint32_t hash_rowmajor_grid(const Shape& s, uint64_t n_rows) {
  const uint32_t nw = hash_waves(s, (size_t)const_lds_words(s) * 4);
  return grid_for(n_rows, nw * (SL_WAVE / row_group(s)), 8192);
}

hipError_t launch_validate(slash_csr rows, uint32_t dim, const uint32_t* kq, uint32_t k_max, uint32_t* flag,
                           hipStream_t st) {
  if (rows.n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate_rows, dim3(grid_for(rows.n_rows, 256, 4096)), dim3(256), 0, st, rows, kq, k_max,
                     flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // indices of all rows are the contiguous range [indptr[0], indptr[n]);
  // the range is read on the host by the caller and passed via rows.indices
  return hipSuccess;
}

hipError_t launch_validate_indices(const int32_t* idx, uint64_t n, uint32_t dim, uint32_t* flag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate_idx, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, idx, n, dim, flag);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_iota_u32(uint32_t* p, uint32_t first, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, p, first, n);
  return hipGetLastError();
}

hipError_t launch_item_ids(uint32_t* vals, uint32_t first_id, uint64_t n_rows, uint64_t items, hipStream_t st) {
  if (items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_ids, dim3(grid_for(items, 256, 8192)), dim3(256), 0, st, vals, first_id, n_rows, items);
  return hipGetLastError();
}

hipError_t launch_check_tables(const uint32_t* ids, const uint32_t* seen, uint64_t n_buckets, uint32_t R,
                               uint64_t n_items, uint32_t* flag, hipStream_t st) {
  if (n_buckets == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_tables, dim3(grid_for(n_buckets * R, 256, 65536)), dim3(256), 0, st, ids, seen,
                     n_buckets, R, n_items, flag);
  return hipGetLastError();
}

void* fill_kernel_ptr() { return (void*)k_fill; }

hipError_t launch_segment_bounds(const uint32_t* skeys, uint64_t n, uint32_t* start, uint32_t* end, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_segment_bounds, dim3(grid_for((n + 7) / 8, 256, 65536)), dim3(256), 0, st, skeys, n, start,
                     end);
  return hipGetLastError();
}

}  // namespace slash
