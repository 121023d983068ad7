// Topkapi buckets (Section 3.1; Appendix 2 "Top-K-API Details").
//
// Every bucket of every table is a sketch of W = cm_rows rows of
// C = 2^log2_cm_width cells, each cell a (heavy hitter, count) pair stored as
// uint2, empty = (EMPTY, 0).  Row r sends id x to cell g_r(x), the count-min
// row hash.  Insertion into a cell: take x with count 1 when the count is 0,
// count up on a match, count down otherwise.
//
// The ids a bucket receives are distinct and arrive in ascending order (row
// order), so the state a cell reaches has a closed form.  Starting from
// (h, c) and given m new ids, all larger than any earlier id: the first c of
// them only count down; after that the cell alternates (x, 1), (x, 0), so it
// ends on the largest new id with count 1 when m - c is odd, and on the
// second largest with count 0 when m - c is even.  Only the number of new ids
// per cell and their two largest values are needed, and both are
// order-independent: they are gathered with LDS atomics (add; max, then max
// of the displaced value), so any number of waves can share a bucket.
//
// A query folds its L bucket sketches cell by cell in table order with the
// merge rule (equal heavy hitters add; otherwise the larger count wins and
// keeps the difference; equal counts give the smaller id and count 0), then
// reports heavy hitters of count >= 1 by (count desc, id asc), an id held by
// several rows scoring its largest count.
#include "doph.h"
#include "slash_internal.h"

namespace slash {

namespace {

constexpr uint32_t kTkWaves = 4;       // waves per block (one bucket / run / query each)

__device__ __forceinline__ uint32_t tk_cells(const Shape& s) { return s.d << s.lw; }

// Final cell state from the stored one and the new ids' count and two
// largest values (see the header comment).
__device__ __forceinline__ uint2 tk_final(uint2 old, uint32_t m, uint32_t top1, uint32_t top2) {
  if (m <= old.y) return make_uint2(old.x, old.y - m);
  return ((m - old.y) & 1u) ? make_uint2(top1, 1u) : make_uint2(top2, 0u);
}

// Per-cell accumulators in LDS: count, largest, second largest.
struct TkAcc {
  uint32_t* cnt;
  uint32_t* top1;
  uint32_t* top2;
};

__device__ __forceinline__ TkAcc tk_acc(uint32_t* base, uint32_t ncp) { return TkAcc{base, base + ncp, base + 2 * ncp}; }

__device__ __forceinline__ void tk_clear(const TkAcc& a, uint32_t nc, uint32_t tid, uint32_t nt) {
  for (uint32_t i = tid; i < nc; i += nt) {
    a.cnt[i] = 0;
    a.top1[i] = 0;
    a.top2[i] = 0;
  }
}

// Add ids[i] for i in [i0, n) step `stride` to the accumulators.
__device__ __forceinline__ void tk_add(const Shape& s, const ConstView& c, const TkAcc& a,
                                       const uint32_t* __restrict__ ids, uint64_t i0, uint64_t n, uint32_t stride) {
  for (uint64_t i = i0; i < n; i += stride) {
    const uint32_t x = ids[i];
    for (uint32_t r = 0; r < s.d; ++r) {
      const uint32_t ci = (r << s.lw) | cm_hash(c.a_r[r], c.b_r[r], x, s.lw);
      atomicAdd(&a.cnt[ci], 1u);
      const uint32_t prev = atomicMax(&a.top1[ci], x);
      // the value displaced from the maximum competes for second place; the
      // last survivor is the second largest whatever the arrival order
      atomicMax(&a.top2[ci], min(prev, x));
    }
  }
}

__device__ __forceinline__ void tk_write(const TkAcc& a, uint2* __restrict__ cells, uint32_t nc, bool fresh,
                                         uint32_t tid, uint32_t nt) {
  for (uint32_t i = tid; i < nc; i += nt) {
    const uint2 old = fresh ? make_uint2(SL_EMPTY, 0u) : cells[i];
    cells[i] = tk_final(old, a.cnt[i], a.top1[i], a.top2[i]);
  }
}

__device__ __forceinline__ uint32_t tk_ncp(uint32_t nc) { return (nc + 63) & ~63u; }

// 32-bit parity words of a sketch (one bit per cell).
__device__ __forceinline__ uint32_t tk_pw(uint32_t nc) { return (nc + 31) / 32; }

// Build, buckets of at most heavy_t ids: one wave per bucket over the
// table's sorted ids (ascending within a bucket); every bucket of the table
// is written, empty ones as empty sketches.  Heavier buckets are listed.
__global__ void __launch_bounds__(kTkWaves * SL_WAVE)
    k_tk_light(Shape s, ConstView c, uint32_t t, const uint32_t* __restrict__ sv, const uint32_t* __restrict__ start,
               const uint32_t* __restrict__ end, TablesView tab, uint32_t heavy_t, uint32_t* __restrict__ heavy_list,
               uint32_t* __restrict__ heavy_n, uint32_t* __restrict__ hpar) {
  extern __shared__ uint32_t lds32[];
  const uint32_t wave = threadIdx.x / SL_WAVE, lane = lane_id();
  const uint32_t nc = tk_cells(s), ncp = tk_ncp(nc);
  const TkAcc a = tk_acc(lds32 + wave * 3 * ncp, ncp);
  for (uint32_t b = blockIdx.x * kTkWaves + wave; b < s.nb; b += gridDim.x * kTkWaves) {
    uint32_t s0, e0;
    bucket_run(start, end, b, s0, e0);
    if (e0 - s0 > heavy_t) {
      if (lane == 0) {
        const uint32_t h = atomicAdd(heavy_n, 1u);
        heavy_list[h] = b;
        for (uint32_t w = 0; w < tk_pw(nc); ++w) hpar[(uint64_t)h * tk_pw(nc) + w] = 0;
      }
      continue;
    }
    tk_clear(a, nc, lane, SL_WAVE);
    wave_sync();
    tk_add(s, c, a, sv, s0 + lane, e0, SL_WAVE);
    wave_sync();
    tk_write(a, (uint2*)tab.ids + ((uint64_t)t * s.nb + b) * nc, nc, true, lane, SL_WAVE);
    if (lane == 0) tab.seen[(uint64_t)t * s.nb + b] = e0 - s0;
    wave_sync();
  }
}

// Build, listed heavy buckets (more than heavy_t ids).  A bucket's ids are
// ascending in the sorted order (the radix sort is stable and the build's
// values are the row numbers), so a cell's two largest ids are its last two
// in that order.  What the final state needs beyond them is only whether the
// cell's count is odd, and a parity adds up without atomics:
//   k_tk_heavy_chunks - chunks of kTkChunk ids, spread over the grid, XOR
//     one bit per (id, row) into per-thread parity words, reduce them over
//     the block and XOR them into the bucket's global parity words; the
//     block holding a bucket's last chunk also scans the bucket backwards,
//     a block-width of ids at a time with LDS atomics, until every cell has
//     two hits (or the bucket's start), and stores each cell's hits (capped
//     at 2), largest and second largest;
//   k_tk_heavy_final - per cell: no hit -> empty; odd parity -> (largest, 1);
//     even -> (second largest, 0).
constexpr uint32_t kTkChunk = 16384;
constexpr uint32_t kTkChunkThreads = 256;

template <int P>  // 64-bit parity words per thread (cells / 64, rounded up)
__global__ void __launch_bounds__(kTkChunkThreads)
    k_tk_heavy_chunks(Shape s, ConstView c, const uint32_t* __restrict__ sv, const uint32_t* __restrict__ start,
                      const uint32_t* __restrict__ end, const uint32_t* __restrict__ heavy_list,
                      const uint32_t* __restrict__ heavy_n, uint32_t* __restrict__ hpar, uint32_t* __restrict__ htop) {
  extern __shared__ uint32_t lds32[];
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / SL_WAVE;
  constexpr uint32_t NW = kTkChunkThreads / SL_WAVE;
  const uint32_t nc = tk_cells(s), ncp = tk_ncp(nc), pw = tk_pw(nc);
  uint32_t* wpar = lds32;                    // [NW][2 * P] per-wave parity
  uint32_t* flag = lds32 + NW * 2 * P;       // [1] some cell still lacks two hits
  const TkAcc a = tk_acc(lds32 + NW * 2 * P + 2, ncp);
  const uint32_t nh = *heavy_n;
  uint64_t base = 0;  // chunks of the buckets before h
  for (uint32_t h = 0; h < nh; ++h) {
    const uint32_t b = heavy_list[h];
    uint32_t s0, e0;
    bucket_run(start, end, b, s0, e0);
    const uint32_t nch = (e0 - s0 + kTkChunk - 1) / kTkChunk;
    // this block's chunks of bucket h: global chunk numbers = blockIdx.x (mod grid)
    uint64_t j0 = (blockIdx.x + gridDim.x - (uint32_t)(base % gridDim.x)) % gridDim.x;
    for (uint64_t j = j0; j < nch; j += gridDim.x) {
      const uint32_t c0 = s0 + (uint32_t)j * kTkChunk, c1 = min(e0, c0 + kTkChunk);
      uint64_t par[P];
#pragma unroll
      for (int w = 0; w < P; ++w) par[w] = 0;
      for (uint32_t i = c0 + tid; i < c1; i += kTkChunkThreads) {
        const uint32_t x = sv[i];
        for (uint32_t r = 0; r < s.d; ++r) {
          const uint32_t ci = (r << s.lw) | cm_hash(c.a_r[r], c.b_r[r], x, s.lw);
#pragma unroll
          for (int w = 0; w < P; ++w) par[w] ^= (ci >> 6) == (uint32_t)w ? (1ull << (ci & 63)) : 0ull;
        }
      }
#pragma unroll
      for (int w = 0; w < P; ++w) {
        uint32_t lo = (uint32_t)par[w], hi = (uint32_t)(par[w] >> 32);
#pragma unroll
        for (int o = SL_WAVE / 2; o > 0; o >>= 1) {
          lo ^= __shfl_xor(lo, o, SL_WAVE);
          hi ^= __shfl_xor(hi, o, SL_WAVE);
        }
        if (lane == 0) {
          wpar[wave * 2 * P + 2 * w] = lo;
          wpar[wave * 2 * P + 2 * w + 1] = hi;
        }
      }
      __syncthreads();
      if (tid < pw) {
        uint32_t v = 0;
        for (uint32_t q = 0; q < NW; ++q) v ^= wpar[q * 2 * P + tid];
        if (v) atomicXor(&hpar[(uint64_t)h * pw + tid], v);
      }
      __syncthreads();
      if (j + 1 == nch) {
        // the bucket's two largest ids per cell, from its end backwards
        tk_clear(a, nc, tid, kTkChunkThreads);
        __syncthreads();
        for (uint32_t stop = e0; stop > s0;) {
          const uint32_t from = stop > s0 + kTkChunkThreads ? stop - kTkChunkThreads : s0;
          if (from + tid < stop) {
            const uint32_t x = sv[from + tid];
            for (uint32_t r = 0; r < s.d; ++r) {
              const uint32_t ci = (r << s.lw) | cm_hash(c.a_r[r], c.b_r[r], x, s.lw);
              atomicAdd(&a.cnt[ci], 1u);
              const uint32_t prev = atomicMax(&a.top1[ci], x);
              atomicMax(&a.top2[ci], min(prev, x));
            }
          }
          if (tid == 0) *flag = 0;
          __syncthreads();
          for (uint32_t i = tid; i < nc; i += kTkChunkThreads)
            if (a.cnt[i] < 2) *flag = 1;
          __syncthreads();
          const uint32_t more = *flag;
          __syncthreads();
          if (!more) break;
          stop = from;
        }
        uint32_t* top = htop + (uint64_t)h * nc * 3;
        for (uint32_t i = tid; i < nc; i += kTkChunkThreads) {
          top[3 * i] = min(a.cnt[i], 2u);
          top[3 * i + 1] = a.top1[i];
          top[3 * i + 2] = a.top2[i];
        }
        __syncthreads();
      }
    }
    base += nch;
  }
}

__global__ void __launch_bounds__(kTkChunkThreads)
    k_tk_heavy_final(Shape s, uint32_t t, const uint32_t* __restrict__ start, const uint32_t* __restrict__ end,
                     TablesView tab, const uint32_t* __restrict__ heavy_list, const uint32_t* __restrict__ heavy_n,
                     const uint32_t* __restrict__ hpar, const uint32_t* __restrict__ htop) {
  const uint32_t nc = tk_cells(s), pw = tk_pw(nc), nh = *heavy_n;
  for (uint32_t h = blockIdx.x; h < nh; h += gridDim.x) {
    const uint32_t b = heavy_list[h];
    uint2* cells = (uint2*)tab.ids + ((uint64_t)t * s.nb + b) * nc;
    const uint32_t* top = htop + (uint64_t)h * nc * 3;
    for (uint32_t i = threadIdx.x; i < nc; i += kTkChunkThreads) {
      const uint32_t odd = (hpar[(uint64_t)h * pw + (i >> 5)] >> (i & 31)) & 1u;
      cells[i] = top[3 * i] == 0 ? make_uint2(SL_EMPTY, 0u)
                 : odd           ? make_uint2(top[3 * i + 1], 1u)
                                 : make_uint2(top[3 * i + 2], 0u);
    }
    if (threadIdx.x == 0) {
      uint32_t s0, e0;
      bucket_run(start, end, b, s0, e0);
      tab.seen[(uint64_t)t * s.nb + b] = e0 - s0;
    }
  }
}

// Insert, sorted (table << B | bucket) keys with ascending ids per segment:
// one wave per segment folds the new ids into the stored sketch.
__global__ void __launch_bounds__(kTkWaves * SL_WAVE)
    k_tk_segments(Shape s, ConstView c, const uint32_t* __restrict__ sk, const uint32_t* __restrict__ sv, uint64_t n,
                  const uint32_t* __restrict__ seg_start, const uint32_t* __restrict__ nseg, TablesView tab) {
  extern __shared__ uint32_t lds32[];
  const uint32_t wave = threadIdx.x / SL_WAVE, lane = lane_id();
  const uint32_t nc = tk_cells(s), ncp = tk_ncp(nc);
  const TkAcc a = tk_acc(lds32 + wave * 3 * ncp, ncp);
  const uint32_t ns = *nseg;
  for (uint32_t g = blockIdx.x * kTkWaves + wave; g < ns; g += gridDim.x * kTkWaves) {
    const uint32_t s0 = seg_start[g];
    const uint32_t e0 = g + 1 < ns ? seg_start[g + 1] : (uint32_t)n;
    const uint32_t ck = sk[s0];
    const uint32_t t = ck >> s.B, b = ck & (s.nb - 1);
    tk_clear(a, nc, lane, SL_WAVE);
    wave_sync();
    tk_add(s, c, a, sv, s0 + lane, e0, SL_WAVE);
    wave_sync();
    tk_write(a, (uint2*)tab.ids + ((uint64_t)t * s.nb + b) * nc, nc, false, lane, SL_WAVE);
    if (lane == 0) tab.seen[(uint64_t)t * s.nb + b] += e0 - s0;
    wave_sync();
  }
}

// Insert, small batches: one wave per run record (bucket, first | len << 16)
// of the LDS grouping pass; the run's ids are items[first .. first + len).
__global__ void __launch_bounds__(kTkWaves * SL_WAVE)
    k_tk_runs(Shape s, ConstView c, const uint2* __restrict__ recs, const uint32_t* __restrict__ items, uint32_t n,
              TablesView tab) {
  extern __shared__ uint32_t lds32[];
  const uint32_t wave = threadIdx.x / SL_WAVE, lane = lane_id();
  const uint32_t nc = tk_cells(s), ncp = tk_ncp(nc);
  const TkAcc a = tk_acc(lds32 + wave * 3 * ncp, ncp);
  const uint64_t run = (uint64_t)blockIdx.x * kTkWaves + wave;
  if (run >= (uint64_t)s.L * n) return;
  const uint2 rec = recs[run];
  const uint32_t len = rec.y >> 16;
  if (len == 0) return;
  const uint32_t t = (uint32_t)(run / n), first = rec.y & 0xFFFFu, b = rec.x;
  tk_clear(a, nc, lane, SL_WAVE);
  wave_sync();
  tk_add(s, c, a, items + (uint64_t)t * n + first, lane, len, SL_WAVE);
  wave_sync();
  tk_write(a, (uint2*)tab.ids + ((uint64_t)t * s.nb + b) * nc, nc, false, lane, SL_WAVE);
  if (lane == 0) tab.seen[(uint64_t)t * s.nb + b] += len;
}

// Query: one wave per query.  LDS per wave: DOPH scratch, the L bucket ids,
// the merged sketch and the compacted candidate keys.
struct TkQLayout {
  uint32_t doph, bk, sh, sc, keys, words;  // offsets in 32-bit words
};

__host__ __device__ inline TkQLayout tk_qlayout(const Shape& s) {
  TkQLayout o;
  const uint32_t ncp = (((s.d << s.lw) + 63) / 64) * 64;
  o.doph = 0;
  o.bk = o.doph + 2 * s.M + ((s.M + 63) / 64) * 2;
  o.sh = o.bk + s.L;
  o.sc = o.sh + ncp;
  o.keys = (o.sc + ncp + 1) & ~1u;  // 8-byte aligned
  o.words = o.keys + 2 * ncp;
  return o;
}

template <int E>  // cells per lane
__global__ void __launch_bounds__(kTkWaves * SL_WAVE)
    k_tk_query(Shape s, ConstView c, TablesView tab, QueryArgs a, uint32_t waves) {
  extern __shared__ uint32_t lds32[];
  const uint32_t wave = threadIdx.x / SL_WAVE, lane = lane_id();
  const uint64_t q = (uint64_t)blockIdx.x * waves + wave;
  if (wave >= waves || q >= a.q.n_rows) return;
  const TkQLayout lay = tk_qlayout(s);
  uint32_t* base = lds32 + wave * lay.words;
  uint32_t* bk = base + lay.bk;
  uint32_t* sh = base + lay.sh;
  uint32_t* sc = base + lay.sc;
  uint64_t* keys = (uint64_t*)(base + lay.keys);
  const uint32_t nc = tk_cells(s);
  // 1. bucket ids of the query
  {
    const int64_t beg = a.q.indptr[q], end = a.q.indptr[q + 1];
    const uint32_t* h = doph_wave<false>(s, c, a.q.indices + beg, (uint32_t)(end - beg), base + lay.doph);
    for (uint32_t t = lane; t < s.L; t += SL_WAVE) bk[t] = table_bucket<false>(s, c, h, t);
  }
  wave_sync();
  // 2. fold the L sketches in table order, eight tables' cells in flight
  uint2 S[E];
#pragma unroll
  for (int e = 0; e < E; ++e) S[e] = make_uint2(SL_EMPTY, 0u);
  const uint2* cells = (const uint2*)tab.ids;
  for (uint32_t t0 = 0; t0 < s.L; t0 += 8) {
    uint2 v[8][E];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t t = t0 + j;
      const uint64_t row = t < s.L ? ((uint64_t)t * s.nb + bk[t]) * nc : 0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const uint32_t ci = lane + 64u * e;
        v[j][e] = (t < s.L && ci < nc) ? cells[row + ci] : make_uint2(SL_EMPTY, 0u);
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const uint2 x = v[j][e];
        uint2& y = S[e];
        if (y.x == x.x) {
          y.y += x.y;
        } else if (x.y > y.y) {
          y = make_uint2(x.x, x.y - y.y);
        } else if (x.y < y.y) {
          y.y -= x.y;
        } else {
          y = make_uint2(min(x.x, y.x), 0u);
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t ci = lane + 64u * e;
    if (ci < nc) {
      sh[ci] = S[e].x;
      sc[ci] = S[e].y;
    }
  }
  wave_sync();
  // 3. candidates: count >= 1, and no other row holds the same id with a
  //    larger count (or an equal count in an earlier row)
  uint32_t nv = 0;
  uint64_t mykey[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t ci = lane + 64u * e;
    const uint32_t id = S[e].x, n = S[e].y;
    bool ok = ci < nc && n >= 1 && id != SL_EMPTY;
    if (ok) {
      const uint32_t r = ci >> s.lw;
      for (uint32_t r2 = 0; r2 < s.d; ++r2) {
        if (r2 == r) continue;
        const uint32_t c2 = (r2 << s.lw) | cm_hash(c.a_r[r2], c.b_r[r2], id, s.lw);
        const uint32_t n2 = sc[c2];
        if (sh[c2] == id && (n2 > n || (n2 == n && r2 < r))) ok = false;
      }
    }
    mykey[e] = ok ? (((uint64_t)(~n) << 32) | id) : ~0ull;
    const uint64_t m = ballot64(ok);
    if (ok) keys[nv + (uint32_t)__builtin_popcountll(m & lanemask_lt())] = mykey[e];
    nv += (uint32_t)__builtin_popcountll(m);
  }
  wave_sync();
  // 4. rank every candidate among the others and write the first kk
  uint32_t kq = a.kq ? a.kq[q] : a.k;
  if (kq > s.k_max) kq = s.k_max;
  const uint32_t kk = min(kq, nv);
  uint32_t* oid = a.out_ids + q * s.k_max;
  uint32_t* osc = a.out_scores + q * s.k_max;
  uint32_t rank[E];
#pragma unroll
  for (int e = 0; e < E; ++e) rank[e] = 0;
  for (uint32_t j = 0; j < nv; ++j) {
    const uint64_t kj = keys[j];
#pragma unroll
    for (int e = 0; e < E; ++e) rank[e] += kj < mykey[e] ? 1u : 0u;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (mykey[e] != ~0ull && rank[e] < kk) {
      oid[rank[e]] = (uint32_t)mykey[e];
      osc[rank[e]] = ~(uint32_t)(mykey[e] >> 32);
    }
  }
  for (uint32_t i = kk + lane; i < s.k_max; i += SL_WAVE) {
    oid[i] = SL_EMPTY;
    osc[i] = 0;
  }
}

uint32_t tk_grid(uint64_t work, uint32_t per_block, uint32_t cap) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

size_t tk_acc_lds(const Shape& s) { return (size_t)3 * ((((s.d << s.lw) + 63) / 64) * 64) * 4; }

uint32_t tk_query_waves(const Shape& s) {
  const size_t per = (size_t)tk_qlayout(s).words * 4;
  uint32_t w = kTkWaves;
  while (w > 1 && per * w > 65536) --w;
  return w;
}

}  // namespace

bool tk_supported(const Shape& s) {
  const uint32_t nc = s.d << s.lw;
  return s.lw <= 8 && nc >= 1 && nc <= 256 && (size_t)tk_qlayout(s).words * 4 <= 160 * 1024;
}

hipError_t launch_tk_light(const Shape& s, const ConstView& c, uint32_t t, const uint32_t* sv, const uint32_t* start,
                           const uint32_t* end, TablesView tab, uint32_t heavy_t, uint32_t* heavy_list,
                           uint32_t* heavy_n, uint32_t* hpar, hipStream_t st) {
  hipLaunchKernelGGL(k_tk_light, dim3(tk_grid(s.nb, kTkWaves, 16384)), dim3(kTkWaves * SL_WAVE),
                     kTkWaves * tk_acc_lds(s), st, s, c, t, sv, start, end, tab, heavy_t, heavy_list, heavy_n, hpar);
  return hipGetLastError();
}

size_t tk_heavy_scratch_words(const Shape& s, uint64_t max_heavy) {
  const uint64_t nc = s.d << s.lw;
  return (size_t)max_heavy * ((nc + 31) / 32 + 3 * nc);
}

hipError_t launch_tk_heavy(const Shape& s, const ConstView& c, uint32_t t, const uint32_t* sv, const uint32_t* start,
                           const uint32_t* end, TablesView tab, const uint32_t* heavy_list, const uint32_t* heavy_n,
                           uint64_t n, uint32_t* scratch, hipStream_t st) {
  // heavy buckets hold more than kTkChunk ids each, so there are at most
  // n / kTkChunk of them and at most 2 n / kTkChunk chunks
  const uint64_t max_heavy = n / kTkChunk + 1;
  const uint32_t nc = s.d << s.lw;
  uint32_t* hpar = scratch;
  uint32_t* htop = scratch + max_heavy * ((nc + 31) / 32);
  const uint32_t P = (nc + 63) / 64;
  const uint32_t grid = tk_grid(2 * (n / kTkChunk) + 2, 1, 2048);
  const size_t lds = (size_t)((kTkChunkThreads / SL_WAVE) * 2 * P + 2) * 4 + tk_acc_lds(s);
  if (P <= 1)
    hipLaunchKernelGGL(k_tk_heavy_chunks<1>, dim3(grid), dim3(kTkChunkThreads), lds, st, s, c, sv, start, end,
                       heavy_list, heavy_n, hpar, htop);
  else if (P <= 2)
    hipLaunchKernelGGL(k_tk_heavy_chunks<2>, dim3(grid), dim3(kTkChunkThreads), lds, st, s, c, sv, start, end,
                       heavy_list, heavy_n, hpar, htop);
  else
    hipLaunchKernelGGL(k_tk_heavy_chunks<4>, dim3(grid), dim3(kTkChunkThreads), lds, st, s, c, sv, start, end,
                       heavy_list, heavy_n, hpar, htop);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tk_heavy_final, dim3(tk_grid(max_heavy, 1, 1024)), dim3(kTkChunkThreads), 0, st, s, t, start,
                     end, tab, heavy_list, heavy_n, hpar, htop);
  return hipGetLastError();
}

__global__ void k_tk_clear(uint2* __restrict__ p, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = make_uint2(SL_EMPTY, 0u);
}

hipError_t launch_tk_clear(const Shape& s, TablesView tab, hipStream_t st) {
  const uint64_t n = (uint64_t)s.L * s.nb * (s.d << s.lw);
  hipLaunchKernelGGL(k_tk_clear, dim3(tk_grid(n, 256, 65536)), dim3(256), 0, st, (uint2*)tab.ids, n);
  return hipGetLastError();
}

hipError_t launch_tk_segments(const Shape& s, const ConstView& c, const uint32_t* sk, const uint32_t* sv, uint64_t n,
                              const uint32_t* seg_start, const uint32_t* nseg, TablesView tab, hipStream_t st) {
  hipLaunchKernelGGL(k_tk_segments, dim3(tk_grid(n, kTkWaves, 16384)), dim3(kTkWaves * SL_WAVE),
                     kTkWaves * tk_acc_lds(s), st, s, c, sk, sv, n, seg_start, nseg, tab);
  return hipGetLastError();
}

hipError_t launch_tk_runs(const Shape& s, const ConstView& c, const uint2* recs, const uint32_t* items, uint32_t n,
                          TablesView tab, hipStream_t st) {
  const uint64_t runs = (uint64_t)s.L * n;
  hipLaunchKernelGGL(k_tk_runs, dim3((uint32_t)((runs + kTkWaves - 1) / kTkWaves)), dim3(kTkWaves * SL_WAVE),
                     kTkWaves * tk_acc_lds(s), st, s, c, recs, items, n, tab);
  return hipGetLastError();
}

hipError_t launch_tk_query(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& a,
                           hipStream_t st) {
  if (a.q.n_rows == 0) return hipSuccess;
  if (!tk_supported(s)) return hipErrorInvalidValue;
  const uint32_t waves = tk_query_waves(s);
  const size_t lds = (size_t)tk_qlayout(s).words * 4 * waves;
  const uint32_t E = ((s.d << s.lw) + 63) / 64;
  const void* f = E <= 1 ? (const void*)k_tk_query<1>
                  : E <= 2 ? (const void*)k_tk_query<2>
                           : (const void*)k_tk_query<4>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const uint64_t blocks = (a.q.n_rows + waves - 1) / waves;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  Shape sh = s;
  ConstView cv = c;
  TablesView tv = tab;
  QueryArgs qa = a;
  uint32_t w = waves;
  void* args[] = {&sh, &cv, &tv, &qa, &w};
  hipError_t e = hipLaunchKernel(f, dim3((uint32_t)blocks), dim3(kTkWaves * SL_WAVE), args, lds, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace slash
