// Query kernel (Section 2.3 query phase, "Cheap Frequency based Filtering";
// Algorithm 2 on one node; Section 2.4 / Appendix 2 for the count-min style
// frequency sketch whose top-k identities are the answer).
//
// One work-group answers one query at a time:
//   1. wave 0 hashes the query (DOPH) into its L bucket ids;
//   2. every thread gathers reservoir slots (table t, slot j) of the probed
//      buckets straight from HBM (coalesced R-slot rows; EMPTY slots skipped);
//   3. count-min: d rows of w 16-bit counters in LDS, incremented with LDS
//      atomics (a counter never exceeds L * R <= 65535);
//   4. estimate = min over rows; duplicates of an id are folded by an LDS
//      open-addressing set so each distinct id is ranked once;
//   5. the k-th largest key (estimate << 32 | ~id) is found by an MSD radix
//      select over 8-bit digits, the winners are ranked by counting and
//      written with stride k_max, padded with (EMPTY, 0).
// The persistent form loops over queries taken from a device work counter.
#include "doph.h"

namespace slash {

namespace {

constexpr uint32_t kMaxSpt = 16;  // reservoir slots per thread

struct QLayout {
  uint32_t doph, buckets, cm, hs, hist, sel, misc, total;  // offsets in 32-bit words
  uint32_t cm_words, hs_size;
};

__host__ __device__ inline uint32_t next_pow2(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

__host__ __device__ inline QLayout q_layout(const Shape& s) {
  QLayout o;
  uint32_t w = 1u << s.lw;
  o.doph = 0;
  o.buckets = o.doph + 2 * s.M + ((s.M + 63) / 64) * 2;
  o.cm = o.buckets + s.L;
  o.cm_words = (s.d * w + 1) / 2;
  o.hs_size = next_pow2(2 * s.L * s.R);
  if (o.hs_size < 64) o.hs_size = 64;
  o.hs = o.cm + o.cm_words;
  o.hist = o.hs + o.hs_size;
  o.sel = o.hist + 256;
  if (o.sel & 1) o.sel++;
  o.misc = o.sel + 2 * s.k_max;
  o.total = o.misc + 16;
  return o;
}

__device__ __forceinline__ uint32_t hs_slot(uint32_t id, uint32_t mask) { return (id * 0x9E3779B1u) & mask; }

template <int WAVES>
__device__ void query_one(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& a, uint32_t q,
                          uint32_t* lds, const QLayout& lay) {
  constexpr uint32_t NT = WAVES * SL_WAVE;
  const uint32_t tid = threadIdx.x, wave = tid / SL_WAVE, lane = lane_id();
  uint32_t* bk = lds + lay.buckets;
  uint32_t* cmw = lds + lay.cm;
  uint32_t* hs = lds + lay.hs;
  uint32_t* hist = lds + lay.hist;
  uint64_t* sel = (uint64_t*)(lds + lay.sel);
  uint32_t* misc = lds + lay.misc;
  const uint32_t hs_mask = lay.hs_size - 1;
  const uint32_t slots = s.L * s.R;
  const uint32_t spt = (slots + NT - 1) / NT;

  // clear sketch, id set and counters
  for (uint32_t e = tid; e < lay.cm_words; e += NT) cmw[e] = 0;
  for (uint32_t e = tid; e < lay.hs_size; e += NT) hs[e] = SL_EMPTY;
  if (tid < 16) misc[tid] = 0;
  // 1. hash
  if (wave == 0) {
    const int64_t beg = a.q.indptr[q], end = a.q.indptr[q + 1];
    const uint32_t* h = doph_wave(s, c, a.q.indices + beg, (uint32_t)(end - beg), lds + lay.doph);
    for (uint32_t t = lane; t < s.L; t += SL_WAVE) bk[t] = table_bucket(s, c, h, t);
  }
  __syncthreads();
  // 2. gather + 3. count
  uint32_t id[kMaxSpt];
#pragma unroll
  for (uint32_t i = 0; i < kMaxSpt; ++i) {
    id[i] = SL_EMPTY;
    if (i < spt) {
      uint32_t sl = tid + i * NT;
      if (sl < slots) {
        uint32_t t = sl / s.R, j = sl - t * s.R;
        id[i] = tab.ids[((uint64_t)t * s.nb + bk[t]) * s.R + j];
      }
    }
  }
#pragma unroll
  for (uint32_t i = 0; i < kMaxSpt; ++i) {
    if (i < spt && id[i] != SL_EMPTY) {
      for (uint32_t r = 0; r < s.d; ++r) {
        uint32_t g = (r << s.lw) + cm_hash(c.a_r[r], c.b_r[r], id[i], s.lw);
        atomicAdd(&cmw[g >> 1], 1u << ((g & 1u) * 16));
      }
    }
  }
  __syncthreads();
  // 4. estimates and distinct representatives
  uint64_t key[kMaxSpt];
  uint32_t nrep = 0;
#pragma unroll
  for (uint32_t i = 0; i < kMaxSpt; ++i) {
    key[i] = 0;
    if (i < spt && id[i] != SL_EMPTY) {
      uint32_t est = 0xFFFFFFFFu;
      for (uint32_t r = 0; r < s.d; ++r) {
        uint32_t g = (r << s.lw) + cm_hash(c.a_r[r], c.b_r[r], id[i], s.lw);
        uint32_t v = (cmw[g >> 1] >> ((g & 1u) * 16)) & 0xFFFFu;
        est = min(est, v);
      }
      uint32_t h = hs_slot(id[i], hs_mask);
      bool rep = false;
      for (;;) {
        uint32_t prev = atomicCAS(&hs[h], SL_EMPTY, id[i]);
        if (prev == SL_EMPTY) {
          rep = true;
          break;
        }
        if (prev == id[i]) break;
        h = (h + 1) & hs_mask;
      }
      if (rep) {
        key[i] = ((uint64_t)est << 32) | (uint32_t)~id[i];
        ++nrep;
      }
    }
  }
  // block total of representatives
  {
    uint32_t v = nrep;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, SL_WAVE);
    if (lane == 0) atomicAdd(&misc[0], v);
  }
  __syncthreads();
  const uint32_t total = misc[0];
  uint32_t kq = a.kq ? a.kq[q] : a.k;
  if (kq > s.k_max) kq = s.k_max;
  const uint32_t kk = min(kq, total);
  uint32_t* oid = a.out_ids + (uint64_t)q * s.k_max;
  uint32_t* osc = a.out_scores + (uint64_t)q * s.k_max;
  // 5. threshold key: keys >= thr are exactly the kk largest
  uint64_t thr = 1;  // every representative (their keys are >= 2^32)
  if (kk > 0 && kk < total) {
    uint64_t prefix = 0;
    uint32_t remaining = kk;
    for (int shift = 40; shift >= 0; shift -= 8) {
      for (uint32_t e = tid; e < 256; e += NT) hist[e] = 0;
      __syncthreads();
      const uint64_t hi_mask = shift + 8 >= 64 ? 0ull : (~0ull << (shift + 8));
#pragma unroll
      for (uint32_t i = 0; i < kMaxSpt; ++i) {
        if (key[i] != 0 && (key[i] & hi_mask) == (prefix & hi_mask))
          atomicAdd(&hist[(uint32_t)(key[i] >> shift) & 255u], 1u);
      }
      __syncthreads();
      if (wave == 0) {
        // lane owns digits 4*lane .. 4*lane+3; suffix sums from the top
        uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
        uint32_t mine = h0 + h1 + h2 + h3;
        uint32_t above = 0;  // sum over lanes > lane
        uint32_t v = mine;
        for (int o = 1; o < SL_WAVE; o <<= 1) {
          uint32_t y = __shfl_down(v, o, SL_WAVE);
          if (lane + o < SL_WAVE) v += y;
        }
        above = v - mine;
        uint32_t hh[4] = {h0, h1, h2, h3};
        uint32_t cum = above;
        for (int j = 3; j >= 0; --j) {
          if (cum < remaining && remaining <= cum + hh[j]) {
            misc[1] = 4 * lane + j;
            misc[2] = cum;
            misc[3] = hh[j];
          }
          cum += hh[j];
        }
      }
      __syncthreads();
      uint32_t D = misc[1], cum = misc[2], cnt = misc[3];
      remaining -= cum;
      prefix |= (uint64_t)D << shift;
      __syncthreads();
      if (remaining == cnt) break;  // the whole digit bin is selected
    }
    thr = prefix;
  }
  // 6. collect winners
  if (kk > 0) {
#pragma unroll
    for (uint32_t i = 0; i < kMaxSpt; ++i) {
      if (key[i] != 0 && key[i] >= thr) {
        uint32_t p = atomicAdd(&misc[4], 1u);
        sel[p] = key[i];
      }
    }
  }
  __syncthreads();
  // 7. rank winners by counting (keys are distinct) and write the row
  for (uint32_t e = tid; e < kk; e += NT) {
    uint64_t x = sel[e];
    uint32_t r = 0;
    for (uint32_t j = 0; j < kk; ++j) r += sel[j] > x ? 1u : 0u;
    oid[r] = ~(uint32_t)x;
    osc[r] = (uint32_t)(x >> 32);
  }
  for (uint32_t e = kk + tid; e < s.k_max; e += NT) {
    oid[e] = SL_EMPTY;
    osc[e] = 0;
  }
  __syncthreads();
}

template <int WAVES>
__global__ void __launch_bounds__(WAVES * SL_WAVE) k_query(Shape s, ConstView c, TablesView tab, QueryArgs a) {
  extern __shared__ uint32_t lds[];
  const QLayout lay = q_layout(s);
  for (uint64_t q = blockIdx.x; q < a.q.n_rows; q += gridDim.x) query_one<WAVES>(s, c, tab, a, (uint32_t)q, lds, lay);
}

template <int WAVES>
__global__ void __launch_bounds__(WAVES * SL_WAVE)
    k_query_persistent(Shape s, ConstView c, TablesView tab, QueryArgs a, uint32_t per_ticket, uint32_t* ticket) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t base_sh;
  const QLayout lay = q_layout(s);
  const uint64_t n = a.q.n_rows;
  for (;;) {
    if (threadIdx.x == 0) base_sh = atomicAdd(ticket, per_ticket);
    __syncthreads();
    const uint64_t base = base_sh;
    __syncthreads();
    if (base >= n) break;
    const uint64_t stop = base + per_ticket < n ? base + per_ticket : n;
    for (uint64_t q = base; q < stop; ++q) query_one<WAVES>(s, c, tab, a, (uint32_t)q, lds, lay);
  }
}

template <int WAVES>
hipError_t set_lds_attr(size_t lds) {
  static bool done = false;
  if (!done && lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_query<WAVES>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_query_persistent<WAVES>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
    done = true;
  }
  return hipSuccess;
}

}  // namespace

uint32_t query_default_waves(const Shape& s) {
  uint32_t slots = s.L * s.R;
  uint32_t w = (slots + kMaxSpt * SL_WAVE - 1) / (kMaxSpt * SL_WAVE);
  uint32_t waves = 1;
  while (waves < w) waves <<= 1;
  if (waves < 4 && slots >= 4 * SL_WAVE * 2) waves = 4;
  return waves;
}

int query_block_threads(const Shape& s, uint32_t waves) { return (int)(waves * SL_WAVE); }

size_t query_lds_bytes(const Shape& s, uint32_t waves) {
  (void)waves;
  return (size_t)q_layout(s).total * 4;
}

bool query_supported(const Shape& s, uint32_t waves) {
  if (waves == 0 || waves > 16) return false;
  if (s.L * s.R > kMaxSpt * SL_WAVE * waves) return false;
  if (s.L * s.R > 65535u) return false;
  return query_lds_bytes(s, waves) <= 160 * 1024;
}

bool query_supported(const Shape& s) { return query_supported(s, query_default_waves(s)); }

#define SLASH_Q_DISPATCH(W, ...)        \
  switch (W) {                          \
    case 1: __VA_ARGS__(1); break;      \
    case 2: __VA_ARGS__(2); break;      \
    case 4: __VA_ARGS__(4); break;      \
    case 8: __VA_ARGS__(8); break;      \
    case 16: __VA_ARGS__(16); break;    \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_query_waves(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& a,
                              uint32_t waves, hipStream_t st) {
  if (a.q.n_rows == 0) return hipSuccess;
  if (!query_supported(s, waves)) return hipErrorInvalidValue;
  size_t lds = query_lds_bytes(s, waves);
  uint32_t grid = (uint32_t)(a.q.n_rows < (1u << 30) ? a.q.n_rows : (1u << 30));
  hipError_t e = hipSuccess;
#define L1(W)                                                                                 \
  do {                                                                                        \
    e = set_lds_attr<W>(lds);                                                                 \
    if (e == hipSuccess)                                                                      \
      hipLaunchKernelGGL(k_query<W>, dim3(grid), dim3(W * SL_WAVE), lds, st, s, c, tab, a);   \
  } while (0)
  SLASH_Q_DISPATCH(waves, L1)
#undef L1
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_query(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& a,
                        hipStream_t st) {
  return launch_query_waves(s, c, tab, a, query_default_waves(s), st);
}

hipError_t launch_query_persistent(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& a,
                                   uint32_t waves, uint32_t per_ticket, uint32_t grid, uint32_t* ticket,
                                   hipStream_t st) {
  if (!query_supported(s, waves)) return hipErrorInvalidValue;
  if (per_ticket == 0) per_ticket = 1;
  size_t lds = query_lds_bytes(s, waves);
  hipError_t e = hipSuccess;
#define L2(W)                                                                                        \
  do {                                                                                               \
    e = set_lds_attr<W>(lds);                                                                        \
    if (e == hipSuccess)                                                                             \
      hipLaunchKernelGGL(k_query_persistent<W>, dim3(grid), dim3(W * SL_WAVE), lds, st, s, c, tab, a, \
                         per_ticket, ticket);                                                        \
  } while (0)
  SLASH_Q_DISPATCH(waves, L2)
#undef L2
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

void* persistent_query_kernel(uint32_t waves) {
  switch (waves) {
    case 1: return (void*)k_query_persistent<1>;
    case 2: return (void*)k_query_persistent<2>;
    case 4: return (void*)k_query_persistent<4>;
    case 8: return (void*)k_query_persistent<8>;
    case 16: return (void*)k_query_persistent<16>;
    default: return nullptr;
  }
}

// Occupancy of the persistent kernel: resident work-groups per CU.
hipError_t query_occupancy(const Shape& s, uint32_t waves, int* per_cu) {
  size_t lds = query_lds_bytes(s, waves);
  hipError_t e = hipSuccess;
#define L3(W)                                                                                                \
  do {                                                                                                       \
    e = set_lds_attr<W>(lds);                                                                                \
    if (e == hipSuccess)                                                                                     \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (const void*)k_query_persistent<W>, W * SL_WAVE, \
                                                       lds);                                                 \
  } while (0)
  SLASH_Q_DISPATCH(waves, L3)
#undef L3
  return e;
}

}  // namespace slash
