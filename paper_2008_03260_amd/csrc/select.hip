// Bottom-R reservoir selection (Section 3 "Avoid Skewed buckets": heavy
// buckets are sub-sampled to a fixed size; here the kept set is the R ids of
// smallest priority, which does not depend on insertion order).
//
// One wave streams the ids of one bucket (or one chunk of a heavy bucket)
// through a sorted list of at most R (priority, id) keys held in LDS.  An id
// can only enter when its key is below the current R-th key; entrants gather
// in a 64-slot buffer that is sorted across the wave (bitonic, shuffles) and
// merged into the list (each element's new position = its own index + the
// number of smaller elements in the other sorted list, found by binary
// search).  Work is bounded per wave, so skewed buckets split into chunks
// whose partial bottom-R lists are reduced again.
#include "merge16.h"
#include "slash_internal.h"

namespace slash {

namespace {

constexpr int kSelWaves = 4;
constexpr uint32_t kNoKey = 0xFFFFFFFFu;  // filler above every priority but the largest, which ties

// A wave's bottom-R list of priorities (distinct within a table; the id of a
// priority is recovered by the inverse bijection when the list is written).
struct WaveList {
  uint32_t* a;    // current list [R], ascending
  uint32_t* b;    // merge target [R]
  uint32_t* buf;  // pending entrants [64]
  uint32_t cnt;   // live entries of a (uniform)
  uint32_t nbuf;  // live entries of buf (uniform)
  uint32_t R;
};

// Ascending bitonic sort of one 32-bit key per lane across the wave.
__device__ __forceinline__ uint32_t wave_sort32(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int k = 2; k <= SL_WAVE; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t y = (uint32_t)__shfl_xor((int)x, j, SL_WAVE);
      const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
      x = keep_min ? min(x, y) : max(x, y);
    }
  }
  return x;
}

// Inverse of an odd number modulo 2^32 (Newton's iteration; m * m = 1 mod 8
// gives 3 correct bits, each step doubles them).
__device__ __forceinline__ uint32_t inv_odd(uint32_t m) {
  uint32_t v = m;
#pragma unroll
  for (int i = 0; i < 4; ++i) v *= 2u - m * v;
  return v;
}

// The id whose priority (the bijection `priority`) is p; im1 and im2 are the
// inverses of m1 and m2.  Each step of the priority undone in reverse order.
__device__ __forceinline__ uint32_t priority_inverse(uint32_t p, uint32_t key, uint32_t im1, uint32_t im2) {
  uint32_t x = p ^ (p >> 15) ^ (p >> 30);
  x *= im2;
  x ^= x >> 16;
  x *= im1;
  return x ^ key;
}

// Number of entries of sorted arr[0..n) below x.
__device__ __forceinline__ uint32_t lower_bound32(const uint32_t* arr, uint32_t n, uint32_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (arr[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void wl_flush(WaveList& w) {
  if (w.nbuf == 0) return;
  const uint32_t lane = lane_id();
  uint32_t x = lane < w.nbuf ? w.buf[lane] : kNoKey;
  wave_sync();
  x = wave_sort32(x);
  w.buf[lane] = x;
  wave_sync();
  // new position of each pending key
  if (lane < w.nbuf) {
    uint32_t pos = lane + lower_bound32(w.a, w.cnt, x);
    if (pos < w.R) w.b[pos] = x;
  }
  // new position of each listed key
  for (uint32_t i = lane; i < w.cnt; i += SL_WAVE) {
    uint32_t y = w.a[i];
    uint32_t pos = i + lower_bound32(w.buf, w.nbuf, y);
    if (pos < w.R) w.b[pos] = y;
  }
  wave_sync();
  uint32_t* t = w.a;
  w.a = w.b;
  w.b = t;
  w.cnt = min(w.R, w.cnt + w.nbuf);
  w.nbuf = 0;
}

// Offer one key per lane (valid lanes only).
__device__ __forceinline__ void wl_offer(WaveList& w, bool valid, uint32_t key) {
  uint32_t thr = w.cnt < w.R ? kNoKey : w.a[w.R - 1];
  bool pass = valid && (w.cnt < w.R || key < thr);
  uint64_t m = ballot64(pass);
  uint32_t np = (uint32_t)__builtin_popcountll(m);
  if (np == 0) return;
  if (w.nbuf + np > SL_WAVE) wl_flush(w);
  if (pass) w.buf[w.nbuf + (uint32_t)__builtin_popcountll(m & lanemask_lt())] = key;
  wave_sync();
  w.nbuf += np;
}

// Stream ids src[off .. off+len) (EMPTY entries skipped) through the list.
// Four 64-id chunks are loaded before any is offered, so a bucket of up to
// 256 ids costs one memory round trip.
__device__ __forceinline__ void wl_stream(WaveList& w, const uint32_t* __restrict__ src, uint64_t off, uint64_t len,
                                          uint32_t key, uint32_t m1, uint32_t m2) {
  constexpr int kChunks = 4;
  const uint32_t lane = lane_id();
  for (uint64_t i = 0; i < len; i += kChunks * SL_WAVE) {
    uint32_t id[kChunks];
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const uint64_t j = i + (uint64_t)c * SL_WAVE + lane;
      id[c] = j < len ? src[off + j] : SL_EMPTY;
    }
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      if (i + (uint64_t)c * SL_WAVE >= len) break;  // wave-uniform
      const bool v = id[c] != SL_EMPTY;
      wl_offer(w, v, v ? priority(id[c], key, m1, m2) : kNoKey);
    }
  }
  wl_flush(w);
}

// Write the list's ids (im1, im2: inverses of the table's m1, m2).
__device__ __forceinline__ void wl_write(const WaveList& w, uint32_t* __restrict__ out, uint32_t R, uint32_t key,
                                         uint32_t im1, uint32_t im2) {
  for (uint32_t i = lane_id(); i < R; i += SL_WAVE)
    out[i] = i < w.cnt ? priority_inverse(w.a[i], key, im1, im2) : SL_EMPTY;
}

__device__ __forceinline__ WaveList wl_init(uint32_t* lds, uint32_t R) {
  WaveList w;
  w.a = lds;
  w.b = lds + R;
  w.buf = lds + 2 * R;
  w.cnt = 0;
  w.nbuf = 0;
  w.R = R;
  return w;
}

// Per-wave LDS (u32 words): the list, its merge target and the entrant
// buffer; at least 256 words, which the small-bucket select uses as a
// 256-bin histogram; a multiple of 4 so that every wave's region is 16-byte
// aligned.
__host__ __device__ constexpr uint32_t wl_words(uint32_t R) {
  return ((2 * R + SL_WAVE > 256 ? 2 * R + SL_WAVE : 256) + 3) & ~3u;
}

// Bottom-R of a bucket of at most 64·kC ids (R <= 64), all held in registers:
// an MSD radix select over 8-bit digits of the priority finds the R-th
// smallest priority (priorities of one table are distinct), the R kept
// priorities are compacted into LDS and sorted across the wave once, and each
// id is recovered from its priority by the inverse bijection (im1, im2: the
// inverses of m1, m2).  Writes R slots of out (EMPTY past the bucket's size).
template <int kC>
__device__ __forceinline__ void select_small(uint32_t* lds, const uint32_t* __restrict__ src, uint64_t off,
                                             uint32_t n, uint32_t R, uint32_t key, uint32_t m1, uint32_t m2,
                                             uint32_t im1, uint32_t im2, uint32_t* __restrict__ out) {
  const uint32_t lane = lane_id();
  uint32_t id[kC];
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    const uint32_t j = c * SL_WAVE + lane;
    id[c] = j < n ? src[off + j] : SL_EMPTY;
  }
  uint32_t pr[kC];
#pragma unroll
  for (int c = 0; c < kC; ++c) pr[c] = id[c] != SL_EMPTY ? priority(id[c], key, m1, m2) : 0u;
  // upper bound (inclusive) of the kept priorities
  uint32_t upper = 0xFFFFFFFFu;
  if (n > R) {
    uint32_t* hist = lds;
    uint32_t need = R, prefix = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
      const uint32_t hi_mask = shift == 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
      typedef uint32_t v4u __attribute__((ext_vector_type(4)));
      v4u* hv = (v4u*)hist;  // lane owns digits 4*lane .. 4*lane+3 as one vector
      hv[lane] = (v4u)(0u);
      wave_sync();
#pragma unroll
      for (int c = 0; c < kC; ++c)
        if (id[c] != SL_EMPTY && (pr[c] & hi_mask) == prefix) atomicAdd(&hist[(pr[c] >> shift) & 255u], 1u);
      wave_sync();
      // lane owns digits 4*lane .. 4*lane+3
      const v4u hl = hv[lane];
      const uint32_t h[4] = {hl.x, hl.y, hl.z, hl.w};
      const uint32_t mine = h[0] + h[1] + h[2] + h[3];
      uint32_t inc = mine;
#pragma unroll
      for (int o = 1; o < SL_WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, SL_WAVE);
        if (lane >= (uint32_t)o) inc += y;
      }
      uint32_t cum = inc - mine, digit = 0, below = 0, cnt = 0;
      bool here = false;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (cum < need && need <= cum + h[c]) {
          here = true;
          digit = 4 * lane + c;
          below = cum;
          cnt = h[c];
        }
        cum += h[c];
      }
      const uint32_t src_lane = (uint32_t)__builtin_ctzll(ballot64(here));
      digit = __shfl(digit, src_lane, SL_WAVE);
      below = __shfl(below, src_lane, SL_WAVE);
      cnt = __shfl(cnt, src_lane, SL_WAVE);
      wave_sync();
      need -= below;
      prefix |= digit << shift;
      if (need == cnt) {  // the whole digit bin is kept
        upper = prefix | (shift ? (1u << shift) - 1u : 0u);
        break;
      }
    }
  }
  // compact the kept priorities (exactly min(n, R)) and sort them once; the
  // filler 0xFFFFFFFF may equal a kept priority, which changes nothing since
  // the first `base` sorted values are the kept ones either way.  With one id
  // per lane the kept priorities are sorted where they are.
  uint32_t base = 0;
  uint32_t x;
  if constexpr (kC == 1) {
    const bool keep = id[0] != SL_EMPTY && pr[0] <= upper;
    base = (uint32_t)__builtin_popcountll(ballot64(keep));
    x = keep ? pr[0] : 0xFFFFFFFFu;
  } else {
    uint32_t* kept = lds;
#pragma unroll
    for (int c = 0; c < kC; ++c) {
      const bool keep = id[c] != SL_EMPTY && pr[c] <= upper;
      const uint64_t m = ballot64(keep);
      const uint32_t pos = base + (uint32_t)__builtin_popcountll(m & lanemask_lt());
      if (keep && pos < SL_WAVE) kept[pos] = pr[c];
      base += (uint32_t)__builtin_popcountll(m);
    }
    wave_sync();
    x = lane < min(base, (uint32_t)SL_WAVE) ? kept[lane] : 0xFFFFFFFFu;
  }
  x = wave_sort32(x);
  if (lane < R) out[lane] = lane < base ? priority_inverse(x, key, im1, im2) : SL_EMPTY;
  wave_sync();
}

// 8 waves per SIMD (64 VGPRs): the wave-per-bucket loop is latency-bound
__global__ void __launch_bounds__(kSelWaves * SL_WAVE, 8)
    k_select_light(Shape s, ConstView c, uint32_t t, const uint32_t* __restrict__ svals,
                   const uint32_t* __restrict__ start, const uint32_t* __restrict__ end, TablesView tab,
                   uint32_t heavy_t, uint32_t* heavy_list, uint32_t* heavy_n) {
  extern __shared__ uint32_t lds32[];
  const uint32_t wave = threadIdx.x / SL_WAVE, lane = lane_id();
  uint32_t* my = lds32 + wave * wl_words(s.R);
  const uint32_t key = c.key_t[t], m1 = c.m1_t[t], m2 = c.m2_t[t];
  const uint32_t im1 = inv_odd(m1), im2 = inv_odd(m2);
  const uint32_t nwaves = gridDim.x * kSelWaves;
  // the bounds of the wave's next bucket are loaded while this one is reduced
  uint32_t b = blockIdx.x * kSelWaves + wave;
  uint32_t s_next = 0, e_next = 0;
  if (b < s.nb) bucket_run(start, end, b, s_next, e_next);
  for (; b < s.nb; b += nwaves) {
    const uint32_t s0 = s_next, e0 = e_next;
    if (b + nwaves < s.nb) bucket_run(start, end, b + nwaves, s_next, e_next);
    const uint32_t n = e0 - s0;
    uint32_t* out = tab.ids + ((uint64_t)t * s.nb + b) * s.R;
    if (n <= 8 * SL_WAVE && s.R <= SL_WAVE) {
      // as many ids per lane as the bucket needs (most buckets hold at most
      // two per lane)
      if (n <= SL_WAVE)
        select_small<1>(my, svals, s0, n, s.R, key, m1, m2, im1, im2, out);
      else if (n <= 2 * SL_WAVE)
        select_small<2>(my, svals, s0, n, s.R, key, m1, m2, im1, im2, out);
      else if (n <= 4 * SL_WAVE)
        select_small<4>(my, svals, s0, n, s.R, key, m1, m2, im1, im2, out);
      else
        select_small<8>(my, svals, s0, n, s.R, key, m1, m2, im1, im2, out);
      if (lane == 0) tab.seen[(uint64_t)t * s.nb + b] = n;
      continue;
    }
    if (n > heavy_t) {
      if (lane == 0) {
        uint32_t slot = atomicAdd(heavy_n, 1u);
        heavy_list[3 * slot] = b;
        heavy_list[3 * slot + 1] = s0;
        heavy_list[3 * slot + 2] = n;
      }
      continue;
    }
    WaveList w = wl_init(my, s.R);
    wl_stream(w, svals, s0, n, key, m1, m2);
    wl_write(w, out, s.R, key, im1, im2);
    if (lane == 0) tab.seen[(uint64_t)t * s.nb + b] = n;
    wave_sync();
  }
}

// Heavy buckets planned on the device (no host round trip): one block turns
// the heavy list written by k_select_light into chunk work (kHeavy ids per
// chunk, each reduced to a bottom-R list in its own candidate slot) and one
// final item per bucket (its chunks' candidate lists, merged by one wave).
__global__ void __launch_bounds__(256)
    k_heavy_plan(const uint32_t* __restrict__ heavy_list, const uint32_t* __restrict__ heavy_n, uint32_t R,
                 uint32_t chunk_len, ChunkWork* __restrict__ chunks, FinalWork* __restrict__ finals,
                 uint32_t* __restrict__ n_chunks) {
  __shared__ uint32_t part[4];
  __shared__ uint32_t carry_sh;
  // the 256 buckets of one round: first chunk, source offset and length
  __shared__ uint32_t b_first[256], b_off[256], b_len[256];
  const uint32_t nh = *heavy_n, tid = threadIdx.x, lane = lane_id(), wave = tid / SL_WAVE;
  if (tid == 0) carry_sh = 0;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < nh; b0 += 256) {
    const uint32_t i = b0 + tid;
    uint32_t bucket = 0, off = 0, len = 0, nch = 0;
    if (i < nh) {
      bucket = heavy_list[3 * i];
      off = heavy_list[3 * i + 1];
      len = heavy_list[3 * i + 2];
      nch = (len + chunk_len - 1) / chunk_len;
    }
    uint32_t inc = nch;
    for (int o = 1; o < SL_WAVE; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, SL_WAVE);
      if (lane >= (uint32_t)o) inc += y;
    }
    if (lane == SL_WAVE - 1) part[wave] = inc;
    __syncthreads();
    const uint32_t carry = carry_sh;
    uint32_t before = carry;
    for (uint32_t w = 0; w < wave; ++w) before += part[w];
    const uint32_t first = before + inc - nch;
    b_first[tid] = first;
    b_off[tid] = off;
    b_len[tid] = len;
    if (i < nh) finals[i] = FinalWork{(uint64_t)first * R, nch * R, bucket, len, 0};
    __syncthreads();
    // the round's chunks, spread over the block: chunk j belongs to the last
    // bucket whose first chunk is at most j (buckets without chunks share
    // their successor's first and are skipped by the search)
    const uint32_t total = b_first[255] + (b0 + 255 < nh ? (b_len[255] + chunk_len - 1) / chunk_len : 0u);
    for (uint32_t j = carry + tid; j < total; j += 256) {
      uint32_t lo = 0, hi = 255;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) / 2;
        if (b_first[mid] <= j) lo = mid; else hi = mid - 1;
      }
      const uint32_t o = (j - b_first[lo]) * chunk_len;
      chunks[j] = ChunkWork{(uint64_t)b_off[lo] + o, min(chunk_len, b_len[lo] - o), j};
    }
    __syncthreads();
    if (tid == 0) carry_sh = total;
    __syncthreads();
  }
  if (tid == 0) *n_chunks = carry_sh;
}

// Chunk and final reductions of the heavy buckets (work counts read on the device).
__global__ void __launch_bounds__(kSelWaves * SL_WAVE)
    k_select_chunks(Shape s, ConstView c, uint32_t t, const uint32_t* __restrict__ src,
                        const ChunkWork* __restrict__ work, const uint32_t* __restrict__ n_work,
                        uint32_t* __restrict__ dst) {
  extern __shared__ uint32_t lds32[];
  const uint32_t wave = threadIdx.x / SL_WAVE;
  uint32_t* my = lds32 + wave * wl_words(s.R);
  const uint32_t key = c.key_t[t], m1 = c.m1_t[t], m2 = c.m2_t[t];
  const uint32_t im1 = inv_odd(m1), im2 = inv_odd(m2);
  const uint32_t nw = *n_work;
  for (uint32_t wi = blockIdx.x * kSelWaves + wave; wi < nw; wi += gridDim.x * kSelWaves) {
    ChunkWork cw = work[wi];
    WaveList w = wl_init(my, s.R);
    wl_stream(w, src, cw.off, cw.len, key, m1, m2);
    wl_write(w, dst + (uint64_t)cw.dst * s.R, s.R, key, im1, im2);
    wave_sync();
  }
}

// One work-group per heavy bucket: each wave reduces a contiguous quarter of
// the bucket's chunk candidates to a bottom-R list, then wave 0 merges the
// other waves' lists into its own and writes the reservoir.
__global__ void __launch_bounds__(kSelWaves * SL_WAVE)
    k_select_final(Shape s, ConstView c, uint32_t t, const uint32_t* __restrict__ src,
                   const FinalWork* __restrict__ work, const uint32_t* __restrict__ n_work, TablesView tab) {
  extern __shared__ uint32_t lds32[];
  const uint32_t wave = threadIdx.x / SL_WAVE, lane = lane_id();
  uint32_t* my = lds32 + wave * wl_words(s.R);
  uint32_t* lists = lds32 + kSelWaves * wl_words(s.R);  // [kSelWaves][R] priorities
  uint32_t* counts = lists + kSelWaves * s.R;           // [kSelWaves]
  const uint32_t key = c.key_t[t], m1 = c.m1_t[t], m2 = c.m2_t[t];
  const uint32_t im1 = inv_odd(m1), im2 = inv_odd(m2);
  const uint32_t nw = *n_work;
  for (uint32_t wi = blockIdx.x; wi < nw; wi += gridDim.x) {
    const FinalWork fw = work[wi];
    const uint32_t q = ((fw.len + kSelWaves - 1) / kSelWaves + SL_WAVE - 1) / SL_WAVE * SL_WAVE;
    const uint32_t lo = min(fw.len, wave * q), hi = min(fw.len, lo + q);
    WaveList w = wl_init(my, s.R);
    wl_stream(w, src, fw.off + lo, hi - lo, key, m1, m2);
    for (uint32_t i = lane; i < s.R; i += SL_WAVE) lists[wave * s.R + i] = i < w.cnt ? w.a[i] : kNoKey;
    if (lane == 0) counts[wave] = w.cnt;
    __syncthreads();
    if (wave == 0) {
      for (uint32_t o = 1; o < kSelWaves; ++o) {
        const uint32_t n_o = counts[o];
        for (uint32_t i = 0; i < n_o; i += SL_WAVE) {
          const bool v = i + lane < n_o;
          wl_offer(w, v, v ? lists[o * s.R + i + lane] : kNoKey);
        }
      }
      wl_flush(w);
      wl_write(w, tab.ids + ((uint64_t)t * s.nb + fw.bucket) * s.R, s.R, key, im1, im2);
      if (lane == 0) tab.seen[(uint64_t)t * s.nb + fw.bucket] = fw.seen;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- insert

__global__ void k_head_flags(const uint32_t* __restrict__ sk, uint64_t n, uint32_t* __restrict__ flag) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    flag[i] = (i == 0 || sk[i - 1] != sk[i]) ? 1u : 0u;
}

// After the exclusive scan, flag[i] is the segment number of a head i.
__global__ void k_head_scatter(const uint32_t* __restrict__ sk, uint64_t n, const uint32_t* __restrict__ segno,
                               uint32_t* __restrict__ seg_start, uint32_t* __restrict__ nseg) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    bool head = i == 0 || sk[i - 1] != sk[i];
    if (head) seg_start[segno[i]] = (uint32_t)i;
    if (i + 1 == n) *nseg = segno[i] + (head ? 1u : 0u);
  }
}

// One wave per touched (table, bucket): seed the list with the current
// reservoir (already in ascending priority), stream the new ids, write back.
__global__ void __launch_bounds__(kSelWaves * SL_WAVE)
    k_insert_merge(Shape s, ConstView c, const uint32_t* __restrict__ sk, const uint32_t* __restrict__ sv,
                   uint64_t n, const uint32_t* __restrict__ seg_start, const uint32_t* __restrict__ nseg,
                   TablesView tab) {
  extern __shared__ uint32_t lds32[];
  const uint32_t wave = threadIdx.x / SL_WAVE, lane = lane_id();
  uint32_t* my = lds32 + wave * wl_words(s.R);
  const uint32_t ns = *nseg;
  for (uint32_t g = blockIdx.x * kSelWaves + wave; g < ns; g += gridDim.x * kSelWaves) {
    const uint32_t s0 = seg_start[g];
    const uint32_t e0 = g + 1 < ns ? seg_start[g + 1] : (uint32_t)n;
    const uint32_t ck = sk[s0];
    const uint32_t t = ck >> s.B, b = ck & (s.nb - 1);
    const uint32_t key = c.key_t[t], m1 = c.m1_t[t], m2 = c.m2_t[t];
    uint32_t* res = tab.ids + ((uint64_t)t * s.nb + b) * s.R;
    uint32_t* seen = tab.seen + (uint64_t)t * s.nb + b;
    WaveList w = wl_init(my, s.R);
    const uint32_t old = *seen;
    const uint32_t fill = min(old, s.R);
    for (uint32_t i = lane; i < fill; i += SL_WAVE) w.a[i] = priority(res[i], key, m1, m2);
    w.cnt = fill;
    wave_sync();
    wl_stream(w, sv, s0, e0 - s0, key, m1, m2);
    wl_write(w, res, s.R, key, inv_odd(m1), inv_odd(m2));
    if (lane == 0) *seen = old + (e0 - s0);
    wave_sync();
  }
}

// Small insert batches (n <= kSmallInsert rows), two kernels after hashing:
// k_insert_group - one block per table groups the table's n new (bucket, id)
//   pairs by bucket in an LDS open-addressing table, then writes one run
//   record (bucket, first item, length) per distinct bucket, the ids of each
//   run contiguously, and zero-length records up to n;
// k_insert_merge16 - sixteen lanes per run record, over the whole GPU: the
//   group holds the bucket's reservoir in registers (E entries per lane, in
//   ascending priority) and inserts each new id whose priority is below the
//   current R-th one at its rank (group sum of per-lane counts, one shift).
// The bottom-R set does not depend on the order in which ids arrive, so the
// grouping order is free.
constexpr uint32_t kSmallInsert = 4096;
constexpr uint32_t kGroupThreads = 1024;
constexpr uint32_t kGroupItems = kSmallInsert / kGroupThreads;  // items per thread
constexpr uint32_t kMergeThreads = 256;

__host__ __device__ inline uint32_t group_cap_log2(uint32_t n) {
  uint32_t c = 6;  // at least 64 slots, at most half full
  while ((1u << c) < 2 * n) ++c;
  return c;
}

// Block-wide exclusive scan of one value per thread (kGroupThreads threads);
// returns the prefix and writes the total to *total.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const uint32_t lane = lane_id(), wave = threadIdx.x / SL_WAVE;
  constexpr uint32_t NW = kGroupThreads / SL_WAVE;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < SL_WAVE; o <<= 1) {
    uint32_t y = __shfl_up(x, o, SL_WAVE);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == SL_WAVE - 1) wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {
    uint32_t w = lane < NW ? wsum[lane] : 0u;
#pragma unroll
    for (int o = 1; o < (int)NW; o <<= 1) {
      uint32_t y = __shfl_up(w, o, SL_WAVE);
      if (lane >= (uint32_t)o) w += y;
    }
    if (lane < NW) wsum[lane] = w;  // inclusive
  }
  __syncthreads();
  uint32_t before = wave ? wsum[wave - 1] : 0u;
  *total = wsum[NW - 1];
  return before + x - v;
}

__global__ void __launch_bounds__(kGroupThreads)
    k_insert_group(const uint32_t* __restrict__ keys, uint32_t n, uint32_t first_id, uint2* __restrict__ recs,
                   uint32_t* __restrict__ items, GroupSignal sig) {
  extern __shared__ uint32_t lds32[];
  const uint32_t t = blockIdx.x, tid = threadIdx.x;
  const uint32_t cl = group_cap_log2(n), cap = 1u << cl;
  uint32_t* slot_key = lds32;          // [cap] bucket or EMPTY
  uint32_t* slot_cnt = lds32 + cap;    // [cap] ids in the run, then its first item
  uint32_t* wsum = lds32 + 2 * cap;    // [kGroupThreads / SL_WAVE]
  for (uint32_t i = tid; i < cap; i += kGroupThreads) {
    slot_key[i] = 0xFFFFFFFFu;
    slot_cnt[i] = 0;
  }
  uint32_t key[kGroupItems];
#pragma unroll
  for (uint32_t j = 0; j < kGroupItems; ++j) {
    uint32_t i = tid + j * kGroupThreads;
    key[j] = i < n ? keys[(uint64_t)t * n + i] : 0u;
  }
  __syncthreads();
  uint32_t slot[kGroupItems], rank[kGroupItems];
#pragma unroll
  for (uint32_t j = 0; j < kGroupItems; ++j) {
    uint32_t i = tid + j * kGroupThreads;
    if (i < n) {
      // linear probing from a multiplicative hash of the bucket id; the table
      // is at most half full, so a free or matching slot is always found
      uint32_t h = (key[j] * 0x9E3779B1u) >> (32 - cl);
      for (;;) {
        uint32_t prev = atomicCAS(&slot_key[h], 0xFFFFFFFFu, key[j]);
        if (prev == 0xFFFFFFFFu || prev == key[j]) break;
        h = (h + 1) & (cap - 1);
      }
      slot[j] = h;
      rank[j] = atomicAdd(&slot_cnt[h], 1u);
    }
  }
  __syncthreads();
  // number the runs and place their ids: each thread owns a slice of slots
  const uint32_t per = (cap + kGroupThreads - 1) / kGroupThreads;
  const uint32_t s0 = min(cap, tid * per), s1 = min(cap, s0 + per);
  uint32_t nrun = 0, nitem = 0;
  for (uint32_t h = s0; h < s1; ++h) {
    uint32_t c = slot_cnt[h];
    nrun += c ? 1u : 0u;
    nitem += c;
  }
  uint32_t tot;
  // both counts are <= 4096: scan them packed in one word
  uint32_t pre = block_scan_excl((nrun << 16) | nitem, wsum, &tot);
  uint32_t r = pre >> 16, o = pre & 0xFFFFu;
  uint2* rec = recs + (uint64_t)t * n;
  for (uint32_t h = s0; h < s1; ++h) {
    uint32_t c = slot_cnt[h];
    if (c) {
      rec[r++] = make_uint2(slot_key[h], o | (c << 16));
      slot_cnt[h] = o;
      o += c;
    }
  }
  for (uint32_t i = (tot >> 16) + tid; i < n; i += kGroupThreads) rec[i] = make_uint2(0u, 0u);
  __syncthreads();
  uint32_t* it = items + (uint64_t)t * n;
#pragma unroll
  for (uint32_t j = 0; j < kGroupItems; ++j) {
    uint32_t i = tid + j * kGroupThreads;
    if (i < n) it[slot_cnt[slot[j]] + rank[j]] = first_id + i;
  }
  if (sig.flag) {
    // the block's writes reach L2 at the barrier; the fence makes them
    // visible device-wide before the block counts itself done; the last
    // block resets the counter and sets the host-visible word
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      if (atomicAdd(sig.counter, 1u) == gridDim.x - 1) {
        *sig.counter = 0;
        __threadfence_system();
        *(volatile uint64_t*)sig.flag = sig.value;
      }
    }
  }
}

template <int E>
__global__ void __launch_bounds__(kMergeThreads)
    k_insert_merge16(Shape s, ConstView c, const uint2* __restrict__ recs, const uint32_t* __restrict__ items,
                     uint32_t n, TablesView tab) {
  const uint64_t run = ((uint64_t)blockIdx.x * kMergeThreads + threadIdx.x) >> 4;
  // both conditions are uniform over the sixteen lanes of a group
  if (run >= (uint64_t)s.L * n) return;
  const uint2 rec = recs[run];
  if ((rec.y >> 16) == 0) return;
  const uint32_t t = (uint32_t)(run / n);
  merge_run16<E>(s, c, rec, t, items + (uint64_t)t * n, tab);
}

uint32_t grid_for(uint64_t work, uint32_t per_block, uint32_t cap) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

}  // namespace

hipError_t launch_select_light(const Shape& s, const ConstView& c, uint32_t t, const uint32_t* svals,
                               const uint32_t* start, const uint32_t* end, TablesView tab, uint32_t heavy_t,
                               uint32_t* heavy_list, uint32_t* heavy_n, hipStream_t st) {
  size_t lds = (size_t)kSelWaves * wl_words(s.R) * 4;
  hipLaunchKernelGGL(k_select_light, dim3(grid_for(s.nb, kSelWaves, 16384)), dim3(kSelWaves * SL_WAVE), lds, st,
                     s, c, t, svals, start, end, tab, heavy_t, heavy_list, heavy_n);
  return hipGetLastError();
}

size_t heavy_chunk_capacity(uint64_t n, uint32_t chunk_len) { return (size_t)(2 * (n / chunk_len) + 2); }

hipError_t launch_heavy(const Shape& s, const ConstView& c, uint32_t t, const uint32_t* svals, uint64_t n,
                        const uint32_t* heavy_list, const uint32_t* heavy_n, uint32_t chunk_len, ChunkWork* chunks,
                        FinalWork* finals, uint32_t* n_chunks, uint32_t* cand, TablesView tab, hipStream_t st) {
  hipLaunchKernelGGL(k_heavy_plan, dim3(1), dim3(256), 0, st, heavy_list, heavy_n, s.R, chunk_len, chunks, finals,
                     n_chunks);
  const size_t lds = (size_t)kSelWaves * wl_words(s.R) * 4;
  const uint32_t max_chunks = (uint32_t)heavy_chunk_capacity(n, chunk_len);
  hipLaunchKernelGGL(k_select_chunks, dim3(grid_for(max_chunks, kSelWaves, 4096)), dim3(kSelWaves * SL_WAVE), lds,
                     st, s, c, t, svals, chunks, n_chunks, cand);
  const uint32_t max_heavy = (uint32_t)(n / chunk_len + 1);
  const size_t lds_f = lds + (size_t)kSelWaves * s.R * 4 + kSelWaves * 4;
  hipLaunchKernelGGL(k_select_final, dim3(max_heavy < 1024 ? max_heavy : 1024), dim3(kSelWaves * SL_WAVE), lds_f, st,
                     s, c, t, cand, finals, heavy_n, tab);
  return hipGetLastError();
}

bool small_insert_ok(const Shape& s, uint64_t n) { return n >= 1 && n <= kSmallInsert; }

// run records [L][n] (uint2) then run ids [L][n]
size_t small_insert_scratch(const Shape& s, uint64_t n) { return (size_t)s.L * n * 12 + 64; }

hipError_t launch_insert_group(const Shape& s, const uint32_t* keys, uint32_t n, uint32_t first_id, void* scratch,
                               hipStream_t st, const GroupSignal& sig) {
  if (n == 0 || n > kSmallInsert) return hipErrorInvalidValue;
  uint2* recs = (uint2*)scratch;
  uint32_t* items = (uint32_t*)(recs + (size_t)s.L * n);
  const size_t lds = ((size_t)2 << group_cap_log2(n)) * 4 + (kGroupThreads / SL_WAVE) * 4;
  hipError_t e;
  if (lds > 65536 &&
      (e = hipFuncSetAttribute((const void*)k_insert_group, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
          hipSuccess)
    return e;
  hipLaunchKernelGGL(k_insert_group, dim3(s.L), dim3(kGroupThreads), lds, st, keys, n, first_id, recs, items, sig);
  return hipGetLastError();
}

bool insert_run_arrays(const Shape& s, void* scratch, uint32_t n, const uint2** recs, const uint32_t** items) {
  if (n == 0 || n > kSmallInsert || !scratch) return false;
  *recs = (const uint2*)scratch;
  *items = (const uint32_t*)(*recs + (size_t)s.L * n);
  return true;
}

hipError_t launch_insert_runs(const Shape& s, const ConstView& c, void* scratch, uint32_t n, TablesView tab,
                              hipStream_t st) {
  if (n == 0 || n > kSmallInsert) return hipErrorInvalidValue;
  uint2* recs = (uint2*)scratch;
  uint32_t* items = (uint32_t*)(recs + (size_t)s.L * n);
  if (s.bucket) return launch_tk_runs(s, c, recs, items, n, tab, st);
  const uint64_t lanes = (uint64_t)s.L * n * 16;
  const dim3 grid((uint32_t)((lanes + kMergeThreads - 1) / kMergeThreads));
  if (s.R <= 16)
    hipLaunchKernelGGL(k_insert_merge16<1>, grid, dim3(kMergeThreads), 0, st, s, c, recs, items, n, tab);
  else if (s.R <= 32)
    hipLaunchKernelGGL(k_insert_merge16<2>, grid, dim3(kMergeThreads), 0, st, s, c, recs, items, n, tab);
  else if (s.R <= 64)
    hipLaunchKernelGGL(k_insert_merge16<4>, grid, dim3(kMergeThreads), 0, st, s, c, recs, items, n, tab);
  else if (s.R <= 128)
    hipLaunchKernelGGL(k_insert_merge16<8>, grid, dim3(kMergeThreads), 0, st, s, c, recs, items, n, tab);
  else
    hipLaunchKernelGGL(k_insert_merge16<16>, grid, dim3(kMergeThreads), 0, st, s, c, recs, items, n, tab);
  return hipGetLastError();
}

hipError_t launch_insert_small(const Shape& s, const ConstView& c, const uint32_t* keys, uint32_t n, uint32_t first_id,
                               void* scratch, TablesView tab, hipStream_t st) {
  hipError_t e = launch_insert_group(s, keys, n, first_id, scratch, st);
  return e == hipSuccess ? launch_insert_runs(s, c, scratch, n, tab, st) : e;
}

hipError_t launch_insert_merge(const Shape& s, const ConstView& c, const uint32_t* skeys, const uint32_t* svals,
                               uint64_t n, uint32_t* seg_scratch, uint32_t* part, TablesView tab, hipStream_t st) {
  if (n == 0) return hipSuccess;
  // seg_scratch: [0, n) flags -> segment numbers, [n, 2n) starts, [2n] count
  uint32_t* segno = seg_scratch;
  uint32_t* seg_start = seg_scratch + n;
  uint32_t* nseg = seg_scratch + 2 * n;
  hipLaunchKernelGGL(k_head_flags, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, skeys, n, segno);
  hipError_t e = exclusive_scan(segno, n, part, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_head_scatter, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, skeys, n, segno, seg_start,
                     nseg);
  if (s.bucket) return launch_tk_segments(s, c, skeys, svals, n, seg_start, nseg, tab, st);
  size_t lds = (size_t)kSelWaves * wl_words(s.R) * 4;
  hipLaunchKernelGGL(k_insert_merge, dim3(grid_for(n, kSelWaves, 16384)), dim3(kSelWaves * SL_WAVE), lds, st, s, c,
                     skeys, svals, n, seg_start, nseg, tab);
  return hipGetLastError();
}

}  // namespace slash
