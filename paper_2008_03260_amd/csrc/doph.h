// Wave-level densified one-permutation hashing (Section 2.2) and table
// addresses (Section 2.3), used by the build, insert, hash and query kernels.
#pragma once

#include "slash_internal.h"

namespace slash {

// Loads of hash constants.  With CL = true the pointer is a staged copy in
// LDS and is read with LDS instructions; otherwise from global memory.
typedef __attribute__((address_space(3))) const uint64_t lds_u64;
typedef __attribute__((address_space(3))) const uint32_t lds_u32;

template <bool CL>
__device__ __forceinline__ uint64_t cld64(const uint64_t* p, uint32_t i) {
  if constexpr (CL)
    return ((lds_u64*)p)[i];
  else
    return p[i];
}

template <bool CL>
__device__ __forceinline__ uint32_t cld32(const uint32_t* p, uint32_t i) {
  if constexpr (CL)
    return ((lds_u32*)p)[i];
  else
    return p[i];
}

// Words of the per-row non-empty mask (built 64 bins at a time).
__host__ __device__ constexpr uint32_t mask_words(uint32_t M) { return ((M + 63) / 64) * 2; }

// LDS words one wave needs for doph_wave: minima[M] + densified[M] + mask.
__host__ __device__ constexpr uint32_t doph_lds_words(uint32_t M) { return 2 * M + mask_words(M); }

// Nonzero-hash constant pairs (a_h, b_h): one for the single DOPH pass
// (mode 0), one per table (mode 1), one per MinHash function (mode 2).
__host__ __device__ inline uint32_t n_hash_pairs(const Shape& s) { return s.mode == 2 ? s.M : (s.mode ? s.L : 1u); }

// 32-bit LDS words of the staged hash constants: u64 a_h, b_h, a_tj, b_t,
// a_r, b_r, then the u32 direction words.
__host__ __device__ inline uint32_t const_words(const Shape& s) {
  uint32_t n_h = n_hash_pairs(s);
  return 2 * (2 * n_h + s.M + s.L + 2 * s.d) + (s.M + 31) / 32 + 1;
}

// Largest constant table staged in LDS (larger ones are read from global).
constexpr uint32_t kConstCapWords = 4096;

// Copy the hash constants into LDS at `dst` (8-byte aligned) with all
// `nthreads` threads of the block; returns a view of the staged copy.  The
// caller synchronises the block before use.  The device table is one
// contiguous block in this order (a_h, b_h, a_tj, b_t, a_r, b_r as u64, then
// the u32 direction words), so it is copied as const_words(s) flat words,
// every load of a thread issued before its stores.
__device__ inline ConstView stage_consts(const Shape& s, const ConstView& c, uint32_t* dst, uint32_t nthreads) {
  const uint32_t n_h = n_hash_pairs(s);
  const uint32_t W = const_words(s);
  const uint32_t* src = (const uint32_t*)c.a_h;
  for (uint32_t base = 0; base < W; base += 4 * nthreads) {
    uint32_t x[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      const uint32_t i = base + j * nthreads + threadIdx.x;
      x[j] = i < W ? src[i] : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      const uint32_t i = base + j * nthreads + threadIdx.x;
      if (i < W) dst[i] = x[j];
    }
  }
  ConstView v = c;
  const uint64_t* p = (const uint64_t*)dst;
  v.a_h = p;
  v.b_h = p += n_h;
  v.a_tj = p += n_h;
  v.b_t = p += s.M;
  v.a_r = p += s.L;
  v.b_r = p += s.d;
  v.dirw = (const uint32_t*)(p + s.d);
  return v;
}

// Nearest set bit of `mask` walking right (increasing, circular) from pos
// inside the domain [lo, lo + n).  Callers guarantee a set bit in the domain
// other than pos; the walk is still bounded (one lap over the domain's words)
// and returns pos when nothing is found.
__device__ __forceinline__ uint32_t find_right(const lds_u32* mask, uint32_t lo, uint32_t n, uint32_t pos) {
  const uint32_t end = lo + n;
  uint32_t q = pos + 1 == end ? lo : pos + 1;
  for (uint32_t step = 0; step <= n / 32 + 2; ++step) {
    uint32_t o = q & 31u;
    uint32_t bits = mask[q >> 5] >> o;
    uint32_t span = min(32u - o, end - q);
    if (span < 32u) bits &= (1u << span) - 1u;
    if (bits) return q + (uint32_t)__builtin_ctz(bits);
    q += span;
    if (q >= end) q = lo;
  }
  return pos;
}

// Same, walking left (decreasing, circular).
__device__ __forceinline__ uint32_t find_left(const lds_u32* mask, uint32_t lo, uint32_t n, uint32_t pos) {
  uint32_t q = pos == lo ? lo + n - 1 : pos - 1;
  for (uint32_t step = 0; step <= n / 32 + 2; ++step) {
    uint32_t o = q & 31u;
    uint32_t bits = mask[q >> 5] << (31u - o);
    uint32_t span = min(o + 1u, q - lo + 1u);
    if (span < 32u) bits &= ~((1u << (32u - span)) - 1u);
    if (bits) return q - (uint32_t)__builtin_clz(bits);
    if (span == q - lo + 1u)
      q = lo + n - 1;
    else
      q -= span;
  }
  return pos;
}

__device__ __forceinline__ bool domain_any(const lds_u32* mask, uint32_t lo, uint32_t n) {
  for (uint32_t q = lo; q < lo + n;) {
    uint32_t o = q & 31u;
    uint32_t span = min(32u - o, lo + n - q);
    uint32_t bits = mask[q >> 5] >> o;
    if (span < 32u) bits &= (1u << span) - 1u;
    if (bits) return true;
    q += span;
  }
  return false;
}

// Per-bin minima of one row's nonzero hashes (mode 0): a group of G lanes
// takes 4·G nonzeros per round, loading all of them before hashing any, so a
// row of up to 4·G nonzeros costs one memory round trip.  load_batch loads
// one round; a caller may load the first round early (x0, PRE = true) so that
// its latency overlaps other work.
template <int G>
__device__ __forceinline__ void load_batch(const int32_t* __restrict__ idx, uint32_t e0, uint32_t nnz, uint32_t gl,
                                           uint32_t (&x)[4]) {
#pragma unroll
  for (uint32_t c = 0; c < 4; ++c) {
    const uint32_t e = e0 + c * G + gl;
    x[c] = e < nnz ? (uint32_t)idx[e] : 0u;
  }
}

// With `bad` set, an index outside [0, dim) ORs 2 into *bad (the build checks
// its input while hashing it).
template <int G>
__device__ __forceinline__ void minima_batch(const Shape& s, uint64_t a, uint64_t bb, const uint32_t (&x)[4],
                                             uint32_t e0, uint32_t nnz, uint32_t gl, uint32_t* lds_m,
                                             uint32_t* bad) {
  const uint32_t msh = s.mshift;
  bool out = false;
#pragma unroll
  for (uint32_t c = 0; c < 4; ++c) {
    if (e0 + c * G + gl < nnz) {
      out |= (int32_t)x[c] < 0 || x[c] >= s.dim;
      const uint32_t u = nz_hash(a, bb, x[c]);
      const uint32_t bin = msh == 0xFFu ? range_bin(u, s.M) : (msh ? u >> (32 - msh) : 0u);
      atomicMin(&lds_m[bin], u);
    }
  }
  if (bad && out) atomicOr(bad, 2u);
}

template <int G, bool PRE = false>
__device__ __forceinline__ void row_minima(const Shape& s, uint64_t a, uint64_t bb, const int32_t* __restrict__ idx,
                                           uint32_t nnz, uint32_t gl, uint32_t* lds_m, const uint32_t* x0 = nullptr,
                                           uint32_t* bad = nullptr) {
  uint32_t e0 = 0;
  if constexpr (PRE) {
    const uint32_t x[4] = {x0[0], x0[1], x0[2], x0[3]};
    minima_batch<G>(s, a, bb, x, 0, nnz, gl, lds_m, bad);
    e0 = 4 * G;
  }
  for (; e0 < nnz; e0 += 4 * G) {
    uint32_t x[4];
    load_batch<G>(idx, e0, nnz, gl, x);
    minima_batch<G>(s, a, bb, x, e0, nnz, gl, lds_m, bad);
  }
}

// A group of G consecutive lanes (G = 16, 32 or 64) hashes one row: per-bin
// minima of the nonzero hashes, then densification (an empty bin copies the
// nearest non-empty bin in its fixed direction, circularly, reading the
// pre-densification minima; all-empty domains stay EMPTY).  A wave holds
// 64 / G groups, each with its own row and its own LDS scratch lds_m (see
// doph_lds_words).  Every lane of the wave must call (the synchronisation is
// wave-wide); `idx` points at the group's row of nnz indices.  Returns the
// densified values (lds_m + M, M entries).
template <int G, bool CL>
__device__ __forceinline__ const uint32_t* doph_group(const Shape& s, const ConstView& c,
                                                      const int32_t* __restrict__ idx, uint32_t nnz,
                                                      uint32_t* lds_m) {
  static_assert(G == 16 || G == 32 || G == 64, "group size");
  const uint32_t lane = lane_id();
  const uint32_t gl = lane & (G - 1);
  const uint32_t gshift = lane & ~(uint32_t)(G - 1);
  const uint32_t M = s.M;
  uint32_t* lds_h = lds_m + M;
  uint32_t* mask = lds_m + 2 * M;
  typedef __attribute__((address_space(3))) uint32_t lw32;
  lw32* m3 = (lw32*)lds_m;
  lw32* h3 = (lw32*)lds_h;
  const lds_u32* k3 = (const lds_u32*)mask;
  for (uint32_t b = gl; b < M; b += G) m3[b] = SL_EMPTY;
  // every mask word, including bits past M that no ballot covers
  for (uint32_t w = gl; w < mask_words(M); w += G) mask[w] = 0u;
  wave_sync();
  if (s.mode == 0) {
    row_minima<G>(s, cld64<CL>(c.a_h, 0), cld64<CL>(c.b_h, 0), idx, nnz, gl, lds_m, nullptr, c.bad);
  } else if (s.mode == 2) {
    // classic MinHash: value j is the minimum of u_j over the row; lanes take
    // (function, nonzero) pairs function-major, so a lane keeps its function's
    // constants across consecutive nonzeros
    for (uint32_t w = gl; w < nnz * M; w += G) {
      const uint32_t j = w / nnz, e = w - j * nnz;
      const uint32_t x = (uint32_t)idx[e];
      if (c.bad && ((int32_t)x < 0 || x >= s.dim)) atomicOr(c.bad, 2u);
      atomicMin(&lds_m[j], nz_hash(cld64<CL>(c.a_h, j), cld64<CL>(c.b_h, j), x));
    }
  } else {
    const uint32_t L = s.L, K = s.K;
    for (uint32_t w = gl; w < nnz * L; w += G) {
      uint32_t e = w / L, t = w - e * L;
      const uint32_t x = (uint32_t)idx[e];
      if (c.bad && ((int32_t)x < 0 || x >= s.dim)) atomicOr(c.bad, 2u);
      uint32_t u = nz_hash(cld64<CL>(c.a_h, t), cld64<CL>(c.b_h, t), x);
      atomicMin(&lds_m[t * K + range_bin(u, K)], u);
    }
  }
  wave_sync();
  // non-empty mask, G bins per ballot; any_all: is any bin of the row non-empty
  const uint64_t gmask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1);
  bool any_all = false;
  for (uint32_t base = 0; base < M; base += G) {
    uint32_t b = base + gl;
    bool ne = b < M && m3[b] != SL_EMPTY;
    uint64_t bal = (ballot64(ne) >> gshift) & gmask;
    any_all |= bal != 0ull;
    if (gl == 0) {
      if (G == 64) {
        mask[base / 32] = (uint32_t)bal;
        mask[base / 32 + 1] = (uint32_t)(bal >> 32);
      } else if (G == 32) {
        mask[base / 32] = (uint32_t)bal;
      } else {
        ((uint16_t*)mask)[base / 16] = (uint16_t)bal;
      }
    }
  }
  wave_sync();
  // densify into lds_h, reading only the minima
#pragma unroll 1
  for (uint32_t b = gl; b < M; b += G) {
    uint32_t v = m3[b];
    if (v == SL_EMPTY) {
      // densification domain: every bin (mode 0), the table's K bins (mode
      // 1); a MinHash function (mode 2) is its own domain and stays EMPTY
      uint32_t lo = s.mode == 0 ? 0u : (s.mode == 1 ? (b / s.K) * s.K : b);
      uint32_t n = s.mode == 0 ? M : (s.mode == 1 ? s.K : 1u);
      if (s.mode == 0 ? any_all : domain_any(k3, lo, n)) {
        bool right = (cld32<CL>(c.dirw, b >> 5) >> (b & 31)) & 1u;
        uint32_t src = right ? find_right(k3, lo, n, b) : find_left(k3, lo, n, b);
        v = m3[src];
      }
    }
    h3[b] = v;
  }
  wave_sync();
  return lds_h;
}

// Register form of doph_group for mode 0, for M = G * P with P in {4, 8, 16}
// and K dividing P: lane gl of a group owns the P consecutive bins
// [gl * P, gl * P + P) and with them P / K whole tables.  The minima are taken
// with LDS atomics as in doph_group; densification then runs in registers.
// For each bin the nearest non-empty bin on its right / left is either in
// the lane's own chunk or is the first / last non-empty bin of the nearest
// lane (circularly) whose chunk has one; that lane is found with one ballot
// and its value fetched with one shuffle.  This is the same result as the
// bin-by-bin circular walk over the pre-densification minima (a lane that
// holds the only non-empty bins wraps onto itself).  Returns h, the P
// densified values of the lane's bins.  Every lane of the wave must call;
// lds_m must be 16-byte aligned.
template <int G, int P, bool CL, bool PRE = false>
__device__ __forceinline__ void doph_regs(const Shape& s, const ConstView& c, const int32_t* __restrict__ idx,
                                          uint32_t nnz, uint32_t* lds_m, uint32_t (&h)[P],
                                          const uint32_t* x0 = nullptr) {
  static_assert(P == 4 || P == 8 || P == 16, "bins per lane");
  static_assert(G == 16 || G == 32 || G == 64, "group size");
  const uint32_t lane = lane_id();
  const uint32_t gl = lane & (G - 1);
  const uint32_t gshift = lane & ~(uint32_t)(G - 1);
  const uint32_t b0 = gl * P;
  // the lane's P bins are cleared and read back as 16-byte vectors (lds_m is
  // 16-byte aligned), one LDS instruction per 4 bins
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(3))) v4u lv4u;
  lv4u* m4 = (lv4u*)(lds_m + b0);
#pragma unroll
  for (int q = 0; q < P / 4; ++q) m4[q] = (v4u)(SL_EMPTY);
  wave_sync();
  row_minima<G, PRE>(s, cld64<CL>(c.a_h, 0), cld64<CL>(c.b_h, 0), idx, nnz, gl, lds_m, x0, c.bad);
  wave_sync();
#pragma unroll
  for (int q = 0; q < P / 4; ++q) {
    const v4u t = m4[q];
    h[4 * q] = t.x;
    h[4 * q + 1] = t.y;
    h[4 * q + 2] = t.z;
    h[4 * q + 3] = t.w;
  }
  uint32_t first = SL_EMPTY, last = SL_EMPTY;
#pragma unroll
  for (int j = P - 1; j >= 0; --j)
    if (h[j] != SL_EMPTY) first = h[j];
#pragma unroll
  for (int j = 0; j < P; ++j)
    if (h[j] != SL_EMPTY) last = h[j];
  const uint64_t gmask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1);
  const uint64_t bal = (ballot64(first != SL_EMPTY) >> gshift) & gmask;
  // rotate so that bit i stands for lane (gl + i) mod G
  const uint64_t rot = gl ? (((bal >> gl) | (bal << (G - gl))) & gmask) : bal;
  const uint64_t after = rot & ~1ull;
  const uint32_t up = after ? (gl + (uint32_t)__builtin_ctzll(after)) & (G - 1) : gl;
  const uint32_t down = rot ? (gl + 63u - (uint32_t)__builtin_clzll(rot)) & (G - 1) : gl;
  const uint32_t next_v = (uint32_t)__shfl(first, (int)(gshift + up), SL_WAVE);
  const uint32_t prev_v = (uint32_t)__shfl(last, (int)(gshift + down), SL_WAVE);
  uint32_t r[P];
  uint32_t carry = next_v;
#pragma unroll
  for (int j = P - 1; j >= 0; --j) {
    r[j] = carry;
    if (h[j] != SL_EMPTY) carry = h[j];
  }
  const uint32_t dirs = cld32<CL>(c.dirw, b0 >> 5) >> (b0 & 31);
  carry = prev_v;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const uint32_t v = h[j];
    if (v != SL_EMPTY)
      carry = v;
    else
      h[j] = ((dirs >> j) & 1u) ? r[j] : carry;
  }
}

// Whether doph_regs applies to the shape with G lanes per row.
__host__ __device__ inline uint32_t doph_regs_p(const Shape& s, uint32_t G) {
  if (s.mode != 0 || s.M % G) return 0;
  const uint32_t P = s.M / G;
  if (P != 4 && P != 8 && P != 16) return 0;
  return (s.K <= P && P % s.K == 0) ? P : 0;
}

// Bucket ids of the P / K tables owned by lane gl (doph_regs layout):
// emit(t, bucket) for each, in table order.
template <int P, bool CL, class Emit>
__device__ __forceinline__ void table_buckets_regs(const Shape& s, const ConstView& c, const uint32_t (&h)[P],
                                                   uint32_t gl, Emit emit) {
  const uint32_t b0 = gl * P;
  const uint32_t kmask = s.K - 1, kshift = (uint32_t)__builtin_ctz(s.K);  // K is a power of two here
  uint64_t a[P];
  if constexpr (CL) {
    // the lane's P multipliers as 16-byte LDS vectors (two per vector)
    typedef uint64_t v2u64 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) const v2u64 lv2u64;
    const lv2u64* av = (const lv2u64*)(c.a_tj + b0);
#pragma unroll
    for (int q = 0; q < P / 2; ++q) {
      const v2u64 t = av[q];
      a[2 * q] = t.x;
      a[2 * q + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < P; ++j) a[j] = c.a_tj[b0 + j];
  }
  uint64_t acc = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    acc += a[j] * (uint64_t)h[j];
    if (((j + 1) & kmask) == 0) {
      const uint32_t t = (b0 + j) >> kshift;
      emit(t, (uint32_t)((acc + cld64<CL>(c.b_t, t)) >> (64 - s.B)));
      acc = 0;
    }
  }
}

template <bool CL>
__device__ __forceinline__ const uint32_t* doph_wave(const Shape& s, const ConstView& c,
                                                     const int32_t* __restrict__ idx, uint32_t nnz,
                                                     uint32_t* lds_m) {
  return doph_group<64, CL>(s, c, idx, nnz, lds_m);
}

// Lanes per row for the row-parallel hash kernels.
__host__ __device__ inline uint32_t hash_group(uint32_t M) { return M <= 128 ? 16u : (M <= 512 ? 32u : 64u); }

// Bucket id of table t from densified values h (Section 2.3):
// (b_t + sum_j a_tj * h[tK + j]) >> (64 - B), arithmetic mod 2^64.
template <bool CL>
__device__ __forceinline__ uint32_t table_bucket(const Shape& s, const ConstView& c, const uint32_t* h,
                                                 uint32_t t) {
  uint64_t acc = cld64<CL>(c.b_t, t);
  const uint32_t base = t * s.K;
  const lds_u32* ht = (const lds_u32*)h;
  for (uint32_t j = 0; j < s.K; ++j) acc += cld64<CL>(c.a_tj, base + j) * (uint64_t)ht[base + j];
  return (uint32_t)(acc >> (64 - s.B));
}

}  // namespace slash
