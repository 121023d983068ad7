// Query kernel (Section 2.3 query phase, "Cheap Frequency based Filtering";
// Algorithm 2 on one node; Section 2.4 / Appendix 2 for the count-min style
// frequency sketch whose top-k identities are the answer).
//
// One work-group answers one query at a time:
//   1. wave 0 hashes the query (DOPH) into its L bucket ids;
//   2. every thread gathers reservoir slots (table t, slot j) of the probed
//      buckets straight from HBM (coalesced R-slot rows; EMPTY slots skipped);
//   3. count-min: d rows of w counters in LDS, incremented with LDS atomics;
//      8-bit counters, and a 16-bit recount one row at a time for a query
//      whose counts overflow a byte (a counter never exceeds L * R <= 65535);
//   4. estimate = min over rows; for k <= 16 a lower bound of the k-th
//      largest key (estimate << 32 | ~id) from the waves' lane maxima leaves
//      a few dozen candidates, whose duplicate slots are dropped and which
//      are ranked directly;
//   5. otherwise duplicates of an id are folded by an LDS open-addressing
//      set so each distinct id is ranked once, the k-th largest key is found
//      by an MSD radix select over 8-bit digits, and the winners are ranked
//      by counting.  Results are written with stride k_max, padded with
//      (EMPTY, 0).
// The persistent form loops over queries taken from a device work counter.
#include <array>

#include "doph.h"
#include "merge16.h"

namespace slash {

namespace {

constexpr uint32_t kMaxSpt = 16;     // reservoir slots per thread

struct QLayout {
  uint32_t cst, doph, buckets, cm, hist, sel, misc, ticket, total;  // offsets in 32-bit words
  uint32_t cm_words, cm16_words, hs_size, cst_words, tie_cap;
  bool cst_fit;
};

__host__ __device__ inline uint32_t next_pow2(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

constexpr uint32_t kLdsWords = 160 * 1024 / 4;  // LDS of one CU

__host__ __device__ inline QLayout q_layout(const Shape& s, bool exact = false) {
  QLayout o;
  uint32_t w = 1u << s.lw;
  o.cst_words = const_words(s);
  o.cst_fit = o.cst_words <= kConstCapWords;
  o.cst = 0;
  o.doph = o.cst + (o.cst_fit ? ((o.cst_words + 1) & ~1u) : 0u);
  o.buckets = o.doph + 2 * s.M + ((s.M + 63) / 64) * 2;
  o.cm = (o.buckets + s.L + 3) & ~3u;  // 16-byte aligned: cleared as vectors, ranked keys collected here
  const uint32_t tail = 512 + 2 + 2 * s.k_max + 16;  // hist, alignment, sel, misc
  const uint32_t room = kLdsWords > o.cm + tail ? kLdsWords - (o.cm + tail) : 0u;
  // The id set holds at most L * R distinct ids: twice that (load <= 1/2)
  // when it fits, else the next power of two (a full set still terminates).
  // The exact variant keeps a count beside every id (two words per entry).
  const uint32_t slots = s.L * s.R;
  const uint32_t per = exact ? 2u : 1u;
  o.hs_size = next_pow2(2 * slots);
  if (o.hs_size * per > room && next_pow2(slots) * per <= room) o.hs_size = next_pow2(slots);
  if (o.hs_size < 64) o.hs_size = 64;
  // The sketch is counted with 8-bit counters, all d rows resident; a query
  // whose counts overflow a byte is recounted with 16-bit counters, one row
  // at a time, in the same region.
  o.cm_words = (s.d * w + 3) / 4;
  o.cm16_words = (w + 1) / 2;
  // the id set reuses the count-min region once the estimates are read
  uint32_t region = o.cm_words > o.cm16_words ? o.cm_words : o.cm16_words;
  if (o.hs_size * per > region) region = o.hs_size * per;
  // keys ranked directly when at most this many (collected into the
  // count-min region, free by then, beside one de-duplicated copy)
  o.tie_cap = region / 4 < 128 ? region / 4 : 128;
  o.hist = o.cm + region;
  o.sel = o.hist + 512;
  if (o.sel & 1) o.sel++;
  o.misc = o.sel + 2 * s.k_max;
  // the persistent form's ticket word lives here too: a static LDS variable
  // would shift the dynamic region by 4 bytes and misalign its 64-bit slots
  o.ticket = o.misc + 16;
  o.total = o.ticket + 2;
  return o;
}

// The layout's 64-bit slots (keys collected in the count-min region, the
// radix-select buffer, the top-k bound at misc + 8) must sit on 8-byte
// boundaries: a misaligned 64-bit LDS atomic faults.  Checked on the host
// before any launch.
__host__ __device__ inline bool q_layout_aligned(const QLayout& o) {
  return (o.cm % 2) == 0 && (o.sel % 2) == 0 && (o.misc % 2) == 0 && ((o.misc + 8) % 2) == 0 &&
         (o.doph % 2) == 0 && o.total <= kLdsWords;
}

// Outputs per query up to which the top-k is taken by repeated maximum
// extraction instead of the radix select.
constexpr uint32_t kFewK = 16;

// One DPP step of a 64-bit max: y = x of the lane `ctrl` selects.
template <int CTRL>
__device__ __forceinline__ uint64_t max_dpp(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)x, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(x >> 32), CTRL, 0xF, 0xF, false);
  const uint64_t y = ((uint64_t)hi << 32) | lo;
  return y > x ? y : x;
}

// Maximum over the wave, returned to every lane.  Within each row of 16
// lanes: swap neighbours, swap pairs (quad permutations), mirror each half
// row, mirror the row (DPP moves, no LDS); then the four row maxima are read
// from lanes 0, 16, 32 and 48.
__device__ __forceinline__ uint64_t wave_max64(uint64_t x) {
  x = max_dpp<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x = max_dpp<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x = max_dpp<0x141>(x);  // row_half_mirror
  x = max_dpp<0x140>(x);  // row_mirror
  uint64_t m = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, 16 * r);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), 16 * r);
    const uint64_t y = ((uint64_t)hi << 32) | lo;
    m = y > m ? y : m;
  }
  return m;
}

// Entries of the small distinct-id table (used when at most half as many
// slots have an estimate of 2 or more).
constexpr uint32_t kSmallSetLog2 = 9;
constexpr uint32_t kSmallSet = 1u << kSmallSetLog2;

// Slot of an id in the id set: high bits of a multiplicative hash.
__device__ __forceinline__ uint32_t hs_slot(uint32_t id, uint32_t log2_size) {
  return (id * 0x9E3779B1u) >> (32 - log2_size);
}

// The two quadratic passes over a few dozen collected keys (in LDS).  In
// the 8- and 16-wave groups (one query at a time, latency) they run with
// sixteen lanes per key: lane `sub` of a group visits keys sub, sub + 16,
// ... and the group combines its lanes' results, so a key costs n / 16
// dependent LDS reads instead of n.  The 1- to 4-wave groups (throughput:
// other groups on the CU hide the reads) keep one thread per key, which
// needs fewer registers.  Every thread of the block calls them with the
// same n.

// u[e] = c[e], or 0 when an earlier key equals it.
template <uint32_t NT>
__device__ __forceinline__ void drop_copies(const uint64_t* c, uint64_t* u, uint32_t n) {
  if constexpr (NT < 512) {
    for (uint32_t e = threadIdx.x; e < n; e += NT) {
      const uint64_t x = c[e];
      bool copy = false;
      for (uint32_t j = 0; j < e; ++j) copy |= c[j] == x;
      u[e] = copy ? 0ull : x;
    }
    return;
  }
  const uint32_t sub = threadIdx.x & 15u, grp = threadIdx.x >> 4;
  for (uint32_t e0 = 0; e0 < n; e0 += NT / 16) {
    const uint32_t e = e0 + grp;
    const uint64_t x = e < n ? c[e] : 0ull;
    const uint32_t lim = e < n ? e : 0u;
    uint32_t copy = 0;
    for (uint32_t j = sub; j < lim; j += 16) copy |= c[j] == x ? 1u : 0u;
    copy |= __shfl_xor(copy, 1, 16);
    copy |= __shfl_xor(copy, 2, 16);
    copy |= __shfl_xor(copy, 4, 16);
    copy |= __shfl_xor(copy, 8, 16);
    if (e < n && sub == 0) u[e] = copy ? 0ull : x;
  }
}

// Rank every nonzero key of u[0, n) (distinct) by the number of larger
// keys and write the kk best in order: id = ~low half, score = high half.
template <uint32_t NT>
__device__ __forceinline__ void rank_write(const uint64_t* u, uint32_t n, uint32_t kk, uint32_t* oid, uint32_t* osc) {
  if constexpr (NT < 512) {
    for (uint32_t e = threadIdx.x; e < n; e += NT) {
      const uint64_t x = u[e];
      if (x == 0) continue;
      uint32_t r = 0;
      for (uint32_t j = 0; j < n; ++j) r += u[j] > x ? 1u : 0u;
      if (r < kk) {
        oid[r] = ~(uint32_t)x;
        osc[r] = (uint32_t)(x >> 32);
      }
    }
    return;
  }
  const uint32_t sub = threadIdx.x & 15u, grp = threadIdx.x >> 4;
  for (uint32_t e0 = 0; e0 < n; e0 += NT / 16) {
    const uint32_t e = e0 + grp;
    const uint64_t x = e < n ? u[e] : 0ull;
    const uint32_t lim = e < n ? n : 0u;
    uint32_t r = 0;
    for (uint32_t j = sub; j < lim; j += 16) r += u[j] > x ? 1u : 0u;
    r += __shfl_xor(r, 1, 16);
    r += __shfl_xor(r, 2, 16);
    r += __shfl_xor(r, 4, 16);
    r += __shfl_xor(r, 8, 16);
    if (sub == 0 && x != 0 && r < kk) {
      oid[r] = ~(uint32_t)x;
      osc[r] = (uint32_t)(x >> 32);
    }
  }
}

// Add one to hist[d] for every participating lane, one LDS atomic per
// distinct digit of the wave.
__device__ __forceinline__ void hist_add(uint32_t* hist, bool part, uint32_t d) {
  uint64_t act = ballot64(part);
  if (act == 0) return;
  uint64_t peers = match_digit(d, 8, act);
  if (part && lane_id() == (uint32_t)__builtin_ctzll(peers)) atomicAdd(&hist[d], (uint32_t)__builtin_popcountll(peers));
}

// What a call of query_one does (serving splits a query in two launches):
constexpr int kQueryFull = 0;       // hash, gather, count, rank
constexpr int kQueryGather = 1;     // hash and gather, the slot ids to a.slot_ids[q][slot]
constexpr int kQueryAggregate = 2;  // count and rank the slot ids a gather left in a.slot_ids
// `gathered`, when not null, is counted once the group's slots are all read
// (a table writer may then start; see k_serve_step).  qb, qe, when qb >= 0,
// are query q's row offsets, read from a.q.indptr otherwise.
template <int WAVES, int SPT, bool CL, bool EX, int MODE = kQueryFull>
__device__ void query_one(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& a, uint32_t q,
                          uint32_t* lds, const QLayout& lay, unsigned long long* gathered = nullptr,
                          int64_t qb = -1, int64_t qe = -1) {
  constexpr uint32_t NT = WAVES * SL_WAVE;
  const uint32_t tid = threadIdx.x, wave = tid / SL_WAVE, lane = lane_id();
  uint32_t* bk = lds + lay.buckets;
  uint32_t* cmw = lds + lay.cm;
  uint32_t* hs = lds + lay.cm;  // reused after the estimates
  uint32_t* hist = lds + lay.hist;  // two 256-bin histograms
  uint64_t* sel = (uint64_t*)(lds + lay.sel);
  uint32_t* misc = lds + lay.misc;
  const uint32_t hs_mask = lay.hs_size - 1;
  const uint32_t hs_log2 = 31 - __builtin_clz(lay.hs_size);
  const uint32_t slots = s.L * s.R;

  // 0. clear the sketch, histograms and counters; hash the query (wave 0)
  for (uint32_t e = tid; e < lay.cm_words; e += NT) cmw[e] = 0;
  for (uint32_t e = tid; e < 512; e += NT) hist[e] = 0;
  if (tid < 16) misc[tid] = 0;
  if (MODE == kQueryAggregate) {
    // the slots were read by the gather
  } else if (a.qbk) {
    for (uint32_t t = tid; t < s.L; t += NT) bk[t] = a.qbk[(uint64_t)q * s.L + t];
  } else if (wave == 0) {
    const int64_t beg = qb >= 0 ? qb : a.q.indptr[q], end = qb >= 0 ? qe : a.q.indptr[q + 1];
    const uint32_t* h = doph_wave<CL>(s, c, a.q.indices + beg, (uint32_t)(end - beg), lds + lay.doph);
    for (uint32_t t = lane; t < s.L; t += SL_WAVE) bk[t] = table_bucket<CL>(s, c, h, t);
  }
  __syncthreads();
  // 1. gather the probed reservoirs and count every occurrence.  The slot
  //    arithmetic (a division by R per slot) is redone for every query: left
  //    to itself the compiler keeps it across queries in registers, which at
  //    the occupancy this kernel runs at means spilling it to scratch.
  uint32_t tid_q = tid;
  asm volatile("" : "+v"(tid_q));
  uint32_t id[SPT];
  // slot -> (table, position): a shift when R is a power of two (uniform
  // branch), else a division
  const bool rpow = (s.R & (s.R - 1)) == 0;
  const uint32_t rsh = (uint32_t)__builtin_ctz(s.R);
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    uint32_t sl = tid_q + i * NT;
    id[i] = SL_EMPTY;
    if (sl < slots) {
      if constexpr (MODE == kQueryAggregate) {
        id[i] = a.slot_ids[(uint64_t)q * slots + sl];
      } else {
        const uint32_t t = rpow ? sl >> rsh : sl / s.R;
        const uint32_t j = sl - t * s.R;
        id[i] = tab.ids[((uint64_t)t * s.nb + bk[t]) * s.R + j];
      }
    }
  }
  if constexpr (MODE == kQueryGather) {
    // the stores take the loaded ids, so once every thread has passed the
    // barrier all of this query's table reads are done
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      const uint32_t sl = tid_q + i * NT;
      if (sl < slots) a.slot_ids[(uint64_t)q * slots + sl] = id[i];
    }
    __syncthreads();
    if (gathered && tid == 0) atomicAdd(gathered, 1ull);
    return;
  }
  uint64_t key[SPT];
  uint32_t nrep = 0, emax = 0;
  bool overflow = false;
  if constexpr (!EX) {
    // 2. count-min with 8-bit counters.  Every live slot adds one to each of
    //    the d rows, so without overflow the counters sum to d * live; an
    //    increment that wraps a byte loses 255 or 256 from that sum.  A query
    //    whose sum falls short is recounted with 16-bit counters (one row per
    //    pass; a counter never exceeds L * R <= 65535).  The estimate (min over
    //    rows) goes into the high half of the sort key.
    uint32_t est[SPT];
#pragma unroll
    for (int i = 0; i < SPT; ++i) est[i] = 0xFFFFFFFFu;
    // 16-wave groups with up to 4 slots a thread (one group per CU,
    // registers to spare; 8 slots would spill in the serving step): every
    // slot's cells are kept, 16 bits each, when d <= 4 and d * w <= 65536, and
    // the estimate pass reads them back instead of hashing again
    constexpr bool kCache = NT >= 1024 && SPT <= 4;
    const bool cache = kCache && s.d <= 4 && (s.d << s.lw) <= 65536u;
    uint32_t gc[kCache ? 2 * SPT : 1];  // rows 0, 1 of slot i in gc[2i], rows 2, 3 in gc[2i + 1]
    {
      uint32_t live = 0;
      if (cache) {
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
          if (r < s.d) {
            const uint64_t ar = cld64<CL>(c.a_r, r), br = cld64<CL>(c.b_r, r);
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
              const uint32_t g = (r << s.lw) + cm_hash(ar, br, id[i], s.lw);
              uint32_t& w = gc[kCache ? 2 * i + r / 2 : 0];
              w = (r & 1) ? w | (g << 16) : g;
              if (id[i] != SL_EMPTY) atomicAdd(&cmw[g >> 2], 1u << ((g & 3u) * 8));
            }
          }
        }
      } else {
        for (uint32_t r = 0; r < s.d; ++r) {
          const uint64_t ar = cld64<CL>(c.a_r, r), br = cld64<CL>(c.b_r, r);
#pragma unroll
          for (int i = 0; i < SPT; ++i) {
            if (id[i] != SL_EMPTY) {
              const uint32_t g = (r << s.lw) + cm_hash(ar, br, id[i], s.lw);
              atomicAdd(&cmw[g >> 2], 1u << ((g & 3u) * 8));
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < SPT; ++i) live += id[i] != SL_EMPTY ? 1u : 0u;
      for (int o = 32; o > 0; o >>= 1) live += __shfl_xor(live, o, SL_WAVE);
      if (lane == 0) atomicAdd(&misc[7], live);
    }
    __syncthreads();
    // every thread has used the ids it loaded (the live count above), so
    // all of this query's table reads are done
    if (gathered && tid == 0) atomicAdd(gathered, 1ull);
    // the counter sum and the 8-bit estimates are read in the same pass; the
    // estimates are redone below in the rare case the sum shows an overflow
    {
      uint32_t sum = 0;
      for (uint32_t e = tid; e < lay.cm_words; e += NT) sum = __builtin_amdgcn_sad_u8(cmw[e], 0u, sum);
      for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, SL_WAVE);
      if (lane == 0) atomicAdd(&misc[6], sum);
      if (cache) {
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
          if (r < s.d) {
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
              const uint32_t g = (gc[kCache ? 2 * i + r / 2 : 0] >> (16 * (r & 1))) & 0xFFFFu;
              est[i] = min(est[i], (cmw[g >> 2] >> ((g & 3u) * 8)) & 255u);
            }
          }
        }
      } else {
        for (uint32_t r = 0; r < s.d; ++r) {
          const uint64_t ar = cld64<CL>(c.a_r, r), br = cld64<CL>(c.b_r, r);
#pragma unroll
          for (int i = 0; i < SPT; ++i) {
            const uint32_t g = (r << s.lw) + cm_hash(ar, br, id[i], s.lw);
            est[i] = min(est[i], (cmw[g >> 2] >> ((g & 3u) * 8)) & 255u);
          }
        }
      }
      // slots whose id may occur more than once (estimate >= 2)
      uint32_t multi = 0;
#pragma unroll
      for (int i = 0; i < SPT; ++i) multi += id[i] != SL_EMPTY && est[i] >= 2 ? 1u : 0u;
      for (int o = 32; o > 0; o >>= 1) multi += __shfl_xor(multi, o, SL_WAVE);
      if (lane == 0) atomicAdd(&misc[11], multi);
    }
    __syncthreads();
    overflow = misc[6] != s.d * misc[7];
    if (overflow) {
#pragma unroll
      for (int i = 0; i < SPT; ++i) est[i] = 0xFFFFFFFFu;
      for (uint32_t r = 0; r < s.d; ++r) {
        const uint64_t ar = cld64<CL>(c.a_r, r), br = cld64<CL>(c.b_r, r);
        for (uint32_t e = tid; e < lay.cm16_words; e += NT) cmw[e] = 0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
          if (id[i] != SL_EMPTY) {
            const uint32_t g = cm_hash(ar, br, id[i], s.lw);
            atomicAdd(&cmw[g >> 1], 1u << ((g & 1u) * 16));
          }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
          const uint32_t g = cm_hash(ar, br, id[i], s.lw);
          est[i] = min(est[i], (cmw[g >> 1] >> ((g & 1u) * 16)) & 0xFFFFu);
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int i = 0; i < SPT; ++i) key[i] = id[i] != SL_EMPTY ? ((uint64_t)est[i] << 32) | (uint32_t)~id[i] : 0ull;
  } else {
    // 2'. exact variant: the id set also counts the occurrences of each id
    //     (its multiplicity among the probed slots, at most L); the slot that
    //     inserted the id represents it and takes the count as its score
    uint32_t* hc = hs + lay.hs_size;  // counts beside the ids
    for (uint32_t e = tid; e < lay.hs_size; e += NT) {
      hs[e] = SL_EMPTY;
      hc[e] = 0;
    }
    __syncthreads();
    uint32_t at[SPT];
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      key[i] = 0;
      at[i] = 0xFFFFFFFFu;
      if (id[i] != SL_EMPTY) {
        uint32_t h = hs_slot(id[i], hs_log2);
        for (;;) {
          uint32_t prev = atomicCAS(&hs[h], SL_EMPTY, id[i]);
          if (prev == SL_EMPTY) {
            at[i] = h;  // representative
            break;
          }
          if (prev == id[i]) break;
          h = (h + 1) & hs_mask;
        }
        atomicAdd(&hc[h], 1u);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      if (at[i] != 0xFFFFFFFFu) {
        const uint32_t cnt = hc[at[i]];
        key[i] = ((uint64_t)cnt << 32) | (uint32_t)~id[i];
        ++nrep;
        emax = max(emax, cnt);
      }
    }
  }
  uint32_t kq = a.kq ? a.kq[q] : a.k;
  if (kq > s.k_max) kq = s.k_max;
  uint32_t kk = kq;  // outputs written; fewer when there are fewer distinct ids
  uint32_t* oid = a.out_ids + (uint64_t)q * s.k_max;
  uint32_t* osc = a.out_scores + (uint64_t)q * s.k_max;
  // 3'. few outputs: a lower bound B of the kq-th largest distinct key prunes
  //     the rest.  Keys of one id are equal, so in the count-min variant an
  //     id may still hold several slots here.  Within a wave, taking the
  //     largest lane maximum kq times, and each time retiring every lane that
  //     holds it, yields kq distinct keys, so the last of them is at most the
  //     kq-th largest distinct key of the group; B is the largest such bound
  //     over the waves.  The keys >= B (every distinct key of the top kq, with
  //     their copies) are collected, one copy of each is kept and the copies
  //     ranked directly when they fit; otherwise, or when no wave holds kq
  //     distinct keys, the general path below runs.  The order is exactly
  //     (estimate desc, id asc).
  bool done = false;
  if (kq > 0 && kq <= kFewK) {
    uint64_t lm = 0;
#pragma unroll
    for (int i = 0; i < SPT; ++i) lm = key[i] > lm ? key[i] : lm;
    uint64_t* bound = (uint64_t*)(misc + 8);  // cleared with misc
    // With several waves, the lane maxima go through LDS and wave 0 alone
    // takes the rounds, each of its lanes offering the largest of the lane
    // maxima at its position in every wave (the other waves skip the rounds;
    // the extracted keys are still distinct keys of the group, so the last
    // one is still a lower bound).  The buffer sits after the collection
    // area in the free sketch region.
    const bool shared = WAVES > 1 && 4 * lay.tie_cap + 2 * NT <= lay.hist - lay.cm;
    if (shared) {
      uint64_t* lmv = (uint64_t*)(lds + lay.cm) + 2 * lay.tie_cap;
      lmv[tid] = lm;
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int w = 1; w < WAVES; ++w) {
          const uint64_t x = lmv[lane + w * SL_WAVE];
          lm = x > lm ? x : lm;
        }
      }
    }
    if (!shared || wave == 0) {
      uint64_t kth = 0;
      for (uint32_t r = 0; r < kq; ++r) {
        const uint64_t m = wave_max64(lm);
        kth = m;  // 0 once the wave has fewer than kq distinct lane maxima
        if (m == 0) break;
        if (lm == m) lm = 0;
      }
      if (lane == 0 && kth) atomicMax((unsigned long long*)bound, (unsigned long long)kth);
    }
    __syncthreads();
    const uint64_t B = *bound;
    if (B != 0) {
      uint64_t* cbf = (uint64_t*)(lds + lay.cm);  // the sketch is no longer needed
      uint64_t* uq = cbf + lay.tie_cap;             // one copy of each collected key
#pragma unroll
      for (int i = 0; i < SPT; ++i) {
        const bool in = key[i] != 0 && key[i] >= B;
        const uint64_t m = ballot64(in);
        if (m) {
          uint32_t base = 0;
          if (lane == (uint32_t)__builtin_ctzll(m)) base = atomicAdd(&misc[10], (uint32_t)__builtin_popcountll(m));
          base = __shfl(base, __builtin_ctzll(m), SL_WAVE);
          const uint32_t p = base + (uint32_t)__builtin_popcountll(m & lanemask_lt());
          if (in && p < lay.tie_cap) cbf[p] = key[i];
        }
      }
      __syncthreads();
      const uint32_t ns = misc[10];
      if (ns <= lay.tie_cap) {
        drop_copies<NT>(cbf, uq, ns);
        __syncthreads();
        rank_write<NT>(uq, ns, kq, oid, osc);
        done = true;
      }
      __syncthreads();
    }
  }
  if (!done) {
  if constexpr (!EX) {
    // 3. distinct ids.  The count-min estimate is never below the true
    //    count, so an id whose estimate is 1 occurs once and represents
    //    itself; only the others go through the LDS id set, where the first
    //    insertion represents the id.  When few slots need it (the usual
    //    case) a small table is used, which is cheaper to clear.
    const bool small = !overflow && kSmallSet < lay.hs_size && misc[11] <= kSmallSet / 2;
    const uint32_t set_size = small ? kSmallSet : lay.hs_size;
    const uint32_t set_log2 = small ? kSmallSetLog2 : hs_log2;
    for (uint32_t e = tid; e < set_size; e += NT) hs[e] = SL_EMPTY;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      if (key[i] != 0) {
        const uint32_t idi = ~(uint32_t)key[i];
        bool rep = (key[i] >> 32) == 1;
        uint32_t h = hs_slot(idi, set_log2);
        while (!rep) {
          uint32_t prev = atomicCAS(&hs[h], SL_EMPTY, idi);
          if (prev == SL_EMPTY) {
            rep = true;
            break;
          }
          if (prev == idi) break;
          h = (h + 1) & (set_size - 1);
        }
        if (rep) {
          ++nrep;
          emax = max(emax, (uint32_t)(key[i] >> 32));
        } else {
          key[i] = 0;
        }
      }
    }
  }
  {
    uint32_t v = nrep, m = emax;
    for (int o = 32; o > 0; o >>= 1) {
      v += __shfl_xor(v, o, SL_WAVE);
      m = max(m, (uint32_t)__shfl_xor(m, o, SL_WAVE));
    }
    if (lane == 0) {
      atomicAdd(&misc[0], v);
      atomicMax(&misc[5], m);
    }
    if constexpr (NT >= 1024) {
      // the largest id among the representatives (the tie guess below)
      uint32_t im = 0;
#pragma unroll
      for (int i = 0; i < SPT; ++i) im = key[i] != 0 ? max(im, ~(uint32_t)key[i]) : im;
      for (int o = 32; o > 0; o >>= 1) im = max(im, (uint32_t)__shfl_xor(im, o, SL_WAVE));
      if (lane == 0) atomicMax(&misc[12], im);
      // the threshold select's first round is counted here (histogram
      // buffer 0: the representatives' estimates below 256, which is that
      // round's histogram when every estimate is; otherwise the select
      // clears it): most estimates are 1 and take one atomic per wave, the
      // others one each.  Up to 4 slots a thread (with 8 the serving step
      // would spill).
#pragma unroll
      for (int i = 0; i < (SPT <= 4 ? SPT : 0); ++i) {
        const uint32_t e = (uint32_t)(key[i] >> 32);
        const bool live = key[i] != 0;
        const uint64_t b1 = ballot64(live && e == 1);
        if (b1 && lane == (uint32_t)__builtin_ctzll(b1)) atomicAdd(&hist[1], (uint32_t)__builtin_popcountll(b1));
        if (live && e != 1 && e < 256) atomicAdd(&hist[e], 1u);
      }
    }
  }
  __syncthreads();
  const uint32_t total = misc[0];
  kk = min(kq, total);
  // 4. threshold key.  MSD radix select over 8-bit digits of
  //    (estimate << 32 | ~id), starting at the estimate's low byte when every
  //    estimate is below 256.  Once the estimate E of the kk-th key is known,
  //    if the keys with estimate >= E are few they are all collected and
  //    ranked directly (ties on E are then ordered by id without more radix
  //    rounds); otherwise the select goes on through the id bytes until the
  //    keys >= thr are exactly the kk largest.
  //    16-wave groups (the latency form; in the 8-wave throughput form the
  //    extra registers would cost a group per CU): when many keys tie on E
  //    (k = 100 against about 2,000 ids of estimate 1), the remaining ones
  //    are the smallest ids among the tied; ids are spread evenly below the
  //    largest one, so one counting pass with a guessed id bound usually
  //    leaves between the needed number and 256 keys, which are ranked
  //    directly; when it does not, the radix rounds go on.
  uint64_t thr = 1;  // every representative (their keys are >= 2^32)
  uint32_t n_c = kk;  // keys collected for ranking
  uint64_t* cb = sel;  // where they are collected
  bool guessed = false;
  uint64_t guess_thr = 0;
  if (kk > 0 && kk < total) {
    uint64_t prefix = 0;
    uint32_t remaining = kk;
    uint32_t cur = 0;
    const int top = misc[5] < 256u ? 32 : 40;
    // 16-wave groups: the round at bit 32 was counted with the distinct ids;
    // when it is not the first round, its buffer starts cleared as usual
    constexpr bool kPre = NT >= 1024 && SPT <= 4;
    if (kPre && top == 40) {
      for (uint32_t e = tid; e < 256; e += NT) hist[e] = 0;
      __syncthreads();
    }
    // 8- and 16-wave groups: every wave reads the histogram itself after one
    // barrier per round.  The two buffers are then never cleared: a round's
    // counts are its buffer's totals minus what the buffer held after its
    // previous round, which every lane keeps for its four digits (sa: the
    // buffer of this round, sb: the other; swapped every round).
    uint32_t sa[4] = {0u, 0u, 0u, 0u}, sb[4] = {0u, 0u, 0u, 0u};
    for (int shift = top; shift >= 0; shift -= 8, cur ^= 1u) {
      uint32_t* H = hist + 256 * cur;
      const uint64_t hi_mask = ~0ull << (shift + 8);
      if (!(kPre && top == 32 && shift == 32)) {
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
          bool part = key[i] != 0 && (key[i] & hi_mask) == (prefix & hi_mask);
          hist_add(H, part, (uint32_t)(key[i] >> shift) & 255u);
        }
        __syncthreads();
      }
      uint32_t D = 0, cum = 0, cnt = 0;
      if constexpr (NT >= 512) {
        uint32_t hh[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t t = H[4 * lane + j];
          hh[j] = t - sa[j];
          sa[j] = sb[j];
          sb[j] = t;
        }
        const uint32_t mine = hh[0] + hh[1] + hh[2] + hh[3];
        uint32_t v = mine;
        for (int o = 1; o < SL_WAVE; o <<= 1) {
          uint32_t y = __shfl_down(v, o, SL_WAVE);
          if (lane + o < SL_WAVE) v += y;
        }
        uint32_t c0 = v - mine, fd = 0, fc = 0, fh = 0;
        bool found = false;
        for (int j = 3; j >= 0; --j) {
          if (c0 < remaining && remaining <= c0 + hh[j]) {
            found = true;
            fd = 4 * lane + j;
            fc = c0;
            fh = hh[j];
          }
          c0 += hh[j];
        }
        const uint64_t fm = ballot64(found);
        const int src = fm ? __builtin_ctzll(fm) : 0;
        D = __shfl(fd, src, SL_WAVE);
        cum = __shfl(fc, src, SL_WAVE);
        cnt = __shfl(fh, src, SL_WAVE);
      } else {
        if (wave == 0) {
          // lane owns digits 4*lane .. 4*lane+3; sums over the digits above
          uint32_t h0 = H[4 * lane], h1 = H[4 * lane + 1], h2 = H[4 * lane + 2], h3 = H[4 * lane + 3];
          H[4 * lane] = 0;
          H[4 * lane + 1] = 0;
          H[4 * lane + 2] = 0;
          H[4 * lane + 3] = 0;
          uint32_t mine = h0 + h1 + h2 + h3;
          uint32_t v = mine;
          for (int o = 1; o < SL_WAVE; o <<= 1) {
            uint32_t y = __shfl_down(v, o, SL_WAVE);
            if (lane + o < SL_WAVE) v += y;
          }
          uint32_t hh[4] = {h0, h1, h2, h3};
          uint32_t c0 = v - mine;
          for (int j = 3; j >= 0; --j) {
            if (c0 < remaining && remaining <= c0 + hh[j]) {
              misc[1] = 4 * lane + j;
              misc[2] = c0;
              misc[3] = hh[j];
            }
            c0 += hh[j];
          }
        }
        __syncthreads();
        D = misc[1];
        cum = misc[2];
        cnt = misc[3];
      }
      remaining -= cum;
      prefix |= (uint64_t)D << shift;
      if (remaining == cnt) break;  // the whole digit bin is selected
      if (shift == 32 && kk - remaining + cnt <= lay.tie_cap) {
        n_c = kk - remaining + cnt;  // every key with estimate >= E
        cb = (uint64_t*)(lds + lay.cm);
        break;
      }
      if constexpr (NT >= 1024) {
        // room for collected keys: the count-min region, two words a key
        const uint32_t cap = min((lay.hist - lay.cm) / 2, 256u);
        const uint32_t above = kk - remaining;  // keys with estimate > E
        if (shift == 32 && remaining < cnt && above + remaining < cap) {
          const uint32_t E = (uint32_t)(prefix >> 32);
          // a little over what is needed (the count found spreads by about
          // its square root), within the room: fewer keys to rank
          const uint32_t want = min((remaining + (cap - above)) / 2,
                                    remaining + 4u + (uint32_t)(2.5f * sqrtf((float)remaining)));
          const uint32_t idmax = misc[12];
          // only a guess (the count below checks it exactly): float arithmetic
          // instead of a 64-bit division
          const float xf = fminf((float)idmax * ((float)want / (float)cnt), 4294967040.0f);  // below 2^32
          const uint32_t X = min((uint32_t)xf, idmax);
          uint32_t c = 0;
#pragma unroll
          for (int i = 0; i < SPT; ++i)
            c += (key[i] != 0 && (uint32_t)(key[i] >> 32) == E && ~(uint32_t)key[i] <= X) ? 1u : 0u;
          for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, SL_WAVE);
          if (lane == 0) atomicAdd(&misc[13], c);
          __syncthreads();
          const uint32_t ct = misc[13];
          if (ct >= remaining && above + ct <= cap) {
            // keys >= (E, ~X): those above E and the tied ids up to X
            n_c = above + ct;
            cb = (uint64_t*)(lds + lay.cm);
            guessed = true;
            guess_thr = ((uint64_t)E << 32) | (uint32_t)~X;
            break;
          }
        }
      }
    }
    thr = guessed ? guess_thr : prefix;
  }
  // 5. collect the n_c keys >= thr, rank each among them by counting (keys
  //    are distinct), write the kk best in order
  if (kk > 0) {
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      if (key[i] != 0 && key[i] >= thr) {
        uint32_t p = atomicAdd(&misc[4], 1u);
        cb[p] = key[i];
      }
    }
  }
  __syncthreads();
  rank_write<NT>(cb, n_c, kk, oid, osc);
  }
  for (uint32_t e = kk + tid; e < s.k_max; e += NT) {
    oid[e] = SL_EMPTY;
    osc[e] = 0;
  }
  __syncthreads();
}

// Register budget per SIMD: the LDS of a query group (about 22 KB for the
// 200M shard) lets 7 groups share a CU, so 4-wave groups with up to 8 slots
// per thread are held to 72 VGPRs (7 waves per SIMD); with 16 slots that
// would spill, so they keep 128 (4 waves), as do 2-wave groups (their LDS
// allows 3.5 per SIMD).
template <int WAVES, int SPT>
constexpr int query_min_waves() {
  return WAVES == 4 ? (SPT <= 8 ? 7 : 4) : (WAVES == 2 ? 4 : (WAVES == 1 ? 2 : 1));
}

template <int WAVES, int SPT, bool CL, bool EX>
__global__ void __launch_bounds__(WAVES * SL_WAVE, (query_min_waves<WAVES, SPT>()))
    k_query(Shape s, ConstView c, TablesView tab, QueryArgs a) {
  extern __shared__ uint32_t lds[];
  const QLayout lay = q_layout(s, EX);
  const ConstView cl = CL ? stage_consts(s, c, lds + lay.cst, WAVES * SL_WAVE) : c;
  __syncthreads();
  for (uint64_t q = blockIdx.x; q < a.q.n_rows; q += gridDim.x)
    query_one<WAVES, SPT, CL, EX>(s, cl, tab, a, (uint32_t)q, lds, lay);
}

template <int WAVES, int SPT, bool CL, bool EX>
__global__ void __launch_bounds__(WAVES * SL_WAVE, (query_min_waves<WAVES, SPT>()))
    k_query_persistent(Shape s, ConstView c, TablesView tab, QueryArgs a, uint32_t per_ticket, uint32_t* ticket) {
  extern __shared__ uint32_t lds[];
  const QLayout lay = q_layout(s, EX);
  uint32_t& base_sh = lds[lay.ticket];
  const ConstView cl = CL ? stage_consts(s, c, lds + lay.cst, WAVES * SL_WAVE) : c;
  const uint64_t n = a.q.n_rows;
  // the next ticket is taken while the current one is answered, so the
  // atomic's round trip is off the critical path
  uint32_t next = 0;
  if (threadIdx.x == 0) next = atomicAdd(ticket, per_ticket);
  for (;;) {
    if (threadIdx.x == 0) base_sh = next;
    __syncthreads();
    const uint64_t base = base_sh;
    __syncthreads();
    if (base >= n) break;
    if (threadIdx.x == 0) next = atomicAdd(ticket, per_ticket);
    const uint64_t stop = base + per_ticket < n ? base + per_ticket : n;
    for (uint64_t q = base; q < stop; ++q) query_one<WAVES, SPT, CL, EX>(s, cl, tab, a, (uint32_t)q, lds, lay);
  }
}

// One serving launch (16-wave work-groups).  Every group takes a ticket when
// it starts; in ticket order the groups are:
//   1. the second half of the previous batch's queries, one group each:
//      count and rank the slot ids their gather left in prev.slot_ids (they
//      read no table);
//   2. this batch's queries, one group each, whole or (gather_only) only the
//      first half (hash, read the slots, store their ids in cur.slot_ids);
//      each counts itself in sync[1] once all its table reads are done;
//   3. the table writers of the insert queued behind this batch (sixteen
//      lanes per run record, the groups striding over the records); before
//      its first live record each wave waits until every query of this
//      batch has counted itself.
// So this batch's queries see the tables without the insert, the next
// launch on the stream sees them with it, and a batch whose insert follows
// it is ranked in the next launch, beside the next batch's reads, instead of
// holding the insert (and every later epoch) back until its slowest query
// is ranked.  A group only waits for groups that took earlier tickets: those
// are running and wait for nothing, so the wait ends; it is bounded all the
// same, and a group that gives up sets *gave_up.  Both counters only grow;
// the host passes their values before this launch.
constexpr uint32_t kStepWaves = 16;
constexpr uint32_t kStepSpinLimit = 1u << 20;  // polls: seconds at most, against microseconds needed

constexpr uint32_t kStepBounds = 32;  // queries of cur whose row offsets come with the launch
struct StepArgs {
  QueryArgs prev, cur;
  uint32_t n_bounds;                  // cur.q's first n_bounds queries: offsets bounds[q], bounds[q + 1]
  uint32_t bounds[kStepBounds + 1];
  uint32_t gather_only;
  uint32_t n_ins, merge_groups;
  const uint2* recs;      // [L][n_ins] run records of the prepared insert
  const uint32_t* items;  // [L][n_ins] their new ids
  unsigned long long* sync;  // [0] tickets taken, [1] queries past their reads
  unsigned long long ticket_base, gathered_target;
  uint32_t* gave_up;  // host-coherent
};

template <int SPT, int E>
__global__ void __launch_bounds__(kStepWaves * SL_WAVE, (query_min_waves<kStepWaves, SPT>()))
    k_serve_step(Shape s, ConstView c, TablesView tab, StepArgs a) {
  constexpr uint32_t NT = kStepWaves * SL_WAVE;
  extern __shared__ uint32_t lds[];
  const QLayout lay = q_layout(s, false);
  if (threadIdx.x == 0) lds[lay.ticket] = (uint32_t)(atomicAdd(&a.sync[0], 1ull) - a.ticket_base);
  __syncthreads();
  const uint32_t ticket = lds[lay.ticket];
  const uint32_t np = (uint32_t)a.prev.q.n_rows, nc = (uint32_t)a.cur.q.n_rows;
  if (ticket < np + nc) {
    const ConstView cl = stage_consts(s, c, lds + lay.cst, NT);
    __syncthreads();
    if (ticket < np)
      query_one<kStepWaves, SPT, true, false, kQueryAggregate>(s, cl, tab, a.prev, ticket, lds, lay);
    else {
      // the query's row offsets from the launch when they came with it (no
      // read of the host-coherent staging before its indices)
      const uint32_t q = ticket - np;
      int64_t qb = -1, qe = -1;
      // up to 4 slots a thread (with more the kernel would spill)
      if (SPT <= 4 && q < a.n_bounds) {
        // constant offsets into the launch's arguments (a variable index
        // would make the compiler copy them to scratch)
#pragma unroll
        for (uint32_t j = 0; j < kStepBounds; ++j)
          if (j == q) {
            qb = a.bounds[j];
            qe = a.bounds[j + 1];
          }
      }
      if (a.gather_only)
        query_one<kStepWaves, SPT, true, false, kQueryGather>(s, cl, tab, a.cur, q, lds, lay, &a.sync[1], qb, qe);
      else
        query_one<kStepWaves, SPT, true, false, kQueryFull>(s, cl, tab, a.cur, q, lds, lay, &a.sync[1], qb, qe);
    }
    return;
  }
  // table writers: each wave takes four records per pass and, before its
  // first live record, waits for the batch's queries (lane 0 polls)
  const uint64_t runs = (uint64_t)s.L * a.n_ins;
  constexpr uint32_t per = NT / 16;  // records per group and pass
  bool waited = false;
  for (uint64_t r0 = (uint64_t)(ticket - np - nc) * per; r0 < runs; r0 += (uint64_t)a.merge_groups * per) {
    const uint64_t run = r0 + threadIdx.x / 16;
    const uint2 rec = run < runs ? a.recs[run] : make_uint2(0u, 0u);
    const bool live = (rec.y >> 16) != 0;
    if (__ballot(live) == 0) continue;
    if (!waited) {
      if (lane_id() == 0) {
        uint32_t spins = 0;
        while (__hip_atomic_load(&a.sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < a.gathered_target) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins == kStepSpinLimit) {
            *(volatile uint32_t*)a.gave_up = 1u;
            break;
          }
        }
      }
      waited = true;
    }
    if (live) {
      const uint32_t t = (uint32_t)(run / a.n_ins);
      merge_run16<E>(s, c, rec, t, a.items + (uint64_t)t * a.n_ins, tab);
    }
  }
}

// serving-step kernels by [log2 slots per thread][log2 entries per lane]
template <int S>
constexpr std::array<const void*, 4> kstep() {
  return {(const void*)k_serve_step<S, 1>, (const void*)k_serve_step<S, 2>, (const void*)k_serve_step<S, 4>,
          (const void*)k_serve_step<S, 8>};
}
const std::array<const void*, 4> kStepKernels[5] = {kstep<1>(), kstep<2>(), kstep<4>(), kstep<8>(), kstep<16>()};

struct KPair {
  const void* plain;
  const void* persistent;
};

template <int W, int S, bool CL, bool EX>
constexpr KPair kp1() {
  return KPair{(const void*)k_query<W, S, CL, EX>, (const void*)k_query_persistent<W, S, CL, EX>};
}
template <int W, int S>
constexpr KPair kp() { return kp1<W, S, true, false>(); }
template <int W, int S>
constexpr KPair kg() { return kp1<W, S, false, false>(); }
template <int W, int S>
constexpr KPair kx() { return kp1<W, S, true, true>(); }

// kernels reading global constants (tables too large for LDS)
const KPair kKernelsG[5][5] = {
    {kg<1, 1>(), kg<1, 2>(), kg<1, 4>(), kg<1, 8>(), kg<1, 16>()},
    {kg<2, 1>(), kg<2, 2>(), kg<2, 4>(), kg<2, 8>(), kg<2, 16>()},
    {kg<4, 1>(), kg<4, 2>(), kg<4, 4>(), kg<4, 8>(), kg<4, 16>()},
    {kg<8, 1>(), kg<8, 2>(), kg<8, 4>(), kg<8, 8>(), kg<8, 16>()},
    {kg<16, 1>(), kg<16, 2>(), kg<16, 4>(), kg<16, 8>(), kg<16, 16>()},
};

// kernels by [log2 waves][log2 slots per thread]
const KPair kKernels[5][5] = {
    {kp<1, 1>(), kp<1, 2>(), kp<1, 4>(), kp<1, 8>(), kp<1, 16>()},
    {kp<2, 1>(), kp<2, 2>(), kp<2, 4>(), kp<2, 8>(), kp<2, 16>()},
    {kp<4, 1>(), kp<4, 2>(), kp<4, 4>(), kp<4, 8>(), kp<4, 16>()},
    {kp<8, 1>(), kp<8, 2>(), kp<8, 4>(), kp<8, 8>(), kp<8, 16>()},
    {kp<16, 1>(), kp<16, 2>(), kp<16, 4>(), kp<16, 8>(), kp<16, 16>()},
};

// exact-multiplicity kernels (constants staged in LDS)
const KPair kKernelsX[5][5] = {
    {kx<1, 1>(), kx<1, 2>(), kx<1, 4>(), kx<1, 8>(), kx<1, 16>()},
    {kx<2, 1>(), kx<2, 2>(), kx<2, 4>(), kx<2, 8>(), kx<2, 16>()},
    {kx<4, 1>(), kx<4, 2>(), kx<4, 4>(), kx<4, 8>(), kx<4, 16>()},
    {kx<8, 1>(), kx<8, 2>(), kx<8, 4>(), kx<8, 8>(), kx<8, 16>()},
    {kx<16, 1>(), kx<16, 2>(), kx<16, 4>(), kx<16, 8>(), kx<16, 16>()},
};

int ilog2(uint32_t x) {
  int b = 0;
  while ((1u << b) < x) ++b;
  return b;
}

// Kernel pair for `waves` waves per query, or nullptr (the exact variant
// needs the constants staged in LDS).
const KPair* pick(const Shape& s, uint32_t waves, bool exact) {
  if (waves == 0 || waves > 16 || (waves & (waves - 1))) return nullptr;
  uint32_t slots = s.L * s.R;
  uint32_t spt = (slots + waves * SL_WAVE - 1) / (waves * SL_WAVE);
  if (spt > kMaxSpt) return nullptr;
  const int wi = ilog2(waves), si = ilog2(spt < 1 ? 1 : spt);
  if (exact) return q_layout(s).cst_fit ? &kKernelsX[wi][si] : nullptr;
  return q_layout(s).cst_fit ? &kKernels[wi][si] : &kKernelsG[wi][si];
}

hipError_t allow_lds(const KPair* k, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(k->plain, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(k->persistent, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace

uint32_t query_default_waves(const Shape& s) {
  // enough waves that a thread holds at most 8 reservoir slots
  uint32_t slots = s.L * s.R;
  uint32_t waves = 1;
  while (waves < 16 && slots > waves * SL_WAVE * 8) waves <<= 1;
  return waves;
}

int query_block_threads(const Shape& s, uint32_t waves) { return (int)(waves * SL_WAVE); }

size_t query_lds_bytes(const Shape& s, uint32_t waves, bool exact) {
  (void)waves;
  return (size_t)q_layout(s, exact).total * 4;
}

bool query_supported(const Shape& s, uint32_t waves, bool exact) {
  if (!pick(s, waves, exact)) return false;
  if (s.L * s.R > 65535u) return false;
  if (!q_layout_aligned(q_layout(s, exact))) return false;
  return query_lds_bytes(s, waves, exact) <= (size_t)kLdsWords * 4;
}

bool query_supported(const Shape& s) { return query_supported(s, query_default_waves(s), false); }

hipError_t launch_query_waves(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& a,
                              uint32_t waves, hipStream_t st) {
  if (a.q.n_rows == 0) return hipSuccess;
  if (!query_supported(s, waves, a.exact != 0)) return hipErrorInvalidValue;
  const KPair* k = pick(s, waves, a.exact != 0);
  size_t lds = query_lds_bytes(s, waves, a.exact != 0);
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  uint32_t grid = (uint32_t)(a.q.n_rows < (1u << 30) ? a.q.n_rows : (1u << 30));
  Shape sh = s;
  ConstView cv = c;
  TablesView tv = tab;
  QueryArgs qa = a;
  void* args[] = {&sh, &cv, &tv, &qa};
  e = hipLaunchKernel(k->plain, dim3(grid), dim3(waves * SL_WAVE), args, lds, st);
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
  if (!query_supported(s, waves, a.exact != 0)) return hipErrorInvalidValue;
  if (per_ticket == 0) per_ticket = 1;
  const KPair* k = pick(s, waves, a.exact != 0);
  size_t lds = query_lds_bytes(s, waves, a.exact != 0);
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  Shape sh = s;
  ConstView cv = c;
  TablesView tv = tab;
  QueryArgs qa = a;
  void* args[] = {&sh, &cv, &tv, &qa, &per_ticket, &ticket};
  e = hipLaunchKernel(k->persistent, dim3(grid), dim3(waves * SL_WAVE), args, lds, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// Serving-step kernel for this shape (count-min queries, constants in LDS,
// R <= 128), or nullptr.
static const void* step_kernel(const Shape& s) {
  if (s.bucket || s.R > 128 || !query_supported(s, kStepWaves, false)) return nullptr;
  if (!q_layout(s).cst_fit) return nullptr;
  const uint32_t spt = (s.L * s.R + kStepWaves * SL_WAVE - 1) / (kStepWaves * SL_WAVE);
  const uint32_t e = (s.R + 15) / 16;
  return kStepKernels[ilog2(spt < 1 ? 1 : spt)][ilog2(e)];
}

bool serve_step_supported(const Shape& s) { return step_kernel(s) != nullptr; }

hipError_t launch_serve_step(const Shape& s, const ConstView& c, const TablesView& tab, const QueryArgs& prev,
                             const QueryArgs& cur, bool gather_only, void* ins_scratch, uint32_t n_ins, int n_cu,
                             FuseSync& fs, hipStream_t st, const int64_t* cur_host_ip) {
  const void* k = step_kernel(s);
  if (!k || !fs.dev || !fs.gave_up) return hipErrorNotSupported;
  if (prev.exact || cur.exact || prev.qbk || cur.qbk || prev.q.n_rows > (1u << 20) || cur.q.n_rows > (1u << 20))
    return hipErrorInvalidValue;
  if ((prev.q.n_rows && !prev.slot_ids) || (gather_only && cur.q.n_rows && !cur.slot_ids)) return hipErrorInvalidValue;
  StepArgs a;
  a.prev = prev;
  a.cur = cur;
  a.gather_only = gather_only ? 1u : 0u;
  a.n_bounds = 0;
  if (cur_host_ip && cur.q.n_rows && cur_host_ip[cur.q.n_rows] <= 0xFFFFFFFFll) {
    a.n_bounds = (uint32_t)std::min<uint64_t>(cur.q.n_rows, kStepBounds);
    for (uint32_t q = 0; q <= a.n_bounds; ++q) a.bounds[q] = (uint32_t)cur_host_ip[q];
  }
  a.n_ins = 0;
  a.merge_groups = 0;
  a.recs = nullptr;
  a.items = nullptr;
  const uint32_t np = (uint32_t)prev.q.n_rows, nc = (uint32_t)cur.q.n_rows;
  if (n_ins) {
    if (!insert_run_arrays(s, ins_scratch, n_ins, &a.recs, &a.items)) return hipErrorInvalidValue;
    const uint64_t runs = (uint64_t)s.L * n_ins;
    constexpr uint32_t per = kStepWaves * SL_WAVE / 16;
    // one 16-wave group per CU beside the queries (what the kernel's
    // registers allow); the groups stride over the records
    const uint64_t want = (runs + per - 1) / per;
    const uint64_t room = (uint64_t)std::max(n_cu - (int)std::min<uint32_t>(np + nc, 1u << 20), 64);
    a.n_ins = n_ins;
    a.merge_groups = (uint32_t)std::max<uint64_t>(1, std::min(want, room));
  }
  const uint32_t grid = np + nc + a.merge_groups;
  if (grid == 0) return hipSuccess;
  const size_t lds = query_lds_bytes(s, kStepWaves, false);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  a.sync = fs.dev;
  a.ticket_base = fs.tickets;
  a.gathered_target = fs.gathered + nc;
  a.gave_up = fs.gave_up;
  Shape sh = s;
  ConstView cv = c;
  TablesView tv = tab;
  void* args[] = {&sh, &cv, &tv, &a};
  hipError_t e = hipLaunchKernel(k, dim3(grid), dim3(kStepWaves * SL_WAVE), args, lds, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return e;
  fs.tickets += grid;
  fs.gathered += nc;
  return hipSuccess;
}

void* persistent_query_kernel(const Shape& s, uint32_t waves, bool exact) {
  const KPair* k = pick(s, waves, exact);
  return k ? const_cast<void*>(k->persistent) : nullptr;
}

void* plain_query_kernel(const Shape& s, uint32_t waves, bool exact) {
  const KPair* k = pick(s, waves, exact);
  return k ? const_cast<void*>(k->plain) : nullptr;
}

// Occupancy of the persistent kernel: resident work-groups per CU.
hipError_t query_occupancy(const Shape& s, uint32_t waves, int* per_cu, bool exact) {
  const KPair* k = pick(s, waves, exact);
  if (!k) return hipErrorInvalidValue;
  size_t lds = query_lds_bytes(s, waves, exact);
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k->persistent, waves * SL_WAVE, lds);
}

}  // namespace slash
