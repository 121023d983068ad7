// Merge of new ids into one stored reservoir by a group of sixteen lanes
// (Section 3 "Avoid Skewed buckets": a bucket keeps a fixed-size sample;
// here the R ids of smallest priority, whatever the arrival order).  Shared
// by the insert kernel and the query kernel that also applies the insert
// queued behind its batch.
#pragma once

#include "slash_internal.h"

namespace slash {

// Entry e of lane g (0..15) of the group is reservoir position g * E + e.
template <int E>
__device__ __forceinline__ void load_row(const uint32_t* __restrict__ row, uint32_t R, uint32_t g, uint32_t (&v)[E]) {
  if (R == 16u * E && E >= 2) {
    const uint32_t* p = row + g * E;
    if constexpr (E == 2) {
      uint2 x = *(const uint2*)p;
      v[0] = x.x;
      v[1] = x.y;
    } else {
#pragma unroll
      for (int q = 0; q < E / 4; ++q) {
        uint4 x = ((const uint4*)p)[q];
        v[4 * q] = x.x;
        v[4 * q + 1] = x.y;
        v[4 * q + 2] = x.z;
        v[4 * q + 3] = x.w;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = g * E + e < R ? row[g * E + e] : 0xFFFFFFFFu;
  }
}

template <int E>
__device__ __forceinline__ void store_row(uint32_t* __restrict__ row, uint32_t R, uint32_t g, const uint32_t (&v)[E]) {
  if (R == 16u * E && E >= 2) {
    uint32_t* p = row + g * E;
    if constexpr (E == 2) {
      *(uint2*)p = make_uint2(v[0], v[1]);
    } else {
#pragma unroll
      for (int q = 0; q < E / 4; ++q) ((uint4*)p)[q] = make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (g * E + e < R) row[g * E + e] = v[e];
  }
}

// Apply run record `rec` of table t (bucket rec.x; rec.y = first item |
// count << 16, items are the run's new ids) to the table.  The sixteen lanes
// of the group hold the reservoir in registers (E entries per lane, in
// ascending priority) and insert each new id whose priority is below the
// current R-th one at its rank (group sum of per-lane counts, one shift);
// the row is written back only when it changed.  Every lane of the group
// calls this with the same arguments, so the group's shuffles only read
// lanes of the same group.  E * 16 >= R.
template <int E>
__device__ __forceinline__ void merge_run16(const Shape& s, const ConstView& c, uint2 rec, uint32_t t,
                                            const uint32_t* __restrict__ items, TablesView tab) {
  const uint32_t lane = lane_id(), g = lane & 15u, gbase = lane & ~15u;
  const uint32_t len = rec.y >> 16;
  const uint32_t start = rec.y & 0xFFFFu, b = rec.x, R = s.R;
  const uint32_t key = c.key_t[t], m1 = c.m1_t[t], m2 = c.m2_t[t];
  uint32_t* row = tab.ids + ((uint64_t)t * s.nb + b) * R;
  uint32_t* seen = tab.seen + (uint64_t)t * s.nb + b;
  const uint32_t* it = items + start;
  uint32_t v[E], p[E];
  load_row<E>(row, R, g, v);
  const uint32_t old = *seen;
  uint32_t nid = g < len ? it[g] : 0u;
  uint32_t fill = min(old, R);
#pragma unroll
  for (int e = 0; e < E; ++e) p[e] = priority(v[e], key, m1, m2);
  // priority of the entry at position R - 1 (meaningful once fill == R)
  const uint32_t last_lane = gbase + (R - 1) / E, last_e = (R - 1) % E;
  auto last_prio = [&]() {
    uint32_t x = p[0];
#pragma unroll
    for (int e = 1; e < E; ++e)
      if ((uint32_t)e == last_e) x = p[e];
    return __shfl(x, last_lane, SL_WAVE);
  };
  bool dirty = false;
  for (uint32_t c0 = 0; c0 < len; c0 += 16) {
    if (c0) nid = c0 + g < len ? it[c0 + g] : 0u;
    const uint32_t nq = priority(nid, key, m1, m2);
    const bool full = fill == R;
    const uint32_t lim = full ? last_prio() : 0u;
    const bool cand = c0 + g < len && (!full || nq < lim);
    uint32_t gm = (uint32_t)((__ballot(cand) >> gbase) & 0xFFFFull);
    while (gm) {
      const uint32_t src = __builtin_ctz(gm);
      gm &= gm - 1;
      const uint32_t x = __shfl(nid, gbase + src, SL_WAVE), q = __shfl(nq, gbase + src, SL_WAVE);
      // rank of q among the live entries
      uint32_t cnt = 0;
#pragma unroll
      for (int e = 0; e < E; ++e) cnt += (g * E + e < fill && p[e] < q) ? 1u : 0u;
      cnt += __shfl_xor(cnt, 1, 16);
      cnt += __shfl_xor(cnt, 2, 16);
      cnt += __shfl_xor(cnt, 4, 16);
      cnt += __shfl_xor(cnt, 8, 16);
      const uint32_t pos = cnt;
      if (pos >= R) continue;  // below none of a full reservoir's entries
      dirty = true;
      const uint32_t pp = __shfl_up(p[E - 1], 1, 16), pv = __shfl_up(v[E - 1], 1, 16);
#pragma unroll
      for (int e = E - 1; e >= 0; --e) {
        const uint32_t k = g * E + e;
        const uint32_t lp = e ? p[e - 1] : pp, lv = e ? v[e - 1] : pv;
        if (k > pos) {
          p[e] = lp;
          v[e] = lv;
        } else if (k == pos) {
          p[e] = q;
          v[e] = x;
        }
      }
      fill = min(R, fill + 1);
    }
  }
  if (dirty) store_row<E>(row, R, g, v);
  if (g == 0) *seen = old + len;
}

}  // namespace slash
