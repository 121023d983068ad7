/*
 * Plain CPU oracle for the SLASH hot path (Meisburger & Shrivastava,
 * "Distributed Tera-Scale Similarity Search with MPI").
 *
 * TEST INFRASTRUCTURE.  This file is the slow, single-threaded, obviously
 * correct statement of what the GPU library must compute, bit for bit.  Only
 * the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code with the GPU library.
 *
 * Where the paper fixes the computation, the code follows it:
 *   - MinHash / densified one-permutation hashing (DOPH): Section 2.2.
 *   - (K, L) tables, each address H_i(x) built from K hashes: Section 2.3.
 *   - Pre-processing inserts every vector into its bucket in each of the L
 *     tables: Algorithm 1 (Section 3.1) and Section 4 "Pre-processing".
 *   - Fixed-size buckets by sub-sampling heavy buckets (reservoirs): Section 3,
 *     "Avoid Skewed buckets"; streaming insertion into fixed-size summaries:
 *     Section 3.1 and Appendix 2.
 *   - Query: hash, probe the L buckets, aggregate candidate frequencies in a
 *     count-min style sketch and report the top-k identities: Section 2.3
 *     "Cheap Frequency based Filtering", Algorithm 2, Section 2.4, Appendix 2.
 *
 * Where the paper is silent, this oracle fixes one reading (all integer, all
 * orders total, so results are unique):
 *   - constants: one SplitMix64 stream (Steele, Lea, Flood 2014) from the
 *     seed, drawn in a fixed order (oracle_constants);
 *   - nonzero hash u(i) = hi32(a_h * i + b_h), bin = hi32(u * M) over
 *     M = K * L contiguous range bins (hash_mode 0), or per table K bins with
 *     a per-table (a_h, b_h) (hash_mode 1), or classic MinHash with M
 *     independent hash functions, one (a_h, b_h) each and no bins
 *     (hash_mode 2);
 *   - densification direction is a fixed bit per bin, the walk is circular
 *     over the pre-densification minima;
 *   - bucket id = (sum_j a_tj * h[tK + j] + b_t) >> (64 - B), mod 2^64;
 *   - the reservoir keeps the R ids of smallest priority p_t(id), an
 *     xor-multiply-xorshift bijection of uint32, in ascending priority;
 *   - count-min row hash g_r(c) = (a_r * c + b_r) >> (64 - log2 w);
 *   - top-k by (estimate desc, id asc), padded with (0xFFFFFFFF, 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))
#define EMPTY 0xFFFFFFFFu

enum { O_OK = 0, O_EINVAL = -1, O_ENOMEM = -2, O_ECAPACITY = -4 };

typedef struct {
  uint32_t dim, K, L, log2_buckets, R, cm_rows, log2_cm_width, hash_mode;
  uint64_t seed;
} oracle_params;

/* ------------------------------------------------------------ constants */

/* Layout of the flat constant table (each entry a uint64). */
typedef struct {
  uint64_t n_h, a_h, b_h, dir, a_tj, b_t, key_t, m1_t, m2_t, a_r, b_r, total;
} layout_t;

static layout_t layout(const oracle_params* p) {
  layout_t o;
  uint64_t M = (uint64_t)p->K * p->L;
  o.n_h = p->hash_mode == 2 ? (uint64_t)p->K * p->L : (p->hash_mode ? p->L : 1);
  o.a_h = 0;
  o.b_h = o.a_h + o.n_h;
  o.dir = o.b_h + o.n_h;
  o.a_tj = o.dir + M;
  o.b_t = o.a_tj + M;
  o.key_t = o.b_t + p->L;
  o.m1_t = o.key_t + p->L;
  o.m2_t = o.m1_t + p->L;
  o.a_r = o.m2_t + p->L;
  o.b_r = o.a_r + p->cm_rows;
  o.total = o.b_r + p->cm_rows;
  return o;
}

EXPORT uint64_t oracle_constants_size(const oracle_params* p) { return layout(p).total; }

/* SplitMix64, as published by Steele, Lea and Flood (OOPSLA 2014). */
static uint64_t splitmix64(uint64_t* state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

EXPORT uint64_t oracle_splitmix64(uint64_t* state) { return splitmix64(state); }

static int params_ok(const oracle_params* p) {
  if (!p) return 0;
  if (p->dim == 0 || p->K == 0 || p->L == 0 || p->R == 0 || p->cm_rows == 0) return 0;
  if (p->log2_buckets == 0 || p->log2_buckets > 32) return 0;
  if (p->log2_cm_width > 32) return 0;
  if (p->hash_mode > 2) return 0;
  return 1;
}

/* The paper shares one random seed among all workers so every node derives
 * the same L x K hash functions (Section 3, "Design"; Section 4
 * "Initialization").  Draw order: (1) a_h|1, b_h (once; per table in
 * hash_mode 1; per hash function in hash_mode 2; interleaved); (2) one
 * direction bit (top bit) per bin; (3) per table K odd multipliers then one
 * offset; (4) per table the priority key and two odd 32-bit multipliers;
 * (5) per count-min row an odd multiplier and an offset. */
EXPORT int oracle_constants(const oracle_params* p, uint64_t* out) {
  if (!params_ok(p) || !out) return O_EINVAL;
  layout_t o = layout(p);
  uint64_t s = p->seed;
  uint64_t M = (uint64_t)p->K * p->L;
  for (uint64_t t = 0; t < o.n_h; ++t) {
    out[o.a_h + t] = splitmix64(&s) | 1u;
    out[o.b_h + t] = splitmix64(&s);
  }
  for (uint64_t b = 0; b < M; ++b) out[o.dir + b] = splitmix64(&s) >> 63;
  for (uint32_t t = 0; t < p->L; ++t) {
    for (uint32_t j = 0; j < p->K; ++j) out[o.a_tj + (uint64_t)t * p->K + j] = splitmix64(&s) | 1u;
    out[o.b_t + t] = splitmix64(&s);
  }
  for (uint32_t t = 0; t < p->L; ++t) {
    out[o.key_t + t] = (uint32_t)splitmix64(&s);
    out[o.m1_t + t] = (uint32_t)splitmix64(&s) | 1u;
    out[o.m2_t + t] = (uint32_t)splitmix64(&s) | 1u;
  }
  for (uint32_t r = 0; r < p->cm_rows; ++r) {
    out[o.a_r + r] = splitmix64(&s) | 1u;
    out[o.b_r + r] = splitmix64(&s);
  }
  return O_OK;
}

/* ------------------------------------------------------------- hashing */

static uint32_t hi32(uint64_t z) { return (uint32_t)(z >> 32); }

/* Densification (Section 2.2): an empty bin takes the minimum of the nearest
 * non-empty bin to its left or right; the side is a fixed function of the bin
 * (its direction bit), the walk wraps around the n bins of its domain and
 * reads the pre-densification minima.  If every bin is empty the values stay
 * EMPTY. */
static void densify(const uint32_t* m, uint32_t* h, uint32_t n, const uint64_t* dir) {
  int any = 0;
  for (uint32_t b = 0; b < n; ++b) any |= (m[b] != EMPTY);
  for (uint32_t b = 0; b < n; ++b) {
    if (m[b] != EMPTY || !any) {
      h[b] = m[b];
      continue;
    }
    int64_t step = dir[b] ? 1 : -1;
    int64_t c = b;
    do {
      c = (c + step + (int64_t)n) % (int64_t)n;
    } while (m[c] == EMPTY);
    h[b] = m[c];
  }
}

/* DOPH values h[0..M) of one row (Section 2.2): every nonzero index i is
 * hashed once, u(i) = hi32(a_h * i + b_h); the hash range is split into M
 * equal bins; each bin keeps the smallest value that falls in it; empty bins
 * are densified.  hash_mode 1 runs this per table with K bins.  hash_mode 2
 * is the classic MinHash of Section 2.2 with the L x K seeds of Section 4
 * "Initialization": value j is min over the row of u_j(i) =
 * hi32(a_h[j] * i + b_h[j]), a 2-universal stand-in for the j-th random
 * permutation; nothing is binned, so nothing is densified. */
static void doph(const oracle_params* p, const uint64_t* cs, const int32_t* idx, uint64_t nnz,
                 uint32_t* m, uint32_t* h) {
  layout_t o = layout(p);
  uint32_t M = p->K * p->L;
  for (uint32_t b = 0; b < M; ++b) m[b] = EMPTY;
  if (p->hash_mode == 0) {
    for (uint64_t e = 0; e < nnz; ++e) {
      uint32_t i = (uint32_t)idx[e];
      uint32_t u = hi32(cs[o.a_h] * (uint64_t)i + cs[o.b_h]);
      uint32_t bin = hi32((uint64_t)u * M);
      if (u < m[bin]) m[bin] = u;
    }
    densify(m, h, M, cs + o.dir);
  } else if (p->hash_mode == 2) {
    for (uint32_t j = 0; j < M; ++j) {
      for (uint64_t e = 0; e < nnz; ++e) {
        uint32_t u = hi32(cs[o.a_h + j] * (uint64_t)(uint32_t)idx[e] + cs[o.b_h + j]);
        if (u < m[j]) m[j] = u;
      }
      h[j] = m[j];
    }
  } else {
    for (uint32_t t = 0; t < p->L; ++t) {
      uint32_t* mt = m + (uint64_t)t * p->K;
      for (uint64_t e = 0; e < nnz; ++e) {
        uint32_t i = (uint32_t)idx[e];
        uint32_t u = hi32(cs[o.a_h + t] * (uint64_t)i + cs[o.b_h + t]);
        uint32_t bin = hi32((uint64_t)u * p->K);
        if (u < mt[bin]) mt[bin] = u;
      }
      densify(mt, h + (uint64_t)t * p->K, p->K, cs + o.dir + (uint64_t)t * p->K);
    }
  }
}

/* Address of table t (Section 2.3): the K values of the table's bins are
 * combined into one B-bit bucket id. */
static uint32_t bucket_of(const oracle_params* p, const uint64_t* cs, const uint32_t* h, uint32_t t) {
  layout_t o = layout(p);
  uint64_t acc = cs[o.b_t + t];
  for (uint32_t j = 0; j < p->K; ++j) acc += cs[o.a_tj + (uint64_t)t * p->K + j] * (uint64_t)h[t * p->K + j];
  return (uint32_t)(acc >> (64 - p->log2_buckets));
}

static int row_ok(const oracle_params* p, const int32_t* idx, uint64_t nnz) {
  if (nnz == 0) return 0;
  for (uint64_t e = 0; e < nnz; ++e)
    if (idx[e] < 0 || (uint32_t)idx[e] >= p->dim) return 0;
  return 1;
}

/* Bucket ids [rows][L] (and optionally the densified DOPH values [rows][M])
 * of rows [row_begin, row_end) of a CSR matrix. */
EXPORT int oracle_hash_rows(const oracle_params* p, const uint64_t* cs, const int64_t* indptr,
                            const int32_t* indices, uint64_t row_begin, uint64_t row_end,
                            uint32_t* buckets, uint32_t* hvals) {
  if (!params_ok(p) || !cs || !indptr || !indices || !buckets) return O_EINVAL;
  uint32_t M = p->K * p->L;
  uint32_t* m = (uint32_t*)malloc(sizeof(uint32_t) * M);
  uint32_t* h = (uint32_t*)malloc(sizeof(uint32_t) * M);
  if (!m || !h) { free(m); free(h); return O_ENOMEM; }
  int rc = O_OK;
  for (uint64_t r = row_begin; r < row_end; ++r) {
    const int32_t* idx = indices + indptr[r];
    uint64_t nnz = (uint64_t)(indptr[r + 1] - indptr[r]);
    if (!row_ok(p, idx, nnz)) { rc = O_EINVAL; break; }
    doph(p, cs, idx, nnz, m, h);
    for (uint32_t t = 0; t < p->L; ++t) buckets[(r - row_begin) * p->L + t] = bucket_of(p, cs, h, t);
    if (hvals) memcpy(hvals + (r - row_begin) * M, h, sizeof(uint32_t) * M);
  }
  free(m);
  free(h);
  return rc;
}

/* -------------------------------------------------------- reservoirs */

/* Reservoir priority of an id in table t: a bijection of uint32, so no two ids
 * tie.  Keeping the R ids of smallest priority is the order-independent
 * stand-in for the paper's online reservoir sub-sampling of heavy buckets
 * (Section 3, "Avoid Skewed buckets"). */
static uint32_t prio(const oracle_params* p, const uint64_t* cs, uint32_t t, uint32_t id) {
  layout_t o = layout(p);
  uint32_t x = id ^ (uint32_t)cs[o.key_t + t];
  x = x * (uint32_t)cs[o.m1_t + t];
  x ^= x >> 16;
  x = x * (uint32_t)cs[o.m2_t + t];
  x ^= x >> 15;
  return x;
}

EXPORT uint32_t oracle_priority(const oracle_params* p, const uint64_t* cs, uint32_t t, uint32_t id) {
  return prio(p, cs, t, id);
}

typedef struct {
  uint32_t bucket, pri, id;
} item_t;

static int cmp_item(const void* a, const void* b) {
  const item_t* x = (const item_t*)a;
  const item_t* y = (const item_t*)b;
  if (x->bucket != y->bucket) return x->bucket < y->bucket ? -1 : 1;
  if (x->pri != y->pri) return x->pri < y->pri ? -1 : 1;
  return 0;
}

/* Pre-processing (Algorithm 1): every vector x, with id = its row number, is
 * inserted into bucket H_t(x) of each table t.  Each bucket keeps seen = its
 * number of insertions and the R smallest-priority ids, in ascending priority,
 * padded with EMPTY.  Tables: ids[L][2^B][R], seen[L][2^B]. */
EXPORT int oracle_build(const oracle_params* p, const uint64_t* cs, const int64_t* indptr,
                        const int32_t* indices, uint64_t n, uint32_t* ids, uint32_t* seen) {
  if (!params_ok(p) || !cs || !ids || !seen) return O_EINVAL;
  if (n > 0xFFFFFFFEull) return O_ECAPACITY;
  uint64_t nb = 1ull << p->log2_buckets;
  uint32_t* bk = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1) * p->L);
  item_t* it = (item_t*)malloc(sizeof(item_t) * (n ? n : 1));
  if (!bk || !it) { free(bk); free(it); return O_ENOMEM; }
  int rc = n ? oracle_hash_rows(p, cs, indptr, indices, 0, n, bk, NULL) : O_OK;
  if (rc != O_OK) { free(bk); free(it); return rc; }
  for (uint64_t x = 0; x < (uint64_t)p->L * nb * p->R; ++x) ids[x] = EMPTY;
  memset(seen, 0, sizeof(uint32_t) * p->L * nb);
  for (uint32_t t = 0; t < p->L; ++t) {
    for (uint64_t r = 0; r < n; ++r) {
      it[r].bucket = bk[r * p->L + t];
      it[r].pri = prio(p, cs, t, (uint32_t)r);
      it[r].id = (uint32_t)r;
    }
    qsort(it, n, sizeof(item_t), cmp_item);
    uint64_t s = 0;
    while (s < n) {
      uint64_t e = s;
      while (e < n && it[e].bucket == it[s].bucket) ++e;
      uint64_t b = it[s].bucket;
      seen[t * nb + b] = (uint32_t)(e - s);
      for (uint64_t i = s; i < e && i - s < p->R; ++i) ids[(t * nb + b) * p->R + (i - s)] = it[i].id;
      s = e;
    }
  }
  free(bk);
  free(it);
  return O_OK;
}

/* Streaming insertion of new vectors (Section 3.1: fixed-size per-bucket
 * summaries ingest a stream).  New ids are first_id, first_id+1, ... in row
 * order.  Each touched bucket keeps the R smallest-priority ids of its old
 * reservoir and the new ids; seen grows by the number of new ids. */
EXPORT int oracle_insert(const oracle_params* p, const uint64_t* cs, uint32_t* ids, uint32_t* seen,
                         uint32_t first_id, const int64_t* indptr, const int32_t* indices, uint64_t n) {
  if (!params_ok(p) || !cs || !ids || !seen) return O_EINVAL;
  if ((uint64_t)first_id + n > 0xFFFFFFFEull) return O_ECAPACITY;
  if (n == 0) return O_OK;
  uint64_t nb = 1ull << p->log2_buckets;
  uint32_t* bk = (uint32_t*)malloc(sizeof(uint32_t) * n * p->L);
  item_t* it = (item_t*)malloc(sizeof(item_t) * (n + p->R));
  if (!bk || !it) { free(bk); free(it); return O_ENOMEM; }
  int rc = oracle_hash_rows(p, cs, indptr, indices, 0, n, bk, NULL);
  if (rc != O_OK) { free(bk); free(it); return rc; }
  for (uint32_t t = 0; t < p->L; ++t) {
    /* bucket by bucket, in ascending bucket order */
    item_t* nw = (item_t*)malloc(sizeof(item_t) * n);
    for (uint64_t r = 0; r < n; ++r) {
      nw[r].bucket = bk[r * p->L + t];
      nw[r].pri = prio(p, cs, t, first_id + (uint32_t)r);
      nw[r].id = first_id + (uint32_t)r;
    }
    qsort(nw, n, sizeof(item_t), cmp_item);
    uint64_t s = 0;
    while (s < n) {
      uint64_t e = s;
      while (e < n && nw[e].bucket == nw[s].bucket) ++e;
      uint64_t b = nw[s].bucket;
      uint32_t* res = ids + (t * nb + b) * p->R;
      uint32_t* sn = seen + t * nb + b;
      uint32_t fill = *sn < p->R ? *sn : p->R;
      uint64_t m = 0;
      for (uint32_t i = 0; i < fill; ++i) {
        it[m].bucket = 0;
        it[m].pri = prio(p, cs, t, res[i]);
        it[m].id = res[i];
        ++m;
      }
      for (uint64_t i = s; i < e; ++i) {
        it[m] = nw[i];
        it[m].bucket = 0;
        ++m;
      }
      qsort(it, m, sizeof(item_t), cmp_item);
      for (uint32_t i = 0; i < p->R; ++i) res[i] = i < m ? it[i].id : EMPTY;
      *sn += (uint32_t)(e - s);
      s = e;
    }
    free(nw);
  }
  free(bk);
  free(it);
  return O_OK;
}

/* ------------------------------------------------------------- queries */

/* Count-min row hash of candidate id c in row r. */
static uint32_t cm_hash(const oracle_params* p, const uint64_t* cs, uint32_t r, uint32_t c) {
  layout_t o = layout(p);
  if (p->log2_cm_width == 0) return 0;
  return (uint32_t)((cs[o.a_r + r] * (uint64_t)c + cs[o.b_r + r]) >> (64 - p->log2_cm_width));
}

typedef struct {
  uint32_t score, id;
} scored_t;

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return (x > y) - (x < y);
}

static int cmp_scored(const void* a, const void* b) {
  const scored_t* x = (const scored_t*)a;
  const scored_t* y = (const scored_t*)b;
  if (x->score != y->score) return x->score > y->score ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

/* Frequency aggregation of one query's candidate multiset cand[0..nc)
 * (Section 2.3 "Cheap Frequency based Filtering"; Section 2.4, Appendix 2):
 * estimate each distinct candidate's frequency with the count-min sketch
 * (min over d rows of w counters) or, when exact != 0, count it exactly, and
 * write the kk best (estimate desc, id asc) into out_ids / out_scores[0..k_max),
 * padded with (EMPTY, 0). */
EXPORT int oracle_aggregate(const oracle_params* p, const uint64_t* cs, const uint32_t* cand, uint64_t nc,
                            uint32_t kk, uint32_t k_max, uint32_t* out_ids, uint32_t* out_scores, int exact) {
  if (!params_ok(p) || !cs || !out_ids || !out_scores || kk > k_max) return O_EINVAL;
  uint64_t w = 1ull << p->log2_cm_width;
  uint32_t* sorted = (uint32_t*)malloc(sizeof(uint32_t) * (nc + 1));
  scored_t* sc = (scored_t*)malloc(sizeof(scored_t) * (nc + 1));
  uint64_t* cm = exact ? NULL : (uint64_t*)malloc(sizeof(uint64_t) * p->cm_rows * w);
  if (!sorted || !sc || (!exact && !cm)) {
    free(sorted);
    free(sc);
    free(cm);
    return O_ENOMEM;
  }
  if (!exact) {
    memset(cm, 0, sizeof(uint64_t) * p->cm_rows * w);
    for (uint64_t i = 0; i < nc; ++i)
      for (uint32_t r = 0; r < p->cm_rows; ++r) cm[r * w + cm_hash(p, cs, r, cand[i])] += 1;
  }
  memcpy(sorted, cand, sizeof(uint32_t) * nc);
  qsort(sorted, nc, sizeof(uint32_t), cmp_u32);
  uint64_t nd = 0;
  for (uint64_t i = 0; i < nc;) {
    uint64_t j = i;
    while (j < nc && sorted[j] == sorted[i]) ++j;
    uint32_t c = sorted[i];
    uint64_t s;
    if (exact) {
      s = j - i;
    } else {
      s = UINT64_MAX;
      for (uint32_t r = 0; r < p->cm_rows; ++r) {
        uint64_t v = cm[r * w + cm_hash(p, cs, r, c)];
        if (v < s) s = v;
      }
    }
    sc[nd].score = (uint32_t)s;
    sc[nd].id = c;
    ++nd;
    i = j;
  }
  qsort(sc, nd, sizeof(scored_t), cmp_scored);
  for (uint32_t i = 0; i < k_max; ++i) {
    int live = i < kk && i < nd;
    out_ids[i] = live ? sc[i].id : EMPTY;
    out_scores[i] = live ? sc[i].score : 0;
  }
  free(sorted);
  free(sc);
  free(cm);
  return O_OK;
}

/* Query (Section 2.3 query phase; Algorithm 2's per-node part): hash the
 * query into its L buckets, take the union (with multiplicity) of the ids they
 * hold, and aggregate (oracle_aggregate).  Output rows have stride k_max. */
EXPORT int oracle_query(const oracle_params* p, const uint64_t* cs, const uint32_t* ids,
                        const uint32_t* seen, const int64_t* qindptr, const int32_t* qindices,
                        uint64_t nq, const uint32_t* kq, uint32_t k, uint32_t k_max,
                        uint32_t* out_ids, uint32_t* out_scores, int exact) {
  if (!params_ok(p) || !cs || !ids || !seen || !out_ids || !out_scores) return O_EINVAL;
  if (k_max == 0) return O_EINVAL;
  uint64_t nb = 1ull << p->log2_buckets;
  uint32_t* bk = (uint32_t*)malloc(sizeof(uint32_t) * p->L);
  uint32_t* cand = (uint32_t*)malloc(sizeof(uint32_t) * ((uint64_t)p->L * p->R + 1));
  int rc = O_OK;
  if (!bk || !cand) rc = O_ENOMEM;
  for (uint64_t q = 0; q < nq && rc == O_OK; ++q) {
    uint32_t kk = kq ? kq[q] : k;
    if (kk > k_max) { rc = O_EINVAL; break; }
    rc = oracle_hash_rows(p, cs, qindptr, qindices, q, q + 1, bk, NULL);
    if (rc != O_OK) break;
    uint64_t nc = 0;
    for (uint32_t t = 0; t < p->L; ++t) {
      uint64_t slot = t * nb + bk[t];
      uint32_t fill = seen[slot] < p->R ? seen[slot] : p->R;
      for (uint32_t i = 0; i < fill; ++i) cand[nc++] = ids[slot * p->R + i];
    }
    rc = oracle_aggregate(p, cs, cand, nc, kk, k_max, out_ids + q * k_max, out_scores + q * k_max, exact);
  }
  free(bk);
  free(cand);
  return rc;
}

/* Priorities of n ids in table t (vector form of oracle_priority). */
EXPORT void oracle_priorities(const oracle_params* p, const uint64_t* cs, uint32_t t,
                              const uint32_t* ids, uint64_t n, uint32_t* out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = prio(p, cs, t, ids[i]);
}

/* ------------------------------------------------- TopKAPI buckets */

/* The paper replaces each bucket by a Topkapi sketch (Section 3.1; Appendix 2
 * "Top-K-API Details"): W rows of C cells, each cell a (heavy hitter, count)
 * pair, empty = (EMPTY, 0).  Here W = cm_rows, C = 2^log2_cm_width, and the
 * row hashes are the count-min row hashes g_r above (one set shared by every
 * bucket of every table, so that any two sketches can be merged).  A sketch
 * is W * C cells of two uint32 words (heavy hitter, count); the tables are
 * cells[L][2^B][W][C][2] and seen[L][2^B].
 *
 * Readings where Appendix 2 is silent: on insertion the empty-or-zero check
 * comes before the match check; two different heavy hitters with equal
 * counts merge to count 0 and the smaller id; the paper's threshold report is
 * read as top-k by count over the heavy hitters of count >= 1, an id held by
 * several rows scoring its largest count, ties by ascending id. */

/* Appendix 2 "Insertion": in every row, the cell g_r(x) takes x with count 1
 * when it is empty or its count is zero, counts up when it holds x, and
 * counts down otherwise. */
static void tk_insert_one(const oracle_params* p, const uint64_t* cs, uint32_t* sk, uint32_t x) {
  uint32_t C = 1u << p->log2_cm_width;
  for (uint32_t r = 0; r < p->cm_rows; ++r) {
    uint32_t* cell = sk + 2 * ((uint64_t)r * C + cm_hash(p, cs, r, x));
    if (cell[0] == EMPTY || cell[1] == 0) {
      cell[0] = x;
      cell[1] = 1;
    } else if (cell[0] == x) {
      cell[1] += 1;
    } else {
      cell[1] -= 1;
    }
  }
}

/* Appendix 2 "Merging": cell by cell, equal heavy hitters add their counts;
 * otherwise the larger count wins and keeps the difference.  dst <- dst (+) src. */
static void tk_merge_cells(uint32_t* dst, const uint32_t* src, uint64_t ncell) {
  for (uint64_t c = 0; c < ncell; ++c) {
    uint32_t h1 = dst[2 * c], c1 = dst[2 * c + 1], h2 = src[2 * c], c2 = src[2 * c + 1];
    if (h1 == h2) {
      dst[2 * c + 1] = c1 + c2;
    } else if (c1 > c2) {
      dst[2 * c + 1] = c1 - c2;
    } else if (c2 > c1) {
      dst[2 * c] = h2;
      dst[2 * c + 1] = c2 - c1;
    } else {
      dst[2 * c] = h1 < h2 ? h1 : h2;
      dst[2 * c + 1] = 0;
    }
  }
}

static uint64_t tk_cells(const oracle_params* p) { return (uint64_t)p->cm_rows << p->log2_cm_width; }

static void tk_clear(uint32_t* sk, uint64_t ncell) {
  for (uint64_t c = 0; c < ncell; ++c) {
    sk[2 * c] = EMPTY;
    sk[2 * c + 1] = 0;
  }
}

/* One sketch of the stream ids[0..n), inserted in the given order. */
EXPORT int oracle_tk_sketch(const oracle_params* p, const uint64_t* cs, const uint32_t* ids, uint64_t n,
                            uint32_t* sk) {
  if (!params_ok(p) || !cs || !sk) return O_EINVAL;
  tk_clear(sk, tk_cells(p));
  for (uint64_t i = 0; i < n; ++i) tk_insert_one(p, cs, sk, ids[i]);
  return O_OK;
}

EXPORT int oracle_tk_merge(const oracle_params* p, uint32_t* dst, const uint32_t* src) {
  if (!params_ok(p) || !dst || !src) return O_EINVAL;
  tk_merge_cells(dst, src, tk_cells(p));
  return O_OK;
}

/* Pre-processing with Topkapi buckets (Algorithm 1 with the sketch insert):
 * ids in ascending order (the row order), each into bucket H_t(x) of every
 * table t. */
EXPORT int oracle_tk_build(const oracle_params* p, const uint64_t* cs, const int64_t* indptr,
                           const int32_t* indices, uint64_t n, uint32_t* cells, uint32_t* seen) {
  if (!params_ok(p) || !cs || !cells || !seen) return O_EINVAL;
  if (n > 0xFFFFFFFEull) return O_ECAPACITY;
  uint64_t nb = 1ull << p->log2_buckets, nc = tk_cells(p);
  for (uint64_t s = 0; s < (uint64_t)p->L * nb; ++s) tk_clear(cells + 2 * nc * s, nc);
  memset(seen, 0, sizeof(uint32_t) * p->L * nb);
  uint32_t* bk = (uint32_t*)malloc(sizeof(uint32_t) * p->L);
  if (!bk) return O_ENOMEM;
  int rc = O_OK;
  for (uint64_t r = 0; r < n && rc == O_OK; ++r) {
    rc = oracle_hash_rows(p, cs, indptr, indices, r, r + 1, bk, NULL);
    for (uint32_t t = 0; t < p->L && rc == O_OK; ++t) {
      uint64_t s = t * nb + bk[t];
      tk_insert_one(p, cs, cells + 2 * nc * s, (uint32_t)r);
      seen[s] += 1;
    }
  }
  free(bk);
  return rc;
}

/* Streaming insertion into Topkapi buckets: new ids first_id, first_id+1, ...
 * in row order, after everything already inserted. */
EXPORT int oracle_tk_insert(const oracle_params* p, const uint64_t* cs, uint32_t* cells, uint32_t* seen,
                            uint32_t first_id, const int64_t* indptr, const int32_t* indices, uint64_t n) {
  if (!params_ok(p) || !cs || !cells || !seen) return O_EINVAL;
  if ((uint64_t)first_id + n > 0xFFFFFFFEull) return O_ECAPACITY;
  uint64_t nb = 1ull << p->log2_buckets, nc = tk_cells(p);
  uint32_t* bk = (uint32_t*)malloc(sizeof(uint32_t) * p->L);
  if (!bk) return O_ENOMEM;
  int rc = O_OK;
  for (uint64_t r = 0; r < n && rc == O_OK; ++r) {
    rc = oracle_hash_rows(p, cs, indptr, indices, r, r + 1, bk, NULL);
    for (uint32_t t = 0; t < p->L && rc == O_OK; ++t) {
      uint64_t s = t * nb + bk[t];
      tk_insert_one(p, cs, cells + 2 * nc * s, first_id + (uint32_t)r);
      seen[s] += 1;
    }
  }
  free(bk);
  return rc;
}

/* Appendix 2 "Querying", read as top-k: every heavy hitter of count >= 1
 * scores its largest count over the cells that hold it; the kk best by
 * (count desc, id asc) go to out_ids / out_scores[0..k_max), padded with
 * (EMPTY, 0). */
EXPORT int oracle_tk_report(const oracle_params* p, const uint32_t* sk, uint32_t kk, uint32_t k_max,
                            uint32_t* out_ids, uint32_t* out_scores) {
  if (!params_ok(p) || !sk || !out_ids || !out_scores || kk > k_max) return O_EINVAL;
  uint64_t nc = tk_cells(p), nd = 0;
  scored_t* sc = (scored_t*)malloc(sizeof(scored_t) * (nc + 1));
  if (!sc) return O_ENOMEM;
  for (uint64_t c = 0; c < nc; ++c) {
    uint32_t h = sk[2 * c], n = sk[2 * c + 1];
    if (h == EMPTY || n == 0) continue;
    uint64_t j = 0;
    while (j < nd && sc[j].id != h) ++j;
    if (j == nd) {
      sc[nd].id = h;
      sc[nd].score = n;
      ++nd;
    } else if (n > sc[j].score) {
      sc[j].score = n;
    }
  }
  qsort(sc, nd, sizeof(scored_t), cmp_scored);
  for (uint32_t i = 0; i < k_max; ++i) {
    int live = i < kk && i < nd;
    out_ids[i] = live ? sc[i].id : EMPTY;
    out_scores[i] = live ? sc[i].score : 0;
  }
  free(sc);
  return O_OK;
}

/* Query with Topkapi buckets (Algorithm 2's per-node part): hash the query,
 * fold the sketches of its L buckets into an empty sketch in table order,
 * S <- Merge(S, T_t(H_t(q))) for t = 0 .. L-1, and report the top-k of S. */
EXPORT int oracle_tk_query(const oracle_params* p, const uint64_t* cs, const uint32_t* cells, const int64_t* qindptr,
                           const int32_t* qindices, uint64_t nq, const uint32_t* kq, uint32_t k, uint32_t k_max,
                           uint32_t* out_ids, uint32_t* out_scores) {
  if (!params_ok(p) || !cs || !cells || !out_ids || !out_scores || k_max == 0) return O_EINVAL;
  uint64_t nb = 1ull << p->log2_buckets, nc = tk_cells(p);
  uint32_t* bk = (uint32_t*)malloc(sizeof(uint32_t) * p->L);
  uint32_t* sk = (uint32_t*)malloc(sizeof(uint32_t) * 2 * nc);
  int rc = (bk && sk) ? O_OK : O_ENOMEM;
  for (uint64_t q = 0; q < nq && rc == O_OK; ++q) {
    uint32_t kk = kq ? kq[q] : k;
    if (kk > k_max) { rc = O_EINVAL; break; }
    rc = oracle_hash_rows(p, cs, qindptr, qindices, q, q + 1, bk, NULL);
    if (rc != O_OK) break;
    tk_clear(sk, nc);
    for (uint32_t t = 0; t < p->L; ++t) tk_merge_cells(sk, cells + 2 * nc * (t * nb + bk[t]), nc);
    rc = oracle_tk_report(p, sk, kk, k_max, out_ids + q * k_max, out_scores + q * k_max);
  }
  free(bk);
  free(sk);
  return rc;
}

/* ------------------------------------------------- quality references */

/* Not part of what the GPU computes: the exact neighbours the method
 * approximates, and the quality measure the paper reports.
 *   - Similarity is Jaccard, |x ∩ y| / |x ∪ y| (Section 2.2; the printed
 *     formula's denominator is read as |x| + |y| - x.y).  A row is a set:
 *     order and repeats inside a row do not count.
 *   - S@k (Section 6, evaluation metrics) is the mean cosine similarity,
 *     |x ∩ y| / sqrt(|x| |y|) for binary vectors, of the returned neighbours
 *     to the query. */

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Sorted copy of a row with repeats dropped; returns its size. */
static uint64_t row_set(const int32_t* idx, uint64_t nnz, int32_t* out) {
  memcpy(out, idx, sizeof(int32_t) * nnz);
  qsort(out, nnz, sizeof(int32_t), cmp_i32);
  uint64_t m = 0;
  for (uint64_t e = 0; e < nnz; ++e)
    if (m == 0 || out[m - 1] != out[e]) out[m++] = out[e];
  return m;
}

/* |a ∩ b| of two sorted sets. */
static uint64_t inter_size(const int32_t* a, uint64_t na, const int32_t* b, uint64_t nb) {
  uint64_t i = 0, j = 0, c = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) {
      ++i;
    } else if (b[j] < a[i]) {
      ++j;
    } else {
      ++c;
      ++i;
      ++j;
    }
  }
  return c;
}

typedef struct {
  uint64_t inter, uni;
  uint32_t id;
} jac_t;

/* Jaccard descending (i1/u1 > i2/u2 compared as i1*u2 > i2*u1, exact), then
 * id ascending. */
static int cmp_jac(const void* a, const void* b) {
  const jac_t* x = (const jac_t*)a;
  const jac_t* y = (const jac_t*)b;
  uint64_t l = x->inter * y->uni, r = y->inter * x->uni;
  if (l != r) return l > r ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

/* Sets of all rows of a CSR matrix, stored back to back; offs[n + 1]. */
static int32_t* csr_sets(const int64_t* indptr, const int32_t* indices, uint64_t n, uint64_t* offs) {
  uint64_t total = (uint64_t)(indptr[n] - indptr[0]);
  int32_t* sets = (int32_t*)malloc(sizeof(int32_t) * (total ? total : 1));
  if (!sets) return NULL;
  offs[0] = 0;
  for (uint64_t r = 0; r < n; ++r) {
    uint64_t nnz = (uint64_t)(indptr[r + 1] - indptr[r]);
    offs[r + 1] = offs[r] + row_set(indices + indptr[r], nnz, sets + offs[r]);
  }
  return sets;
}

/* Brute-force k nearest rows of each query by Jaccard similarity, ties by
 * ascending id (row number).  Output rows of stride k: ids, and the exact
 * similarity as the pair (|x ∩ y|, |x ∪ y|); slots past the data size hold
 * (EMPTY, 0, 0). */
EXPORT int oracle_jaccard_knn(const int64_t* indptr, const int32_t* indices, uint64_t n, const int64_t* qindptr,
                              const int32_t* qindices, uint64_t nq, uint32_t k, uint32_t* out_ids,
                              uint32_t* out_inter, uint32_t* out_union) {
  if (!indptr || !qindptr || !out_ids || !out_inter || !out_union || n > 0xFFFFFFFEull) return O_EINVAL;
  uint64_t* offs = (uint64_t*)malloc(sizeof(uint64_t) * (n + 1));
  jac_t* sc = (jac_t*)malloc(sizeof(jac_t) * (n ? n : 1));
  int32_t* sets = offs ? csr_sets(indptr, indices, n, offs) : NULL;
  int rc = (offs && sc && sets) ? O_OK : O_ENOMEM;
  int32_t* qs = NULL;
  for (uint64_t q = 0; q < nq && rc == O_OK; ++q) {
    uint64_t qn = (uint64_t)(qindptr[q + 1] - qindptr[q]);
    free(qs);
    qs = (int32_t*)malloc(sizeof(int32_t) * (qn ? qn : 1));
    if (!qs) {
      rc = O_ENOMEM;
      break;
    }
    uint64_t qm = row_set(qindices + qindptr[q], qn, qs);
    for (uint64_t r = 0; r < n; ++r) {
      uint64_t xm = offs[r + 1] - offs[r];
      uint64_t in = inter_size(qs, qm, sets + offs[r], xm);
      sc[r].inter = in;
      sc[r].uni = qm + xm - in;
      sc[r].id = (uint32_t)r;
    }
    qsort(sc, n, sizeof(jac_t), cmp_jac);
    for (uint32_t i = 0; i < k; ++i) {
      int live = i < n;
      out_ids[q * k + i] = live ? sc[i].id : EMPTY;
      out_inter[q * k + i] = live ? (uint32_t)sc[i].inter : 0;
      out_union[q * k + i] = live ? (uint32_t)sc[i].uni : 0;
    }
  }
  free(qs);
  free(offs);
  free(sc);
  free(sets);
  return rc;
}

/* S@k terms per query: the mean cosine similarity between query q and the
 * rows ids[q * stride + 0 .. k) that are not EMPTY (out_mean[q]; 0 when none
 * is), and how many there were (out_count[q]).  The caller averages over
 * queries. */
EXPORT int oracle_mean_cosine(const int64_t* indptr, const int32_t* indices, uint64_t n, const int64_t* qindptr,
                              const int32_t* qindices, uint64_t nq, const uint32_t* ids, uint32_t stride, uint32_t k,
                              double* out_mean, uint32_t* out_count) {
  if (!indptr || !qindptr || !ids || !out_mean || !out_count || k > stride) return O_EINVAL;
  int rc = O_OK;
  for (uint64_t q = 0; q < nq && rc == O_OK; ++q) {
    uint64_t qn = (uint64_t)(qindptr[q + 1] - qindptr[q]);
    int32_t* qs = (int32_t*)malloc(sizeof(int32_t) * (qn ? qn : 1));
    if (!qs) {
      rc = O_ENOMEM;
      break;
    }
    uint64_t qm = row_set(qindices + qindptr[q], qn, qs);
    double sum = 0.0;
    uint32_t cnt = 0;
    for (uint32_t i = 0; i < k && rc == O_OK; ++i) {
      uint32_t id = ids[q * stride + i];
      if (id == EMPTY) continue;
      if (id >= n) {
        rc = O_EINVAL;
        break;
      }
      uint64_t xn = (uint64_t)(indptr[id + 1] - indptr[id]);
      int32_t* xs = (int32_t*)malloc(sizeof(int32_t) * (xn ? xn : 1));
      if (!xs) {
        rc = O_ENOMEM;
        break;
      }
      uint64_t xm = row_set(indices + indptr[id], xn, xs);
      uint64_t in = inter_size(qs, qm, xs, xm);
      sum += (double)in / sqrt((double)qm * (double)xm);
      ++cnt;
      free(xs);
    }
    free(qs);
    out_mean[q] = cnt ? sum / cnt : 0.0;
    out_count[q] = cnt;
  }
  return rc;
}
