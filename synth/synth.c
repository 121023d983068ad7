/*
 * Seeded synthetic workload generator (input side only).
 *
 * This module produces the inputs that both the plain CPU oracle and the GPU
 * library consume: binary sparse vectors in CSR form, perturbed queries with a
 * known planted neighbour, and request arrival traces.  It holds none of the
 * similarity-search method's arithmetic.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), used as a counter-based generator.
 * Every row / query / request is a pure function of (stream key, its own
 * counter), so any row can be regenerated on its own, in any order and on any
 * number of threads, with identical results.
 *
 * Workload shapes follow the paper's evaluation data (Criteo-like rows:
 * ~1M features, ~40 nonzeros, skewed feature popularity; Webspam-like width
 * for the wide case): Section 6, Table 1.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

/* ---------------------------------------------------------------- Philox */

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static inline void philox4x32_10(const uint32_t in[4], uint32_t k0, uint32_t k1,
                                 uint32_t out[4]) {
  uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

EXPORT void synth_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox4x32_10(ctr, key[0], key[1], out);
}

/* A stream of 64-bit draws for one (key, counter-owner, tag): draw j uses
 * Philox block j/2, half j%2. */
typedef struct {
  uint32_t k0, k1;
  uint64_t owner;
  uint32_t tag;
  uint32_t blk;  /* block index held in buf, or UINT32_MAX */
  uint32_t buf[4];
} stream_t;

static inline void stream_init(stream_t* s, uint64_t key, uint64_t owner, uint32_t tag) {
  s->k0 = (uint32_t)key;
  s->k1 = (uint32_t)(key >> 32);
  s->owner = owner;
  s->tag = tag;
  s->blk = UINT32_MAX;
}

static inline uint64_t stream_draw(stream_t* s, uint32_t j) {
  uint32_t b = j >> 1;
  if (b != s->blk) {
    uint32_t ctr[4] = {(uint32_t)s->owner, (uint32_t)(s->owner >> 32), s->tag, b};
    philox4x32_10(ctr, s->k0, s->k1, s->buf);
    s->blk = b;
  }
  return (j & 1) ? (((uint64_t)s->buf[3] << 32) | s->buf[2])
                 : (((uint64_t)s->buf[1] << 32) | s->buf[0]);
}

static inline double u53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }
/* floor(x * n / 2^64): uniform integer in [0, n) */
static inline uint64_t mulhi64(uint64_t x, uint64_t n) {
  return (uint64_t)(((unsigned __int128)x * n) >> 64);
}

/* Derive an independent 64-bit stream key from a master seed and a tag. */
EXPORT uint64_t synth_derive(uint64_t master, uint32_t tag) {
  uint32_t ctr[4] = {tag, 0x5EEDu, 0xD1CEu, 0x0u}, o[4];
  philox4x32_10(ctr, (uint32_t)master, (uint32_t)(master >> 32), o);
  return ((uint64_t)o[1] << 32) | o[0];
}

/* ------------------------------------------------------------ row spec */

enum { TAG_NNZ = 1, TAG_IDX = 2, TAG_SRC = 11, TAG_NQ = 12, TAG_F = 13, TAG_K = 14,
       TAG_TRIM = 15, TAG_EXT = 16, TAG_POS = 17, TAG_FRESH = 18,
       TAG_ARR = 21, TAG_KIND = 22, TAG_ISZ = 23 };

typedef struct {
  uint64_t key;       /* data stream key */
  uint32_t dim;       /* number of features D */
  uint32_t index_kind;/* 0 = Zipf(s) over ranks 1..D (index = rank-1), 1 = uniform */
  double zipf_s;
  uint32_t nnz_kind;  /* 0 = Poisson(a), 1 = lognormal(median a, sigma b) */
  double nnz_a, nnz_b;
  uint32_t nnz_lo, nnz_hi; /* clip range (inclusive); lo >= 1 */
} synth_rows_spec;

typedef struct {
  synth_rows_spec s;
  /* Zipf alias table (Walker / Vose), one 64-bit entry per column:
   * low 32 bits = acceptance threshold in 2^-32 units, high 32 bits = alias
   * (alias == column when the column is always accepted). */
  uint64_t* tab;
  /* Poisson inverse-CDF table */
  double* pcdf;
  uint32_t pcdf_n;
} synth_ctx;

EXPORT void synth_ctx_free(synth_ctx* c) {
  if (!c) return;
  free(c->tab);
  free(c->pcdf);
  free(c);
}

EXPORT synth_ctx* synth_ctx_new(const synth_rows_spec* spec) {
  if (!spec || spec->dim == 0 || spec->nnz_lo == 0 || spec->nnz_hi < spec->nnz_lo) return NULL;
  synth_ctx* c = (synth_ctx*)calloc(1, sizeof(synth_ctx));
  c->s = *spec;
  if (c->s.nnz_hi > c->s.dim) c->s.nnz_hi = c->s.dim;
  if (c->s.nnz_lo > c->s.nnz_hi) c->s.nnz_lo = c->s.nnz_hi;
  uint32_t D = spec->dim;
  if (spec->index_kind == 0) {
    /* Vose's alias method; work lists are processed in index order so the
     * table is a deterministic function of (D, s). */
    double* sc = (double*)malloc(sizeof(double) * D);
    uint32_t* small = (uint32_t*)malloc(sizeof(uint32_t) * D);
    uint32_t* large = (uint32_t*)malloc(sizeof(uint32_t) * D);
    double* thr = (double*)malloc(sizeof(double) * D);
    uint32_t* alias = (uint32_t*)malloc(sizeof(uint32_t) * D);
    double z = 0.0;
    for (uint32_t k = 0; k < D; ++k) z += pow((double)k + 1.0, -spec->zipf_s);
    uint32_t ns = 0, nl = 0;
    for (uint32_t k = 0; k < D; ++k) {
      sc[k] = pow((double)k + 1.0, -spec->zipf_s) / z * (double)D;
      alias[k] = k;
      if (sc[k] < 1.0) small[ns++] = k; else large[nl++] = k;
    }
    uint32_t is = 0, il = 0; /* FIFO heads */
    /* small/large as FIFO queues; newly-small items are appended to small */
    uint32_t* sq = small; uint32_t sq_end = ns;
    uint32_t* lq = large; uint32_t lq_end = nl;
    /* queues may grow by re-classification; allocate growth room */
    sq = (uint32_t*)realloc(sq, sizeof(uint32_t) * (2 * (size_t)D + 1));
    lq = (uint32_t*)realloc(lq, sizeof(uint32_t) * (2 * (size_t)D + 1));
    while (is < sq_end && il < lq_end) {
      uint32_t l = sq[is++];
      uint32_t g = lq[il];
      double t = sc[l];
      thr[l] = t;
      alias[l] = g;
      sc[g] = (sc[g] + sc[l]) - 1.0;
      if (sc[g] < 1.0) {
        il++;
        sq[sq_end++] = g;
      }
    }
    while (il < lq_end) thr[lq[il++]] = 2.0;
    while (is < sq_end) thr[sq[is++]] = 2.0; /* rounding leftovers */
    c->tab = (uint64_t*)malloc(sizeof(uint64_t) * D);
    for (uint32_t k = 0; k < D; ++k) {
      double t = thr[k] * 4294967296.0;
      if (t >= 4294967295.0) /* always accepted */
        c->tab[k] = ((uint64_t)k << 32) | 0xFFFFFFFFu;
      else
        c->tab[k] = ((uint64_t)alias[k] << 32) | (uint32_t)t;
    }
    free(thr);
    free(alias);
    free(sc);
    free(sq);
    free(lq);
  }
  if (spec->nnz_kind == 0) {
    double lam = spec->nnz_a;
    uint32_t cap = (uint32_t)(lam + 40.0 * sqrt(lam + 1.0) + 64.0);
    c->pcdf = (double*)malloc(sizeof(double) * cap);
    double p = exp(-lam), acc = 0.0;
    uint32_t n = 0;
    for (uint32_t k = 0; k < cap; ++k) {
      if (k) p *= lam / (double)k;
      acc += p;
      c->pcdf[n++] = acc;
    }
    c->pcdf_n = n;
  }
  return c;
}

static inline uint32_t draw_index(const synth_ctx* c, uint64_t x) {
  uint32_t col = (uint32_t)(((x >> 32) * (uint64_t)c->s.dim) >> 32);
  if (c->s.index_kind == 1) return col;
  uint64_t e = c->tab[col];
  return ((uint32_t)x < (uint32_t)e) ? col : (uint32_t)(e >> 32);
}

static uint32_t clip_u32(double v, uint32_t lo, uint32_t hi) {
  if (!(v >= (double)lo)) return lo;
  if (v > (double)hi) return hi;
  return (uint32_t)v;
}

static uint32_t lognormal_count(uint64_t x0, uint64_t x1, double median, double sigma,
                                uint32_t lo, uint32_t hi) {
  double a = ((double)(x0 >> 11) + 1.0) * 0x1.0p-53; /* (0, 1] */
  double b = u53(x1);
  double z = sqrt(-2.0 * log(a)) * cos(6.283185307179586 * b);
  return clip_u32(floor(median * exp(sigma * z) + 0.5), lo, hi);
}

static uint32_t row_nnz(const synth_ctx* c, uint64_t row) {
  stream_t s;
  stream_init(&s, c->s.key, row, TAG_NNZ);
  if (c->s.nnz_kind == 0) {
    double u = u53(stream_draw(&s, 0));
    uint32_t k = 0;
    while (k < c->pcdf_n && !(u < c->pcdf[k])) ++k;
    return clip_u32((double)k, c->s.nnz_lo, c->s.nnz_hi);
  }
  uint64_t x0 = stream_draw(&s, 0), x1 = stream_draw(&s, 1);
  return lognormal_count(x0, x1, c->s.nnz_a, c->s.nnz_b, c->s.nnz_lo, c->s.nnz_hi);
}

/* ------------------------------------------------ small set of uint32 */

typedef struct {
  uint32_t* slot; /* open addressing, EMPTY = UINT32_MAX */
  uint32_t mask;
} uset;

static void uset_reset(uset* h, uint32_t n) {
  uint32_t cap = 64;
  while (cap < 2 * n + 2) cap <<= 1;
  if (!h->slot || h->mask + 1 < cap) {
    free(h->slot);
    h->slot = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    h->mask = cap - 1;
  }
  memset(h->slot, 0xFF, sizeof(uint32_t) * (h->mask + 1));
}

/* returns 1 if inserted (was absent), 0 if already present */
static inline int uset_add(uset* h, uint32_t v) {
  uint32_t i = (v * 0x9E3779B1u) & h->mask;
  for (;;) {
    uint32_t e = h->slot[i];
    if (e == v) return 0;
    if (e == UINT32_MAX) {
      h->slot[i] = v;
      return 1;
    }
    i = (i + 1) & h->mask;
  }
}

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return (x > y) - (x < y);
}

/* Distinct indices for one row: draws j = 0, 1, 2, ... are accepted when not
 * already present, until nnz are accepted.  Indices stay in acceptance order
 * (the method does not depend on the order of a row's indices). */
static void row_fill(const synth_ctx* c, uint64_t row, uint32_t nnz, uint32_t* out, uset* h) {
  stream_t s;
  stream_init(&s, c->s.key, row, TAG_IDX);
  uint32_t got = 0, j = 0;
  if (nnz <= 48) {
    while (got < nnz) {
      uint32_t v = draw_index(c, stream_draw(&s, j++));
      int dup = 0;
      for (uint32_t q = 0; q < got; ++q) dup |= (out[q] == v);
      if (!dup) out[got++] = v;
    }
  } else {
    uset_reset(h, nnz);
    while (got < nnz) {
      uint32_t v = draw_index(c, stream_draw(&s, j++));
      if (uset_add(h, v)) out[got++] = v;
    }
  }
}

/* ------------------------------------------------------ parallel for */

typedef void (*range_fn)(void* arg, uint64_t b, uint64_t e, uset* h);
typedef struct {
  range_fn fn;
  void* arg;
  uint64_t n, chunk;
  uint64_t next; /* atomic */
} pfor_t;

static void* pfor_worker(void* p) {
  pfor_t* f = (pfor_t*)p;
  uset h = {0, 0};
  for (;;) {
    uint64_t b = __atomic_fetch_add(&f->next, f->chunk, __ATOMIC_RELAXED);
    if (b >= f->n) break;
    uint64_t e = b + f->chunk < f->n ? b + f->chunk : f->n;
    f->fn(f->arg, b, e, &h);
  }
  free(h.slot);
  return NULL;
}

static void pfor(uint64_t n, uint64_t chunk, int threads, range_fn fn, void* arg) {
  pfor_t f = {fn, arg, n, chunk ? chunk : 1, 0};
  if (threads <= 1 || n <= chunk) {
    pfor_worker(&f);
    return;
  }
  if (threads > 256) threads = 256;
  pthread_t th[256];
  for (int i = 0; i < threads; ++i) pthread_create(&th[i], NULL, pfor_worker, &f);
  for (int i = 0; i < threads; ++i) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------- rows API */

typedef struct {
  const synth_ctx* c;
  uint64_t row0;
  uint32_t* nnz;
  const int64_t* indptr;
  int32_t* indices;
} rows_job;

static void rows_nnz_fn(void* a, uint64_t b, uint64_t e, uset* h) {
  (void)h;
  rows_job* j = (rows_job*)a;
  for (uint64_t i = b; i < e; ++i) j->nnz[i] = row_nnz(j->c, j->row0 + i);
}

static void rows_fill_fn(void* a, uint64_t b, uint64_t e, uset* h) {
  rows_job* j = (rows_job*)a;
  for (uint64_t i = b; i < e; ++i) {
    int64_t o = j->indptr[i] - j->indptr[0];
    uint32_t n = (uint32_t)(j->indptr[i + 1] - j->indptr[i]);
    row_fill(j->c, j->row0 + i, n, (uint32_t*)(j->indices + o), h);
  }
}

/* nnz of rows [row0, row0+n) */
EXPORT int synth_rows_nnz(const synth_ctx* c, uint64_t row0, uint64_t n, uint32_t* out, int threads) {
  if (!c || !out) return -1;
  rows_job j = {c, row0, out, NULL, NULL};
  pfor(n, 1 << 16, threads, rows_nnz_fn, &j);
  return 0;
}

/* indices of rows [row0, row0+n) into the CSR layout given by indptr[n+1]
 * (indptr[0] is the base offset of indices[0]). */
EXPORT int synth_rows_fill(const synth_ctx* c, uint64_t row0, uint64_t n, const int64_t* indptr,
                           int32_t* indices, int threads) {
  if (!c || !indptr || !indices) return -1;
  rows_job j = {c, row0, NULL, indptr, indices};
  pfor(n, 1 << 14, threads, rows_fill_fn, &j);
  return 0;
}

/* ----------------------------------------------------------- queries API */

typedef struct {
  uint64_t key;       /* query stream key */
  uint64_t n_data;    /* sources are drawn uniformly from rows [0, n_data) */
  uint32_t nnz_mode;  /* 0 = same nnz as the source, 1 = lognormal(median, sigma) clipped */
  double median, sigma;
  uint32_t lo, hi;
  double f_lo, f_hi;  /* replaced fraction f ~ U[f_lo, f_hi] (fixed when equal) */
  uint32_t n_kmix;    /* top-k drawn uniformly from kmix[0..n_kmix) */
  uint32_t kmix[8];
} synth_query_spec;

typedef struct {
  const synth_ctx* c;
  const synth_query_spec* q;
  uint64_t q0;
  uint64_t* src;
  uint32_t* nnz;
  uint32_t* kq;
  const int64_t* indptr;
  int32_t* indices;
  int status;
} q_job;

static uint32_t query_nnz_target(const q_job* j, uint64_t q, uint64_t* src_out, uint32_t* ns_out,
                                 uint32_t* k_out) {
  stream_t s;
  stream_init(&s, j->q->key, q, TAG_SRC);
  uint64_t src = mulhi64(stream_draw(&s, 0), j->q->n_data);
  uint32_t ns = row_nnz(j->c, src);
  uint32_t nq = ns;
  if (j->q->nnz_mode == 1) {
    stream_t t;
    stream_init(&t, j->q->key, q, TAG_NQ);
    uint64_t x0 = stream_draw(&t, 0), x1 = stream_draw(&t, 1);
    nq = lognormal_count(x0, x1, j->q->median, j->q->sigma, j->q->lo, j->q->hi);
    if (nq > j->c->s.dim) nq = j->c->s.dim;
  }
  if (k_out) {
    stream_t t;
    stream_init(&t, j->q->key, q, TAG_K);
    uint32_t n = j->q->n_kmix ? j->q->n_kmix : 1;
    *k_out = j->q->kmix[mulhi64(stream_draw(&t, 0), n)];
  }
  *src_out = src;
  *ns_out = ns;
  return nq;
}

static void q_nnz_fn(void* a, uint64_t b, uint64_t e, uset* h) {
  (void)h;
  q_job* j = (q_job*)a;
  for (uint64_t i = b; i < e; ++i) {
    uint32_t ns;
    j->nnz[i] = query_nnz_target(j, j->q0 + i, &j->src[i], &ns, &j->kq[i]);
  }
}

static void q_fill_fn(void* a, uint64_t b, uint64_t e, uset* h) {
  q_job* j = (q_job*)a;
  uint32_t cap = 0;
  uint32_t* cur = NULL;
  uset h2 = {0, 0};
  for (uint64_t i = b; i < e; ++i) {
    uint64_t q = j->q0 + i, src;
    uint32_t ns;
    uint32_t nq = query_nnz_target(j, q, &src, &ns, NULL);
    uint32_t need = (ns > nq ? ns : nq) * 2 + 8;
    if (need > cap) {
      free(cur);
      cap = need;
      cur = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    }
    row_fill(j->c, src, ns, cur, h);
    uint32_t n = ns;
    /* trim to a uniformly random subset, or extend with fresh draws */
    if (nq < ns) {
      stream_t s;
      stream_init(&s, j->q->key, q, TAG_TRIM);
      for (uint32_t t = 0; t < nq; ++t) {
        uint32_t r = t + (uint32_t)mulhi64(stream_draw(&s, t), ns - t);
        uint32_t tmp = cur[t]; cur[t] = cur[r]; cur[r] = tmp;
      }
      n = nq;
    }
    uset_reset(&h2, nq + 1);
    for (uint32_t t = 0; t < n; ++t) uset_add(&h2, cur[t]);
    if (nq > ns) {
      stream_t s;
      stream_init(&s, j->q->key, q, TAG_EXT);
      uint32_t d = 0;
      while (n < nq) {
        uint32_t v = draw_index(j->c, stream_draw(&s, d++));
        if (uset_add(&h2, v)) cur[n++] = v;
      }
    }
    /* replace round(f * n) uniformly chosen nonzeros with fresh draws not
     * already present (neither kept nor replaced values) */
    stream_t sf;
    stream_init(&sf, j->q->key, q, TAG_F);
    double f = j->q->f_lo + (j->q->f_hi - j->q->f_lo) * u53(stream_draw(&sf, 0));
    uint32_t r = (uint32_t)floor(f * (double)n + 0.5);
    if (r > n) r = n;
    stream_t sp;
    stream_init(&sp, j->q->key, q, TAG_POS);
    for (uint32_t t = 0; t < r; ++t) {
      uint32_t x = t + (uint32_t)mulhi64(stream_draw(&sp, t), n - t);
      uint32_t tmp = cur[t]; cur[t] = cur[x]; cur[x] = tmp;
    }
    stream_t sn;
    stream_init(&sn, j->q->key, q, TAG_FRESH);
    uint32_t d = 0, got = 0;
    uint64_t guard = 0;
    while (got < r) {
      uint32_t v = draw_index(j->c, stream_draw(&sn, d++));
      if (uset_add(&h2, v)) cur[got++] = v; /* overwrite the replaced slots */
      if (++guard > (uint64_t)1 << 34) { j->status = -2; break; }
    }
    qsort(cur, n, sizeof(uint32_t), cmp_u32);
    int64_t o = j->indptr[i] - j->indptr[0];
    memcpy(j->indices + o, cur, sizeof(uint32_t) * n);
  }
  free(cur);
  free(h2.slot);
}

/* Phase 1: per query, its planted source row, its nnz and its top-k. */
EXPORT int synth_queries_nnz(const synth_ctx* c, const synth_query_spec* q, uint64_t q0, uint64_t n,
                             uint64_t* src, uint32_t* nnz, uint32_t* kq, int threads) {
  if (!c || !q || !src || !nnz || !kq || q->n_data == 0) return -1;
  q_job j = {c, q, q0, src, nnz, kq, NULL, NULL, 0};
  pfor(n, 1 << 12, threads, q_nnz_fn, &j);
  return 0;
}

/* Phase 2: indices of queries [q0, q0+n) into the CSR layout indptr[n+1]. */
EXPORT int synth_queries_fill(const synth_ctx* c, const synth_query_spec* q, uint64_t q0, uint64_t n,
                              const int64_t* indptr, int32_t* indices, int threads) {
  if (!c || !q || !indptr || !indices || q->n_data == 0) return -1;
  q_job j = {c, q, q0, NULL, NULL, NULL, indptr, indices, 0};
  pfor(n, 1 << 10, threads, q_fill_fn, &j);
  return j.status;
}

/* --------------------------------------------------------- arrivals API */

/* Open-loop request trace: Poisson arrivals at `rate` per second; each
 * request is an insert with probability insert_frac, with a log-uniform
 * integer size in [ins_lo, ins_hi]; otherwise a query. */
EXPORT int synth_arrivals(uint64_t key, uint64_t n, double rate, double insert_frac, uint32_t ins_lo,
                          uint32_t ins_hi, double* t_arr, uint8_t* is_insert, uint32_t* ins_size) {
  if (rate <= 0 || ins_lo == 0 || ins_hi < ins_lo) return -1;
  double t = 0.0;
  double llo = log((double)ins_lo), lhi = log((double)ins_hi + 1.0);
  for (uint64_t i = 0; i < n; ++i) {
    stream_t s;
    stream_init(&s, key, i, TAG_ARR);
    double u = ((double)(stream_draw(&s, 0) >> 11) + 1.0) * 0x1.0p-53;
    t += -log(u) / rate;
    t_arr[i] = t;
    stream_t k;
    stream_init(&k, key, i, TAG_KIND);
    is_insert[i] = u53(stream_draw(&k, 0)) < insert_frac;
    stream_t z;
    stream_init(&z, key, i, TAG_ISZ);
    uint32_t sz = (uint32_t)floor(exp(llo + (lhi - llo) * u53(stream_draw(&z, 0))));
    if (sz < ins_lo) sz = ins_lo;
    if (sz > ins_hi) sz = ins_hi;
    ins_size[i] = sz;
  }
  return 0;
}

/* Tables of a row law, for the device build of the generator: alias table
 * (D entries, Zipf only) and Poisson inverse CDF (pcdf_n doubles). */
EXPORT void synth_ctx_tables(const synth_ctx* c, const uint64_t** tab, const double** pcdf, uint32_t* pcdf_n,
                             synth_rows_spec* spec) {
  *tab = c->tab;
  *pcdf = c->pcdf;
  *pcdf_n = c->pcdf_n;
  *spec = c->s;
}
