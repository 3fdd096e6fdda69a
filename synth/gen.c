/*
 * Seeded synthetic inputs: sparse matrices (CSR, raw integer values) and
 * dense vectors. This file holds no modular arithmetic of the method: values
 * are emitted raw (negative, zero, +-1 or any int64) and every consumer
 * reduces them itself.
 *
 * Randomness is counter based: rnd(key, ctr) is the splitmix64 output
 * function (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) applied to key + (ctr+1)*golden. Every row has
 * its own key, so any row range can be generated on its own, in parallel,
 * and the result does not depend on the thread count.
 *
 * Bounded integers use the multiply-high mapping of Lemire ("Fast random
 * integer generation in an interval", TOMACS 2019) without the rejection
 * step; the bias (< range / 2^64) is irrelevant for synthetic workloads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t rnd(uint64_t key, uint64_t ctr) { return mix64(key + (ctr + 1) * GOLDEN); }
static inline uint64_t subkey(uint64_t key, uint64_t tag) { return mix64(key ^ mix64(tag * GOLDEN + 0x632BE59BD9B4E019ULL)); }
/* uniform integer in [0, n) for 1 <= n <= 2^63 */
static inline uint64_t below(uint64_t r, uint64_t n) { return (uint64_t)(((unsigned __int128)r * n) >> 64); }
static inline double unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* ---- specification ------------------------------------------------------ */
enum { LEN_FIXED = 0, LEN_UNIFORM = 1, LEN_ZIPF = 2, LEN_BIMODAL = 3 };
enum { COL_UNIFORM = 0, COL_LIVE = 1, COL_BANDED = 2, COL_BLOCKDIAG = 3 };

typedef struct {
  int64_t nrows, ncols;
  uint64_t seed;
  /* row-length law (ignored by COL_BANDED) */
  int32_t len_kind;
  int32_t len_a, len_b, len_c, len_d; /* fixed: a; uniform: [a,b]; zipf: [a,b]; bimodal: [a,b] w.p. p else [c,d] */
  double len_alpha, len_p;
  /* column law */
  int32_t col_kind;
  int32_t band_lo, band_hi; /* COL_BANDED: offsets j-i in [lo,hi]; others: diagonals overlaid when lo <= hi */
  int64_t ndead;            /* COL_LIVE: number of columns no row uses */
  int64_t block;            /* COL_BLOCKDIAG: block size */
  /* value law: +-1 (fair sign) w.p. p_pm1, else uniform in [val_lo, val_hi] */
  double p_pm1;
  int64_t val_lo, val_hi;
} synth_spec;

typedef struct {
  const synth_spec* s;
  uint64_t k_len, k_col, k_val;
  double* zcdf; /* zipf cumulative table over [len_a, len_b] */
  int64_t* live; /* COL_LIVE: sorted live columns */
  int64_t nlive;
  int64_t cap;  /* buffer capacity per row */
} ctx_t;

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}
static int64_t uniq(int64_t* b, int64_t n) {
  if (n == 0) return 0;
  qsort(b, (size_t)n, sizeof(int64_t), cmp_i64);
  int64_t w = 1;
  for (int64_t i = 1; i < n; ++i)
    if (b[i] != b[w - 1]) b[w++] = b[i];
  return w;
}

static int64_t max_len(const synth_spec* s) {
  int64_t L = 0;
  switch (s->len_kind) {
    case LEN_FIXED: L = s->len_a; break;
    case LEN_UNIFORM: case LEN_ZIPF: L = s->len_b; break;
    case LEN_BIMODAL: L = s->len_b > s->len_d ? s->len_b : s->len_d; break;
  }
  if (s->col_kind == COL_BANDED) L = (int64_t)s->band_hi - s->band_lo + 1;
  else if (s->band_hi >= s->band_lo) L += (int64_t)s->band_hi - s->band_lo + 1;
  return L < 1 ? 1 : L;
}

static int ctx_init(ctx_t* c, const synth_spec* s) {
  memset(c, 0, sizeof(*c));
  c->s = s;
  c->k_len = subkey(s->seed, 1);
  c->k_col = subkey(s->seed, 2);
  c->k_val = subkey(s->seed, 3);
  c->cap = 2 * max_len(s) + 8;
  if (s->len_kind == LEN_ZIPF) {
    int64_t n = (int64_t)s->len_b - s->len_a + 1;
    if (n < 1) return -1;
    c->zcdf = (double*)malloc(sizeof(double) * (size_t)n);
    if (!c->zcdf) return -1;
    double acc = 0;
    for (int64_t k = 0; k < n; ++k) { acc += pow((double)(s->len_a + k), -s->len_alpha); c->zcdf[k] = acc; }
    for (int64_t k = 0; k < n; ++k) c->zcdf[k] /= acc;
  }
  if (s->col_kind == COL_LIVE) {
    int64_t nd = s->ndead;
    if (nd < 0 || nd >= s->ncols) return -1;
    int64_t* dead = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * nd + 8));
    if (!dead) return -1;
    uint64_t kd = subkey(s->seed, 4), ctr = 0;
    int64_t cnt = 0;
    while (cnt < nd) {
      int64_t need = nd - cnt;
      for (int64_t t = 0; t < need; ++t) dead[cnt + t] = (int64_t)below(rnd(kd, ctr++), (uint64_t)s->ncols);
      cnt = uniq(dead, cnt + need);
    }
    c->nlive = s->ncols - nd;
    c->live = (int64_t*)malloc(sizeof(int64_t) * (size_t)(c->nlive + 1));
    if (!c->live) { free(dead); return -1; }
    int64_t w = 0, d = 0;
    for (int64_t j = 0; j < s->ncols; ++j) {
      if (d < nd && dead[d] == j) { ++d; continue; }
      c->live[w++] = j;
    }
    free(dead);
  }
  return 0;
}
static void ctx_free(ctx_t* c) { free(c->zcdf); free(c->live); }

static int64_t row_len(const ctx_t* c, int64_t i) {
  const synth_spec* s = c->s;
  uint64_t k = subkey(c->k_len, (uint64_t)i);
  switch (s->len_kind) {
    case LEN_FIXED: return s->len_a;
    case LEN_UNIFORM: return s->len_a + (int64_t)below(rnd(k, 0), (uint64_t)(s->len_b - s->len_a + 1));
    case LEN_ZIPF: {
      double u = unit(rnd(k, 0));
      int64_t lo = 0, hi = (int64_t)s->len_b - s->len_a; /* first index with cdf > u */
      while (lo < hi) { int64_t mid = (lo + hi) / 2; if (c->zcdf[mid] > u) hi = mid; else lo = mid + 1; }
      return s->len_a + lo;
    }
    case LEN_BIMODAL:
      if (unit(rnd(k, 0)) < s->len_p) return s->len_a + (int64_t)below(rnd(k, 1), (uint64_t)(s->len_b - s->len_a + 1));
      return s->len_c + (int64_t)below(rnd(k, 1), (uint64_t)(s->len_d - s->len_c + 1));
  }
  return 0;
}

/* r distinct uniform draws from [0, range), sorted; buf capacity >= 2r */
static int64_t draw_distinct(uint64_t key, int64_t r, int64_t range, int64_t* buf) {
  if (r > range) r = range;
  uint64_t ctr = 0;
  int64_t cnt = 0;
  while (cnt < r) {
    int64_t need = r - cnt;
    for (int64_t t = 0; t < need; ++t) buf[cnt + t] = (int64_t)below(rnd(key, ctr++), (uint64_t)range);
    cnt = uniq(buf, cnt + need);
  }
  return cnt;
}

/* the sorted distinct columns of row i; returns the row length */
static int64_t gen_row(const ctx_t* c, int64_t i, int64_t* buf) {
  const synth_spec* s = c->s;
  uint64_t kc = subkey(c->k_col, (uint64_t)i);
  int64_t n = 0;
  if (s->col_kind == COL_BANDED) {
    for (int64_t d = s->band_lo; d <= s->band_hi; ++d) {
      int64_t j = i + d;
      if (j >= 0 && j < s->ncols) buf[n++] = j;
    }
    return n;
  }
  int64_t r = row_len(c, i);
  switch (s->col_kind) {
    case COL_UNIFORM: n = draw_distinct(kc, r, s->ncols, buf); break;
    case COL_LIVE:
      n = draw_distinct(kc, r, c->nlive, buf);
      for (int64_t t = 0; t < n; ++t) buf[t] = c->live[buf[t]];
      break;
    case COL_BLOCKDIAG: {
      int64_t b0 = (i / s->block) * s->block;
      int64_t b1 = b0 + s->block; if (b1 > s->ncols) b1 = s->ncols;
      if (b0 >= s->ncols) { n = 0; break; }
      n = draw_distinct(kc, r, b1 - b0, buf);
      for (int64_t t = 0; t < n; ++t) buf[t] += b0;
      break;
    }
  }
  if (s->band_hi >= s->band_lo) {
    for (int64_t d = s->band_lo; d <= s->band_hi; ++d) {
      int64_t j = i + d;
      if (j >= 0 && j < s->ncols) buf[n++] = j;
    }
    n = uniq(buf, n);
  }
  return n;
}

static int64_t gen_val(const ctx_t* c, int64_t i, int64_t pos) {
  const synth_spec* s = c->s;
  uint64_t kv = subkey(c->k_val, (uint64_t)i);
  uint64_t r0 = rnd(kv, 2 * (uint64_t)pos), r1 = rnd(kv, 2 * (uint64_t)pos + 1);
  if (s->p_pm1 > 0 && unit(r0) < s->p_pm1) return (r1 >> 63) ? -1 : 1;
  uint64_t span = (uint64_t)(s->val_hi - s->val_lo) + 1; /* val_hi - val_lo < 2^63 */
  return s->val_lo + (int64_t)below(r1, span);
}

/* Row lengths of rows [r0, r1). Returns their total, or -1 on a bad spec. */
int64_t synth_count(const synth_spec* s, int64_t r0, int64_t r1, int64_t* rowlen) {
  ctx_t c;
  if (r0 < 0 || r1 > s->nrows || r0 > r1) return -1;
  if (ctx_init(&c, s)) { ctx_free(&c); return -1; }
  int64_t total = 0;
#pragma omp parallel reduction(+ : total)
  {
    int64_t* buf = (int64_t*)malloc(sizeof(int64_t) * (size_t)c.cap);
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = r0; i < r1; ++i) {
      int64_t n = gen_row(&c, i, buf);
      rowlen[i - r0] = n;
      total += n;
    }
    free(buf);
  }
  ctx_free(&c);
  return total;
}

/* Columns and raw values of rows [r0, r1); rowptr has r1-r0+1 entries and
 * rowptr[0] may be nonzero (entries are written at rowptr[i-r0]). */
int synth_fill(const synth_spec* s, int64_t r0, int64_t r1, const int64_t* rowptr, int32_t* col, int64_t* val) {
  ctx_t c;
  if (r0 < 0 || r1 > s->nrows || r0 > r1 || s->ncols > 2147483647LL) return -1;
  if (ctx_init(&c, s)) { ctx_free(&c); return -1; }
  int bad = 0;
#pragma omp parallel reduction(| : bad)
  {
    int64_t* buf = (int64_t*)malloc(sizeof(int64_t) * (size_t)c.cap);
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = r0; i < r1; ++i) {
      int64_t n = gen_row(&c, i, buf);
      int64_t base = rowptr[i - r0];
      if (n != rowptr[i - r0 + 1] - base) { bad = 1; continue; }
      for (int64_t t = 0; t < n; ++t) {
        col[base + t] = (int32_t)buf[t];
        val[base + t] = gen_val(&c, i, t);
      }
    }
    free(buf);
  }
  ctx_free(&c);
  return bad ? -2 : 0;
}

/* count uniform integers in [lo, hi] (hi - lo < 2^63), keyed by (seed, tag) */
void synth_vector(uint64_t seed, uint64_t tag, int64_t count, int64_t lo, int64_t hi, int64_t* out) {
  uint64_t k = subkey(seed, 0x100 + tag);
  uint64_t span = (uint64_t)(hi - lo) + 1;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < count; ++t) out[t] = lo + (int64_t)below(rnd(k, (uint64_t)t), span);
}

/* count doubles uniform in [0,1), keyed by (seed, tag) */
void synth_unit(uint64_t seed, uint64_t tag, int64_t count, double* out) {
  uint64_t k = subkey(seed, 0x200 + tag);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < count; ++t) out[t] = unit(rnd(k, (uint64_t)t));
}

/* the raw 64-bit stream itself, for tests of the generator */
void synth_raw(uint64_t key, int64_t count, uint64_t* out) {
  for (int64_t t = 0; t < count; ++t) out[t] = rnd(key, (uint64_t)t);
}
