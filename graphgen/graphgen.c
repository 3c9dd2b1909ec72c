/*
 * graphgen.c -- seeded synthetic input graphs shared by the GPU library's
 * tests/benchmarks and by the CPU oracle.
 *
 * This module holds no triangle-counting arithmetic: it only draws edges and
 * turns an edge multiset into a simple undirected graph stored as a symmetric
 * CSR (rows sorted, no self-loops, no duplicates).
 *
 * Random numbers: counter-based SplitMix64 (Steele, Lea, Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014).  The k-th draw of
 * stream s is mix(s + (k+1)*GAMMA) where mix is the SplitMix64 finaliser, so
 * any draw can be computed independently and generation parallelises without
 * changing the result.
 *
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): each sample descends
 * `scale` levels, choosing quadrant (0,0),(0,1),(1,0),(1,1) with
 * probabilities a,b,c,d.  Thresholds are compared as 32-bit integers, two
 * levels per 64-bit draw.  No noise, no vertex permutation.
 *
 * Erdos-Renyi G(n,p) (Batagelj and Brandes, "Efficient generation of large
 * random networks", Phys. Rev. E 71, 2005): geometric skipping over the
 * pairs (v,w), w<v, of each row v; each row has its own counter stream, which
 * keeps the result exact G(n,p) and independent of thread count.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t gg_draw(uint64_t stream, uint64_t k) {
  return gg_mix(stream + (k + 1) * GG_GAMMA);
}

/* ------------------------------------------------------------------ R-MAT */
typedef struct {
  int scale;
  uint64_t stream;
  uint32_t ta, tab, tabc; /* cumulative thresholds a, a+b, a+b+c scaled by 2^32 */
} rmat_spec;

static inline uint32_t thr32(double x) {
  if (x <= 0.0) return 0u;
  if (x >= 1.0) return 0xFFFFFFFFu;
  return (uint32_t)(x * 4294967296.0);
}

static void rmat_init(rmat_spec* s, int scale, double a, double b, double c, uint64_t seed) {
  s->scale = scale;
  s->stream = gg_mix(seed ^ 0x52A4D47ULL);
  s->ta = thr32(a);
  s->tab = thr32(a + b);
  s->tabc = thr32(a + b + c);
}

static inline void rmat_sample(const rmat_spec* s, uint64_t e, int32_t* pu, int32_t* pv) {
  const int L = s->scale;
  const uint64_t draws = (uint64_t)((L + 1) / 2);
  uint32_t u = 0, v = 0;
  for (int l = 0; l < L; ++l) {
    uint64_t r = gg_draw(s->stream, e * draws + (uint64_t)(l >> 1));
    uint32_t x = (l & 1) ? (uint32_t)(r >> 32) : (uint32_t)r;
    uint32_t bu, bv;
    if (x < s->ta) { bu = 0; bv = 0; }
    else if (x < s->tab) { bu = 0; bv = 1; }
    else if (x < s->tabc) { bu = 1; bv = 0; }
    else { bu = 1; bv = 1; }
    u = (u << 1) | bu;
    v = (v << 1) | bv;
  }
  *pu = (int32_t)u;
  *pv = (int32_t)v;
}

/* Raw R-MAT sample list (with duplicates and self-loops), for small graphs. */
int gg_rmat_edges(int scale, int64_t ne, double a, double b, double c, uint64_t seed,
                  int32_t* src, int32_t* dst) {
  if (scale < 1 || scale > 30 || ne < 0) return -1;
  rmat_spec s;
  rmat_init(&s, scale, a, b, c, seed);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < ne; ++e) rmat_sample(&s, (uint64_t)e, &src[e], &dst[e]);
  return 0;
}

/* ------------------------------------------------------------ Erdos-Renyi */
typedef struct {
  int64_t n;
  double p, lq; /* lq = log(1-p) */
  uint64_t stream;
} er_spec;

static void er_init(er_spec* s, int64_t n, double p, uint64_t seed) {
  s->n = n;
  s->p = p;
  s->lq = log1p(-p);
  s->stream = gg_mix(seed ^ 0xE7D05ULL);
}

/* Calls out for every pair (v,w), w<v, drawn for row v.  Returns row count. */
static inline int64_t er_row(const er_spec* s, int64_t v, int32_t* out) {
  if (s->p <= 0.0 || v == 0) return 0;
  int64_t cnt = 0;
  if (s->p >= 1.0) {
    for (int64_t w = 0; w < v; ++w) { if (out) out[cnt] = (int32_t)w; ++cnt; }
    return cnt;
  }
  uint64_t rs = gg_mix(s->stream + (uint64_t)v * GG_GAMMA);
  int64_t w = -1;
  for (uint64_t k = 0;; ++k) {
    uint64_t r = gg_draw(rs, k);
    double x = ((double)(r >> 11) + 1.0) * (1.0 / 9007199254740992.0); /* (0,1] */
    double skip = floor(log(x) / s->lq);
    if (skip >= (double)v) break;
    w += 1 + (int64_t)skip;
    if (w >= v) break;
    if (out) out[cnt] = (int32_t)w;
    ++cnt;
  }
  return cnt;
}

/* Number of raw ER pairs, then the pairs themselves (rows in order). */
int64_t gg_er_count(int64_t n, double p, uint64_t seed) {
  er_spec s;
  er_init(&s, n, p, seed);
  int64_t tot = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : tot)
  for (int64_t v = 0; v < n; ++v) tot += er_row(&s, v, NULL);
  return tot;
}

int gg_er_edges(int64_t n, double p, uint64_t seed, int64_t ne, int32_t* src, int32_t* dst) {
  er_spec s;
  er_init(&s, n, p, seed);
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!off) return -2;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) off[v + 1] = er_row(&s, v, NULL);
  off[0] = 0;
  for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
  if (off[n] != ne) { free(off); return -1; }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    int64_t c = er_row(&s, v, dst + off[v]);
    for (int64_t t = 0; t < c; ++t) src[off[v] + t] = (int32_t)v;
  }
  free(off);
  return 0;
}

/* ------------------------------------------------- simple symmetric CSR */
/*
 * Two passes over an edge source: pass 0 counts both directions of every
 * non-loop pair, pass 1 scatters them.  Rows are then sorted, deduplicated
 * and compacted in place.  The result does not depend on thread count.
 */
typedef struct {
  int kind; /* 0 = explicit arrays, 1 = rmat, 2 = er */
  int64_t n, ne;
  const int32_t *src, *dst;
  rmat_spec rm;
  er_spec er;
} edge_source;

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

static inline void add_pair(int pass, int64_t* cnt, int32_t* col, int32_t u, int32_t v) {
  if (u == v) return;
  if (pass == 0) {
    __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
  } else {
    int64_t pu = __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
    int64_t pv = __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
    col[pu] = v;
    col[pv] = u;
  }
}

static void source_pass(const edge_source* s, int pass, int64_t* cnt, int32_t* col) {
  if (s->kind == 0) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < s->ne; ++e) add_pair(pass, cnt, col, s->src[e], s->dst[e]);
  } else if (s->kind == 1) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < s->ne; ++e) {
      int32_t u, v;
      rmat_sample(&s->rm, (uint64_t)e, &u, &v);
      add_pair(pass, cnt, col, u, v);
    }
  } else {
#pragma omp parallel
    {
      int32_t* buf = NULL;
      int64_t cap = 0;
#pragma omp for schedule(dynamic, 4096)
      for (int64_t v = 0; v < s->n; ++v) {
        int64_t c = er_row(&s->er, v, NULL);
        if (c == 0) continue;
        if (c > cap) {
          free(buf);
          cap = c * 2;
          buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
        }
        er_row(&s->er, v, buf);
        for (int64_t t = 0; t < c; ++t) add_pair(pass, cnt, col, (int32_t)v, buf[t]);
      }
      free(buf);
    }
  }
}

/*
 * Builds the CSR into caller memory: rowptr holds n+1 int64, col holds `cap`
 * int32 (at least twice the number of raw pairs).  Returns the number of
 * entries kept, or a negative error code.
 */
/* Large builds report each finished phase on stderr (they take minutes). */
static void phase_done(const edge_source* s, const char* what, double t0) {
  if (s->n >= (1LL << 25)) {
    fprintf(stderr, "graphgen: n=%lld %s after %.1f s\n", (long long)s->n, what, omp_get_wtime() - t0);
    fflush(stderr);
  }
}

static int64_t build_csr(const edge_source* s, int64_t* rowptr, int32_t* col, int64_t cap) {
  const int64_t n = s->n;
  const double t0 = omp_get_wtime();
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -2;
  source_pass(s, 0, cnt, NULL);
  phase_done(s, "pairs counted", t0);
  int64_t tot = 0;
  for (int64_t x = 0; x < n; ++x) { int64_t c = cnt[x]; cnt[x] = tot; rowptr[x] = tot; tot += c; }
  rowptr[n] = tot;
  if (tot > cap) { free(cnt); return -3; }
  source_pass(s, 1, cnt, col);
  phase_done(s, "pairs placed", t0);
  /* sort + unique each row; record new lengths in cnt */
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t x = 0; x < n; ++x) {
    int64_t b = rowptr[x], e = rowptr[x + 1];
    int64_t len = e - b;
    if (len > 1) qsort(col + b, (size_t)len, sizeof(int32_t), cmp_i32);
    int64_t w = 0;
    for (int64_t t = 0; t < len; ++t)
      if (w == 0 || col[b + t] != col[b + w - 1]) col[b + w++] = col[b + t];
    cnt[x] = w;
  }
  phase_done(s, "rows sorted", t0);
  /* compact in place: new offsets never exceed old ones */
  int64_t pos = 0;
  for (int64_t x = 0; x < n; ++x) {
    int64_t b = rowptr[x], len = cnt[x];
    if (pos != b && len > 0) memmove(col + pos, col + b, sizeof(int32_t) * (size_t)len);
    rowptr[x] = pos;
    pos += len;
  }
  rowptr[n] = pos;
  free(cnt);
  return pos;
}

int64_t gg_csr_from_edges(int64_t n, int64_t ne, const int32_t* src, const int32_t* dst,
                          int64_t* rowptr, int32_t* col, int64_t cap) {
  for (int64_t e = 0; e < ne; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
  edge_source s;
  memset(&s, 0, sizeof s);
  s.kind = 0; s.n = n; s.ne = ne; s.src = src; s.dst = dst;
  return build_csr(&s, rowptr, col, cap);
}

int64_t gg_rmat_csr(int scale, int64_t ne, double a, double b, double c, uint64_t seed,
                    int64_t* rowptr, int32_t* col, int64_t cap) {
  if (scale < 1 || scale > 30 || ne < 0) return -1;
  edge_source s;
  memset(&s, 0, sizeof s);
  s.kind = 1; s.n = (int64_t)1 << scale; s.ne = ne;
  rmat_init(&s.rm, scale, a, b, c, seed);
  return build_csr(&s, rowptr, col, cap);
}

int64_t gg_er_csr(int64_t n, double p, uint64_t seed, int64_t* rowptr, int32_t* col, int64_t cap) {
  if (n < 0 || n > 2147483647LL || !(p >= 0.0 && p <= 1.0)) return -1;
  edge_source s;
  memset(&s, 0, sizeof s);
  s.kind = 2; s.n = n;
  er_init(&s.er, n, p, seed);
  return build_csr(&s, rowptr, col, cap);
}

int gg_max_threads(void) { return omp_get_max_threads(); }
