/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU triangle counter used to check the GPU
 * library.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load it; the product path never does.  It shares no code,
 * header or table with the GPU library.
 *
 * What it computes (Yasar et al., "Block-Based Triangle Counting Algorithm
 * for Heterogeneous Environments", arXiv 2009.12457):
 *
 *  - Total: the number of 3-vertex sets of a simple undirected graph whose
 *    three edges are all present (Sec. 2, Definition "Triangle Counting
 *    Problem").  Self-loops are dropped and repeated edges collapsed first.
 *  - Ordering: vertices renumbered in non-decreasing degree order (Sec. 4.1),
 *    ties broken by the original id; every edge is stored once, from the
 *    lower to the higher rank (Sec. 2, N(G,u) = {v : (u,v) in E, u < v}).
 *  - Total, list form: Alg. 2 (TC-Intersect) with the two-pointer count of
 *    Alg. 1.  Alg. 1 as printed compares A[b] with B[b] in its first branch;
 *    the intended comparison is A[a] with B[b], which is what is done here.
 *  - Total, hash form: Alg. 3 (TC-HMap) with a dense stamp array whose
 *    initial value is -1 (the paper leaves the initial value unstated).
 *  - Per-task counts: with a vertex partition into p contiguous rank ranges
 *    V_0..V_{p-1} (Sec. 2, 4.1), a task {i,j,k}, i<=j<=k, covers the blocks
 *    G_ij, G_jk, G_ik (Sec. 4.2, Definition "Task").  A triangle with ranks
 *    a<b<c lies in exactly the task (part(a), part(b), part(c)), so the
 *    per-task count is the number of triangles so classified.  Tasks are
 *    indexed in the order of Alg. 4 (bbTaskComposition).
 *  - Cut rule (the paper's partitioner, PBD, is not described in it; this is
 *    the reading used throughout): c_0 = 0, c_p = n, and for 0<i<p, c_i is
 *    the smallest x > c_{i-1} whose prefix of oriented row lengths reaches
 *    ceil(i*m/p), clamped to at most n-(p-i) so no part is empty.  A uniform
 *    rule c_i = floor(i*n/p) is offered as well.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
  int64_t n, m;      /* ids, undirected simple edges */
  int64_t* deg;      /* undirected degree per original id */
  int32_t* rank;     /* rank of each original id */
  int32_t* vert;     /* original id of each rank */
  int64_t* orow;     /* oriented CSR in rank space, n+1 */
  int32_t* ocol;     /* m entries, rows ascending */
} or_graph;

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

void or_free(or_graph* g) {
  if (!g) return;
  free(g->deg); free(g->rank); free(g->vert); free(g->orow); free(g->ocol);
  free(g);
}

/*
 * Canonicalisation.  Every input pair {x,y}, x != y, is filed under its
 * smaller endpoint; each bucket is sorted and repeats removed.  This is
 * "map to (min,max), sort, unique", done bucket by bucket.
 * Input is either an edge list (src,dst,ne) or a CSR (rowptr,colidx).
 */
static or_graph* build(int64_t n, int64_t ne, const int32_t* src, const int32_t* dst,
                       const int64_t* rowptr, const int32_t* colidx) {
  int use_csr = (rowptr != NULL);
  int64_t* bcnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!bcnt) return NULL;
  if (use_csr) {
    for (int64_t x = 0; x < n; ++x)
      for (int64_t e = rowptr[x]; e < rowptr[x + 1]; ++e) {
        int32_t y = colidx[e];
        if (y < 0 || y >= n) { free(bcnt); return NULL; }
        if (y != x) bcnt[x < y ? x : y]++;
      }
  } else {
    for (int64_t e = 0; e < ne; ++e) {
      int32_t x = src[e], y = dst[e];
      if (x < 0 || x >= n || y < 0 || y >= n) { free(bcnt); return NULL; }
      if (x != y) bcnt[x < y ? x : y]++;
    }
  }
  int64_t* bptr = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  bptr[0] = 0;
  for (int64_t x = 0; x < n; ++x) bptr[x + 1] = bptr[x] + bcnt[x];
  int32_t* hi = (int32_t*)malloc(sizeof(int32_t) * (size_t)(bptr[n] > 0 ? bptr[n] : 1));
  memcpy(bcnt, bptr, sizeof(int64_t) * (size_t)n);
  if (use_csr) {
    for (int64_t x = 0; x < n; ++x)
      for (int64_t e = rowptr[x]; e < rowptr[x + 1]; ++e) {
        int32_t y = colidx[e];
        if (y == x) continue;
        int64_t lo = x < y ? x : y, h = x < y ? y : x;
        hi[bcnt[lo]++] = (int32_t)h;
      }
  } else {
    for (int64_t e = 0; e < ne; ++e) {
      int32_t x = src[e], y = dst[e];
      if (x == y) continue;
      int64_t lo = x < y ? x : y, h = x < y ? y : x;
      hi[bcnt[lo]++] = (int32_t)h;
    }
  }
  /* sort + unique each bucket; bcnt[x] becomes its unique length */
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t x = 0; x < n; ++x) {
    int64_t b = bptr[x], len = bptr[x + 1] - b, w = 0;
    if (len > 1) qsort(hi + b, (size_t)len, sizeof(int32_t), cmp_i32);
    for (int64_t t = 0; t < len; ++t)
      if (w == 0 || hi[b + t] != hi[b + w - 1]) hi[b + w++] = hi[b + t];
    bcnt[x] = w;
  }

  or_graph* g = (or_graph*)calloc(1, sizeof(or_graph));
  g->n = n;
  g->deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t m = 0;
  for (int64_t x = 0; x < n; ++x) {
    m += bcnt[x];
    for (int64_t t = 0; t < bcnt[x]; ++t) {
      g->deg[x]++;
      g->deg[hi[bptr[x] + t]]++;
    }
  }
  g->m = m;

  /* Degree order (Sec. 4.1): counting sort by degree, visiting ids in
     increasing order, so equal degrees keep id order. */
  int64_t maxd = 0;
  for (int64_t x = 0; x < n; ++x) if (g->deg[x] > maxd) maxd = g->deg[x];
  int64_t* start = (int64_t*)calloc((size_t)maxd + 2, sizeof(int64_t));
  for (int64_t x = 0; x < n; ++x) start[g->deg[x] + 1]++;
  for (int64_t d = 0; d <= maxd; ++d) start[d + 1] += start[d];
  g->rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  g->vert = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t x = 0; x < n; ++x) {
    int64_t r = start[g->deg[x]]++;
    g->rank[x] = (int32_t)r;
    g->vert[r] = (int32_t)x;
  }
  free(start);

  /* Oriented lists N(G,r) = ranks above r adjacent to r, sorted. */
  g->orow = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t x = 0; x < n; ++x)
    for (int64_t t = 0; t < bcnt[x]; ++t) {
      int32_t a = g->rank[x], b = g->rank[hi[bptr[x] + t]];
      g->orow[(a < b ? a : b) + 1]++;
    }
  for (int64_t r = 0; r < n; ++r) g->orow[r + 1] += g->orow[r];
  g->ocol = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  memcpy(cur, g->orow, sizeof(int64_t) * (size_t)n);
  for (int64_t x = 0; x < n; ++x)
    for (int64_t t = 0; t < bcnt[x]; ++t) {
      int32_t a = g->rank[x], b = g->rank[hi[bptr[x] + t]];
      if (a < b) g->ocol[cur[a]++] = b; else g->ocol[cur[b]++] = a;
    }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < n; ++r) {
    int64_t len = g->orow[r + 1] - g->orow[r];
    if (len > 1) qsort(g->ocol + g->orow[r], (size_t)len, sizeof(int32_t), cmp_i32);
  }
  free(cur); free(bptr); free(bcnt); free(hi);
  return g;
}

or_graph* or_build_edges(int64_t n, int64_t ne, const int32_t* src, const int32_t* dst) {
  if (n < 0 || ne < 0) return NULL;
  return build(n, ne, src, dst, NULL, NULL);
}
or_graph* or_build_csr(int64_t n, const int64_t* rowptr, const int32_t* colidx) {
  if (n < 0) return NULL;
  return build(n, 0, NULL, NULL, rowptr, colidx);
}

int64_t or_n(const or_graph* g) { return g->n; }
int64_t or_m(const or_graph* g) { return g->m; }
void or_rank(const or_graph* g, int32_t* out) { memcpy(out, g->rank, sizeof(int32_t) * (size_t)g->n); }
void or_degree(const or_graph* g, int64_t* out) { memcpy(out, g->deg, sizeof(int64_t) * (size_t)g->n); }
void or_oriented(const or_graph* g, int64_t* orow, int32_t* ocol) {
  memcpy(orow, g->orow, sizeof(int64_t) * ((size_t)g->n + 1));
  memcpy(ocol, g->ocol, sizeof(int32_t) * (size_t)g->m);
}

/* Alg. 1: |A cap B| for sorted A, B (with the first comparison read as A[a] = B[b]). */
static int64_t n_intersect(const int32_t* A, int64_t na, const int32_t* B, int64_t nb) {
  int64_t a = 0, b = 0, c = 0;
  while (a < na && b < nb) {
    if (A[a] == B[b]) { ++c; ++a; ++b; }
    else if (A[a] < B[b]) ++a;
    else ++b;
  }
  return c;
}

/* Alg. 2: tau = sum_u sum_{v in N(u)} |N(u) cap N(v)|. */
uint64_t or_total(const or_graph* g, int nthreads) {
  uint64_t tau = 0;
  const int64_t* R = g->orow;
  const int32_t* C = g->ocol;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : tau) num_threads(nthreads)
  for (int64_t u = 0; u < g->n; ++u)
    for (int64_t e = R[u]; e < R[u + 1]; ++e) {
      int32_t v = C[e];
      tau += (uint64_t)n_intersect(C + R[u], R[u + 1] - R[u], C + R[v], R[v + 1] - R[v]);
    }
  return tau;
}

/* Alg. 2 restricted to the listed rows (ranks) rows[0..nrows): the
   triangles whose lowest-ranked vertex is listed.  Summed over lists that
   partition [0, n) it gives the total; used to time the count on a bounded
   sample of rows.  Returns (uint64_t)-1 if a row is out of range. */
uint64_t or_total_rows(const or_graph* g, const int64_t* rows, int64_t nrows, int nthreads) {
  uint64_t tau = 0;
  const int64_t* R = g->orow;
  const int32_t* C = g->ocol;
  for (int64_t q = 0; q < nrows; ++q)
    if (rows[q] < 0 || rows[q] >= g->n) return (uint64_t)-1;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : tau) num_threads(nthreads)
  for (int64_t q = 0; q < nrows; ++q) {
    const int64_t u = rows[q];
    for (int64_t e = R[u]; e < R[u + 1]; ++e) {
      int32_t v = C[e];
      tau += (uint64_t)n_intersect(C + R[u], R[u + 1] - R[u], C + R[v], R[v + 1] - R[v]);
    }
  }
  return tau;
}

/* Alg. 3: stamp H[v] <- u for v in N(u), then count H[w] = u over w in N(v). */
uint64_t or_total_hmap(const or_graph* g, int nthreads) {
  uint64_t tau = 0;
  const int64_t* R = g->orow;
  const int32_t* C = g->ocol;
#pragma omp parallel num_threads(nthreads) reduction(+ : tau)
  {
    int64_t* H = (int64_t*)malloc(sizeof(int64_t) * (size_t)(g->n > 0 ? g->n : 1));
    for (int64_t x = 0; x < g->n; ++x) H[x] = -1;
#pragma omp for schedule(dynamic, 256)
    for (int64_t u = 0; u < g->n; ++u) {
      for (int64_t e = R[u]; e < R[u + 1]; ++e) H[C[e]] = u;
      for (int64_t e = R[u]; e < R[u + 1]; ++e) {
        int32_t v = C[e];
        for (int64_t f = R[v]; f < R[v + 1]; ++f)
          if (H[C[f]] == u) ++tau;
      }
    }
    free(H);
  }
  return tau;
}

/* Cut rule described in the header.  mode 0 = nnz-balanced, 1 = uniform. */
int or_cuts(const or_graph* g, int32_t p, int mode, int32_t* cuts) {
  const int64_t n = g->n, m = g->m;
  if (p < 1 || p > n) return -1;
  cuts[0] = 0;
  for (int32_t i = 1; i < p; ++i) {
    int64_t c;
    if (mode == 1) {
      c = (int64_t)i * n / p;
    } else {
      int64_t target = ((int64_t)i * m + p - 1) / p; /* ceil(i*m/p) */
      c = cuts[i - 1] + 1;
      while (c < n && g->orow[c] < target) ++c;
    }
    if (c < cuts[i - 1] + 1) c = cuts[i - 1] + 1;
    if (c > n - (p - i)) c = n - (p - i);
    cuts[i] = (int32_t)c;
  }
  cuts[p] = (int32_t)n;
  return 0;
}

/* Alg. 4: tasks (i,j,k), i<=j<=k, in loop order; out holds 3*|T| ints. */
int64_t or_task_list(int32_t p, int32_t* out) {
  int64_t t = 0;
  for (int32_t i = 0; i < p; ++i)
    for (int32_t j = i; j < p; ++j)
      for (int32_t k = j; k < p; ++k) {
        if (out) { out[3 * t] = i; out[3 * t + 1] = j; out[3 * t + 2] = k; }
        ++t;
      }
  return t;
}

/*
 * Per-task counts for the given cuts (checked to be strictly increasing from
 * 0 to n).  per_task has |T| entries in Alg. 4 order; block_nnz (optional)
 * has p(p+1)/2 entries, block (a,b), a<=b, in row-major order.
 * Returns the total, or (uint64_t)-1 on bad cuts.
 */
uint64_t or_tasks(const or_graph* g, int32_t p, const int32_t* cuts, uint64_t* per_task,
                  uint64_t* block_nnz, int nthreads) {
  const int64_t n = g->n;
  if (p < 1 || cuts[0] != 0 || cuts[p] != n) return (uint64_t)-1;
  for (int32_t i = 0; i < p; ++i) if (cuts[i + 1] <= cuts[i]) return (uint64_t)-1;
  int32_t* part = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int32_t i = 0; i < p; ++i)
    for (int64_t r = cuts[i]; r < cuts[i + 1]; ++r) part[r] = i;
  /* task index of (i,j,j), enumerated exactly as Alg. 4 visits them */
  int64_t* base = (int64_t*)malloc(sizeof(int64_t) * (size_t)p * (size_t)p);
  int64_t ntask = 0;
  for (int32_t i = 0; i < p; ++i)
    for (int32_t j = i; j < p; ++j) {
      base[(int64_t)i * p + j] = ntask;
      ntask += p - j;
    }
  memset(per_task, 0, sizeof(uint64_t) * (size_t)ntask);
  if (block_nnz) {
    int64_t nb = (int64_t)p * (p + 1) / 2;
    memset(block_nnz, 0, sizeof(uint64_t) * (size_t)nb);
    int64_t* bb = (int64_t*)malloc(sizeof(int64_t) * (size_t)p * (size_t)p);
    int64_t t = 0;
    for (int32_t a = 0; a < p; ++a) for (int32_t b = a; b < p; ++b) bb[(int64_t)a * p + b] = t++;
    for (int64_t u = 0; u < n; ++u)
      for (int64_t e = g->orow[u]; e < g->orow[u + 1]; ++e)
        block_nnz[bb[(int64_t)part[u] * p + part[g->ocol[e]]]]++;
    free(bb);
  }
  const int64_t* R = g->orow;
  const int32_t* C = g->ocol;
  uint64_t tau = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : tau)
  {
    uint64_t* mine = (uint64_t*)calloc((size_t)ntask, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 256)
    for (int64_t u = 0; u < n; ++u)
      for (int64_t e = R[u]; e < R[u + 1]; ++e) {
        int32_t v = C[e];
        /* walk N(u) and N(v) together (Alg. 1) and classify each common w */
        int64_t a = R[u], ae = R[u + 1], b = R[v], be = R[v + 1];
        while (a < ae && b < be) {
          if (C[a] == C[b]) {
            int32_t w = C[a];
            mine[base[(int64_t)part[u] * p + part[v]] + (part[w] - part[v])]++;
            ++tau; ++a; ++b;
          } else if (C[a] < C[b]) ++a;
          else ++b;
        }
      }
#pragma omp critical
    for (int64_t t = 0; t < ntask; ++t) per_task[t] += mine[t];
    free(mine);
  }
  free(base); free(part);
  return tau;
}

int or_max_threads(void) { return omp_get_max_threads(); }
