/*
 * Drives the oracle (oracle/oracle.c) and the graph generators
 * (graphgen/graphgen.c) over small graphs; tests/test_sanitize_cpu.py builds
 * it with AddressSanitizer and UndefinedBehaviorSanitizer, so every buffer
 * those files allocate, index and free is checked.  Besides running clean it
 * checks what the two files promise one another: the list and hash totals
 * agree (Alg. 2 and Alg. 3), the per-task counts of every cut vector sum to
 * the total and the block nnz to m (Sec. 4.2), the CSR generator's output is
 * symmetric with sorted rows.  Prints one line per graph; exits nonzero on
 * the first disagreement.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct oracle_graph or_graph;  /* opaque here */
or_graph* or_build_edges(int64_t n, int64_t ne, const int32_t* src, const int32_t* dst);
or_graph* or_build_csr(int64_t n, const int64_t* rowptr, const int32_t* colidx);
void or_free(or_graph* g);
int64_t or_n(const or_graph* g);
int64_t or_m(const or_graph* g);
void or_rank(const or_graph* g, int32_t* out);
void or_degree(const or_graph* g, int64_t* out);
void or_oriented(const or_graph* g, int64_t* orow, int32_t* ocol);
uint64_t or_total(const or_graph* g, int nthreads);
uint64_t or_total_rows(const or_graph* g, const int64_t* rows, int64_t nrows, int nthreads);
uint64_t or_total_hmap(const or_graph* g, int nthreads);
int or_cuts(const or_graph* g, int32_t p, int mode, int32_t* cuts);
int64_t or_task_list(int32_t p, int32_t* out);
uint64_t or_tasks(const or_graph* g, int32_t p, const int32_t* cuts, uint64_t* per_task, uint64_t* block_nnz,
                  int nthreads);
int gg_rmat_edges(int scale, int64_t ne, double a, double b, double c, uint64_t seed, int32_t* src, int32_t* dst);
int64_t gg_er_count(int64_t n, double p, uint64_t seed);
int gg_er_edges(int64_t n, double p, uint64_t seed, int64_t ne, int32_t* src, int32_t* dst);
int64_t gg_csr_from_edges(int64_t n, int64_t ne, const int32_t* src, const int32_t* dst, int64_t* rowptr,
                          int32_t* col, int64_t cap);
int64_t gg_rmat_csr(int scale, int64_t ne, double a, double b, double c, uint64_t seed, int64_t* rowptr,
                    int32_t* col, int64_t cap);
int64_t gg_er_csr(int64_t n, double p, uint64_t seed, int64_t* rowptr, int32_t* col, int64_t cap);

#define FAIL(...)                       \
  do {                                  \
    fprintf(stderr, __VA_ARGS__);       \
    fputc('\n', stderr);                \
    exit(1);                            \
  } while (0)

/* sorted, duplicate-free, loop-free and symmetric rows */
static void check_csr(const char* name, int64_t n, const int64_t* rp, const int32_t* col) {
  for (int64_t x = 0; x < n; ++x)
    for (int64_t e = rp[x]; e < rp[x + 1]; ++e) {
      const int32_t y = col[e];
      if (y < 0 || y >= n || y == x) FAIL("%s: entry %lld of row %lld out of range", name, (long long)e, (long long)x);
      if (e > rp[x] && col[e - 1] >= y) FAIL("%s: row %lld not increasing", name, (long long)x);
      int64_t lo = rp[y], hi = rp[y + 1];
      while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (col[mid] < x) lo = mid + 1; else hi = mid;
      }
      if (lo == rp[y + 1] || col[lo] != x) FAIL("%s: (%lld,%d) has no reverse", name, (long long)x, y);
    }
}

static void check_graph(const char* name, or_graph* g) {
  const int64_t n = or_n(g), m = or_m(g);
  int32_t* rank = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int64_t* deg = malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* orow = malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t* ocol = malloc(sizeof(int32_t) * (size_t)(m + 1));
  int64_t* rows = malloc(sizeof(int64_t) * (size_t)(n + 1));
  or_rank(g, rank);
  or_degree(g, deg);
  or_oriented(g, orow, ocol);
  int64_t dsum = 0;
  for (int64_t v = 0; v < n; ++v) dsum += deg[v];
  if (dsum != 2 * m || orow[n] != m) FAIL("%s: degree sum %lld, m %lld", name, (long long)dsum, (long long)m);
  for (int64_t v = 0; v < n; ++v) rows[v] = n - 1 - v;
  const uint64_t t_list = or_total(g, 3), t_hmap = or_total_hmap(g, 2), t_rows = or_total_rows(g, rows, n, 1);
  if (t_list != t_hmap || t_list != t_rows)
    FAIL("%s: totals %llu %llu %llu", name, (unsigned long long)t_list, (unsigned long long)t_hmap,
         (unsigned long long)t_rows);
  const int32_t ps[4] = {1, 2, 5, (int32_t)n};
  for (int q = 0; q < 4; ++q) {
    const int32_t p = ps[q];
    if (p < 1 || p > n || p > 80) continue;
    for (int mode = 0; mode < 2; ++mode) {
      int32_t* cuts = malloc(sizeof(int32_t) * (size_t)(p + 1));
      if (or_cuts(g, p, mode, cuts) != 0) FAIL("%s: or_cuts(p=%d) refused", name, p);
      const int64_t nt = or_task_list(p, NULL);
      int32_t* list = malloc(sizeof(int32_t) * 3 * (size_t)nt);
      if (or_task_list(p, list) != nt || nt != (int64_t)p * (p + 1) * (p + 2) / 6) FAIL("%s: task list", name);
      uint64_t* per = malloc(sizeof(uint64_t) * (size_t)nt);
      const int64_t nb = (int64_t)p * (p + 1) / 2;
      uint64_t* bn = malloc(sizeof(uint64_t) * (size_t)nb);
      const uint64_t tot = or_tasks(g, p, cuts, per, bn, 2);
      uint64_t s = 0, sb = 0;
      for (int64_t t = 0; t < nt; ++t) s += per[t];
      for (int64_t b = 0; b < nb; ++b) sb += bn[b];
      if (tot != t_list || s != t_list || sb != (uint64_t)m) FAIL("%s: p=%d mode %d per-task sum", name, p, mode);
      free(cuts); free(list); free(per); free(bn);
    }
  }
  /* cut vectors the oracle must refuse */
  int32_t bad[3] = {0, 0, (int32_t)n};
  uint64_t per_bad[4];
  if (n > 0 && or_tasks(g, 2, bad, per_bad, NULL, 1) != (uint64_t)-1) FAIL("%s: repeated cut accepted", name);
  if (or_cuts(g, 0, 0, bad) != -1) FAIL("%s: p = 0 accepted", name);
  printf("%s n=%lld m=%lld triangles=%llu\n", name, (long long)n, (long long)m, (unsigned long long)t_list);
  free(rank); free(deg); free(orow); free(ocol); free(rows);
}

static void from_edges(const char* name, int64_t n, int64_t ne, const int32_t* src, const int32_t* dst) {
  or_graph* g = or_build_edges(n, ne, src, dst);
  if (!g) FAIL("%s: or_build_edges failed", name);
  check_graph(name, g);
  /* the same graph through the CSR generator and the oracle's CSR input */
  const int64_t cap = 2 * ne + 1;
  int64_t* rp = malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t* col = malloc(sizeof(int32_t) * (size_t)cap);
  const int64_t nnz = gg_csr_from_edges(n, ne, src, dst, rp, col, cap);
  if (nnz < 0 || nnz != 2 * or_m(g)) FAIL("%s: gg_csr_from_edges gave %lld", name, (long long)nnz);
  check_csr(name, n, rp, col);
  or_graph* h = or_build_csr(n, rp, col);
  if (!h || or_m(h) != or_m(g) || or_total(h, 2) != or_total(g, 2)) FAIL("%s: CSR and edge builds differ", name);
  or_free(h);
  or_free(g);
  free(rp); free(col);
}

int main(void) {
  /* tiny and degenerate graphs: one vertex, no edges, a triangle given with a
     repeated edge, a reversed copy and a self-loop */
  from_edges("single", 1, 0, NULL, NULL);
  from_edges("empty7", 7, 0, NULL, NULL);
  const int32_t ts[6] = {0, 1, 2, 1, 2, 2}, td[6] = {1, 2, 0, 0, 1, 2};
  from_edges("triangle", 3, 6, ts, td);
  /* R-MAT samples (with duplicates and self-loops) at two scales */
  const int scales[2] = {8, 11};
  for (int q = 0; q < 2; ++q) {
    const int64_t ne = (int64_t)8 << scales[q];
    int32_t* s = malloc(sizeof(int32_t) * (size_t)ne);
    int32_t* d = malloc(sizeof(int32_t) * (size_t)ne);
    if (gg_rmat_edges(scales[q], ne, 0.57, 0.19, 0.19, 7 + q, s, d) != 0) FAIL("gg_rmat_edges");
    char name[32];
    snprintf(name, sizeof name, "rmat%d", scales[q]);
    from_edges(name, (int64_t)1 << scales[q], ne, s, d);
    free(s); free(d);
  }
  /* Erdos-Renyi pairs */
  const int64_t n = 300, ne = gg_er_count(n, 0.05, 3);
  int32_t* s = malloc(sizeof(int32_t) * (size_t)(ne + 1));
  int32_t* d = malloc(sizeof(int32_t) * (size_t)(ne + 1));
  if (gg_er_edges(n, 0.05, 3, ne, s, d) != 0) FAIL("gg_er_edges");
  from_edges("er300", n, ne, s, d);
  free(s); free(d);
  /* the direct CSR generators, with a too-small buffer refused first */
  int64_t* rp = malloc(sizeof(int64_t) * ((1 << 10) + 1));
  int32_t* col = malloc(sizeof(int32_t) * (1 << 15));
  if (gg_rmat_csr(10, 1 << 13, 0.57, 0.19, 0.19, 5, rp, col, 16) >= 0) FAIL("gg_rmat_csr: small buffer accepted");
  const int64_t nnz = gg_rmat_csr(10, 1 << 13, 0.57, 0.19, 0.19, 5, rp, col, 1 << 15);
  if (nnz <= 0) FAIL("gg_rmat_csr failed");
  check_csr("rmat_csr10", 1 << 10, rp, col);
  const int64_t nnz2 = gg_er_csr(500, 0.02, 9, rp, col, 1 << 15);
  if (nnz2 <= 0) FAIL("gg_er_csr failed");
  check_csr("er_csr500", 500, rp, col);
  if (gg_er_csr(10, 1.5, 1, rp, col, 1 << 15) != -1) FAIL("gg_er_csr: p > 1 accepted");
  free(rp); free(col);
  printf("oracle driver: all checks passed\n");
  return 0;
}
