// Per-task count on host threads (the CPU side of the hybrid execution of
// arXiv 2009.12457, Sec. 5: CPU threads take light tasks from the tail of the
// estimate-ordered task list while the GPU takes the heavy ones).  A task
// {i,j,k} sums |N(G_ik,u) cap N(G_jk,v)| over the edges (u,v) of G_ij
// (Sec. 4.3), here by the merge intersection of Alg. 1, over the plan's own
// block layout read from host memory: the active columns v of block (i,j)
// with their in-slices, and the out-row slices of the two blocks of part k.
#include "cpu_count.h"

#include <algorithm>

namespace bbtc {

namespace {

// N(G_ak,u) = ocol[lo, hi) for u in part a: stored boundaries above rT,
// binary search below.
inline void out_slice(const HostTables& t, int32_t u, int32_t a, int32_t k, uint32_t& lo, uint32_t& hi) {
  const int64_t sa = std::max<int64_t>(t.cuts[a], t.rT);
  if (u >= sa) {  // column-major per part: column b - a, row u - sa
    const uint64_t ns = (uint64_t)(t.cuts[a + 1] - sa);
    const uint32_t* col = t.bot + t.botp[a] + (uint64_t)(u - sa);
    lo = col[(uint64_t)(k - a) * ns];
    hi = col[(uint64_t)(k - a + 1) * ns];
    return;
  }
  const int32_t* b = t.ocol + t.orow[u];
  const int32_t* e = t.ocol + t.orow[u + 1];
  const int32_t* l = std::lower_bound(b, e, t.cuts[k]);
  const int32_t* h = std::lower_bound(l, e, t.cuts[k + 1]);
  lo = (uint32_t)(l - t.ocol);
  hi = (uint32_t)(h - t.ocol);
}

// |A cap B| for sorted A, B (Alg. 1).
inline uint64_t merge_count(const int32_t* A, uint32_t na, const int32_t* B, uint32_t nb) {
  uint32_t a = 0, b = 0;
  uint64_t c = 0;
  while (a < na && b < nb) {
    if (A[a] == B[b]) {
      ++c;
      ++a;
      ++b;
    } else if (A[a] < B[b]) {
      ++a;
    } else {
      ++b;
    }
  }
  return c;
}

}  // namespace

uint64_t cpu_count_task(const HostTables& t, int32_t i, int32_t j, int32_t k) {
  const int64_t cid = (int64_t)j * (j + 1) / 2 + i;
  uint64_t c = 0;
  for (uint64_t x = t.acp[cid]; x < t.acp[cid + 1]; ++x) {
    uint32_t v0, v1;
    out_slice(t, t.acol[x], j, k, v0, v1);
    if (v1 == v0) continue;
    for (uint32_t e = t.aoff[x]; e < t.aoff[x + 1]; ++e) {
      uint32_t u0, u1;
      out_slice(t, t.icolb[e], i, k, u0, u1);
      if (u1 > u0) c += merge_count(t.ocol + u0, u1 - u0, t.ocol + v0, v1 - v0);
    }
  }
  return c;
}

}  // namespace bbtc
