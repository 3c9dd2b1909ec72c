// Host-side consistency check of a plan's block tables: everything the
// counting kernels index into, checked against the definitions of the
// layout (see GraphView in bbtc_internal.h) from the oriented CSR itself.
// Pure host code, O(m + p^2 + stored boundary words); no device calls.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "bbtc.h"

namespace bbtc {

struct TableView {
  int64_t n, m;
  int32_t p, rT;
  const int32_t* cuts;
  const uint32_t* orow;
  const int32_t* ocol;
  const uint64_t* botp;
  const uint32_t* bot;
  const uint64_t* acp;
  const int32_t* acol;
  const uint32_t* aoff;
  const int32_t* icolb;
};

// Returns "" if every table is consistent, else a description of the first
// violation found.
inline std::string check_tables(const TableView& t) {
  const int64_t n = t.n, m = t.m;
  const int32_t p = t.p;
  auto fmt = [](const char* what, int64_t a, int64_t b) {
    return std::string(what) + " (" + std::to_string(a) + ", " + std::to_string(b) + ")";
  };
  if (p < 1 || p > n) return fmt("p out of range", p, n);
  if (t.cuts[0] != 0 || t.cuts[p] != n) return fmt("cut vector must run from 0 to n", t.cuts[0], t.cuts[p]);
  for (int32_t a = 0; a < p; ++a)
    if (t.cuts[a + 1] <= t.cuts[a]) return fmt("cut vector not strictly increasing at part", a, t.cuts[a + 1]);
  if (t.rT < 0 || t.rT > n) return fmt("rT out of range", t.rT, n);
  std::vector<int32_t> part((size_t)n);
  for (int32_t a = 0; a < p; ++a)
    for (int64_t r = t.cuts[a]; r < t.cuts[a + 1]; ++r) part[(size_t)r] = a;
  // oriented rows: ascending, above their own rank
  if (t.orow[0] != 0 || (int64_t)t.orow[n] != m) return fmt("orow ends", t.orow[0], t.orow[n]);
  std::vector<uint32_t> indeg((size_t)n + 1, 0);
  for (int64_t r = 0; r < n; ++r) {
    if (t.orow[r + 1] < t.orow[r]) return fmt("orow decreases at", r, t.orow[r]);
    for (uint32_t e = t.orow[r]; e < t.orow[r + 1]; ++e) {
      const int32_t w = t.ocol[e];
      if (w <= r || w >= n) return fmt("ocol entry out of range", r, w);
      if (e > t.orow[r] && t.ocol[e - 1] >= w) return fmt("out-row not strictly increasing", r, e);
      indeg[(size_t)w + 1]++;
    }
  }
  // in-rows (the transpose), sorted; degrees non-decreasing with rank
  for (int64_t r = 0; r < n; ++r) indeg[(size_t)r + 1] += indeg[(size_t)r];
  std::vector<int32_t> inn((size_t)m);
  {
    std::vector<uint32_t> at(indeg.begin(), indeg.end() - 1);
    for (int64_t r = 0; r < n; ++r)
      for (uint32_t e = t.orow[r]; e < t.orow[r + 1]; ++e) inn[at[(size_t)t.ocol[e]]++] = (int32_t)r;
  }
  for (int64_t r = 1; r < n; ++r) {
    const uint64_t d0 = (uint64_t)(t.orow[r] - t.orow[r - 1]) + (indeg[(size_t)r] - indeg[(size_t)r - 1]);
    const uint64_t d1 = (uint64_t)(t.orow[r + 1] - t.orow[r]) + (indeg[(size_t)r + 1] - indeg[(size_t)r]);
    if (d1 < d0) return fmt("degree decreases with rank at", r, (int64_t)d1);
  }
  // stored block boundaries: rows max(c_a, rT) .. c_{a+1}-1 of each part,
  // column-major (column b-a holds entry b-a of every stored row)
  if (t.botp[0] != 0) return fmt("boundary table must start at 0", (int64_t)t.botp[0], 0);
  for (int32_t a = 0; a < p; ++a) {
    const int64_t sa = t.cuts[a] > t.rT ? t.cuts[a] : t.rT;
    const int64_t stored = t.cuts[a + 1] > sa ? t.cuts[a + 1] - sa : 0;
    if (t.botp[a + 1] - t.botp[a] != (uint64_t)(stored * (p - a + 1))) return fmt("botp step wrong at part", a, stored);
    for (int64_t u = sa; u < t.cuts[a + 1]; ++u) {  // column-major: column b-a, row u-sa
      const uint32_t* br = t.bot + t.botp[a] + (uint64_t)(u - sa);
      uint32_t e = t.orow[u];
      for (int32_t b = a; b <= p; ++b) {  // entry b-a: first position with a column >= cuts[b]
        while (b < p && e < t.orow[u + 1] && t.ocol[e] < t.cuts[b]) ++e;
        const uint32_t want = b == p ? t.orow[u + 1] : e;
        if (br[(uint64_t)(b - a) * (uint64_t)stored] != want) return fmt("out-side boundary wrong for row", u, b);
      }
    }
  }
  // block-major in side: per block (a,b), column-major, the v in V_b with an
  // in-neighbour in V_a, ascending, each with exactly those in-neighbours as
  // its slice (in any order), slices laid out back to back from 0 to m
  const int64_t nb = (int64_t)p * (p + 1) / 2;
  if (t.acp[0] != 0) return fmt("acp must start at 0", (int64_t)t.acp[0], 0);
  std::vector<std::vector<int32_t>> want((size_t)nb);
  for (int64_t v = 0; v < n; ++v) {
    const int32_t b = part[(size_t)v];
    int32_t last = -1;
    for (uint32_t f = indeg[(size_t)v]; f < indeg[(size_t)v + 1]; ++f) {
      const int32_t a = part[(size_t)inn[f]];
      if (a != last) want[(size_t)b * (b + 1) / 2 + a].push_back((int32_t)v);
      last = a;
    }
  }
  uint64_t ent = 0;
  std::vector<int32_t> got;
  for (int64_t c = 0; c < nb; ++c) {
    if (t.acp[c + 1] < t.acp[c]) return fmt("acp decreases at block", c, (int64_t)t.acp[c]);
    const uint64_t len = t.acp[c + 1] - t.acp[c];
    if (len != want[(size_t)c].size()) return fmt("active-column count wrong for block", c, (int64_t)len);
    int32_t b = 0;
    while ((int64_t)(b + 1) * (b + 2) / 2 <= c) ++b;
    const int32_t a = (int32_t)(c - (int64_t)b * (b + 1) / 2);
    for (uint64_t q = 0; q < len; ++q) {
      const uint64_t x = t.acp[c] + q;
      const int32_t v = t.acol[x];
      if (v != want[(size_t)c][q]) return fmt("active column wrong in block", c, (int64_t)q);
      if (t.aoff[x] != ent) return fmt("in-slice offset wrong for active column", (int64_t)x, t.aoff[x]);
      // in-neighbours of v in V_a: a contiguous run of the sorted transpose
      uint32_t f = indeg[(size_t)v], g = indeg[(size_t)v + 1];
      while (f < g && inn[f] < t.cuts[a]) ++f;
      uint32_t h = f;
      while (h < g && inn[h] < t.cuts[a + 1]) ++h;
      if (t.aoff[x + 1] < t.aoff[x] || t.aoff[x + 1] - t.aoff[x] != h - f)
        return fmt("in-slice length wrong for active column", (int64_t)x, (int64_t)(h - f));
      got.assign(t.icolb + t.aoff[x], t.icolb + t.aoff[x + 1]);
      std::sort(got.begin(), got.end());
      for (uint32_t y = 0; y < h - f; ++y)
        if (got[y] != inn[f + y]) return fmt("in-slice entries wrong for active column", (int64_t)x, (int64_t)y);
      ent += h - f;
    }
  }
  if (ent != (uint64_t)m || t.aoff[t.acp[nb]] != (uint64_t)m) return fmt("in-slices do not end at m", (int64_t)ent, m);
  return "";
}

}  // namespace bbtc
