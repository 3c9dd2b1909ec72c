// Drives the library's pure host code -- the block-table checker
// (csrc/plan_check.h) and the host-thread per-task count of the hybrid
// execution (csrc/cpu_count.cpp) -- over tables read from a file;
// tests/test_sanitize_cpu.py builds it with AddressSanitizer and
// UndefinedBehaviorSanitizer and compares the counts with the oracle's.
//
// Input file: int64 n, m, p, rT, then for each of cuts, orow, ocol, botp,
// bot, acp, acol, aoff, icolb an int64 element count followed by the elements
// (int32, uint32, int32, uint64, uint32, uint64, int32, uint32, int32).
// Output (stdout): the checker's verdict on the tables ("ok" or its message),
// then one line per task (i, j, k), i <= j <= k in loop order (Alg. 4):
// "i j k count"; then the verdicts on tables with one entry changed, each of
// which must be rejected.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "cpu_count.h"
#include "plan_check.h"

namespace {

template <typename T>
std::vector<T> read_array(FILE* f) {
  int64_t len = -1;
  if (std::fread(&len, sizeof len, 1, f) != 1 || len < 0) {
    std::fprintf(stderr, "bad array length\n");
    std::exit(2);
  }
  std::vector<T> v((size_t)len);
  if (len && std::fread(v.data(), sizeof(T), (size_t)len, f) != (size_t)len) {
    std::fprintf(stderr, "short array\n");
    std::exit(2);
  }
  return v;
}

struct Tables {
  int64_t n = 0, m = 0, p = 0, rT = 0;
  std::vector<int32_t> cuts, ocol, acol, icolb;
  std::vector<uint32_t> orow, bot, aoff;
  std::vector<uint64_t> botp, acp;
  bbtc::TableView view() const {
    return bbtc::TableView{n, m, (int32_t)p, (int32_t)rT, cuts.data(), orow.data(), ocol.data(), botp.data(),
                           bot.data(), acp.data(), acol.data(), aoff.data(), icolb.data()};
  }
};

void verdict(const char* what, const Tables& t) {
  const std::string msg = bbtc::check_tables(t.view());
  std::printf("%s: %s\n", what, msg.empty() ? "ok" : msg.c_str());
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: host_driver TABLES\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) {
    std::perror(argv[1]);
    return 2;
  }
  Tables t;
  int64_t head[4];
  if (std::fread(head, sizeof(int64_t), 4, f) != 4) return 2;
  t.n = head[0];
  t.m = head[1];
  t.p = head[2];
  t.rT = head[3];
  t.cuts = read_array<int32_t>(f);
  t.orow = read_array<uint32_t>(f);
  t.ocol = read_array<int32_t>(f);
  t.botp = read_array<uint64_t>(f);
  t.bot = read_array<uint32_t>(f);
  t.acp = read_array<uint64_t>(f);
  t.acol = read_array<int32_t>(f);
  t.aoff = read_array<uint32_t>(f);
  t.icolb = read_array<int32_t>(f);
  std::fclose(f);
  verdict("tables", t);
  const bbtc::HostTables h{(int32_t)t.p, (int32_t)t.rT, t.cuts.data(), t.orow.data(), t.ocol.data(),
                           t.botp.data(), t.bot.data(), t.acp.data(), t.acol.data(), t.aoff.data(),
                           t.icolb.data()};
  for (int32_t i = 0; i < t.p; ++i)
    for (int32_t j = i; j < t.p; ++j)
      for (int32_t k = j; k < t.p; ++k)
        std::printf("%d %d %d %llu\n", i, j, k, (unsigned long long)bbtc::cpu_count_task(h, i, j, k));
  // one changed entry per table: the checker must name a violation
  if (!t.bot.empty()) {
    Tables b = t;
    b.bot.back() += 100;
    verdict("bot changed", b);
  }
  if (t.acol.size() > 1) {
    Tables b = t;
    b.acol[1] += 1;
    verdict("acol changed", b);
  }
  if (t.m > 1) {
    Tables b = t;
    b.orow[t.n] -= 1;
    verdict("orow changed", b);
  }
  if (t.p > 1) {
    Tables b = t;
    b.cuts[1] = b.cuts[0];
    verdict("cuts changed", b);
  }
  return 0;
}
