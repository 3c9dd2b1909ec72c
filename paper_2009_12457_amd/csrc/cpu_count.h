// Host-thread per-task count over a plan's block layout in host memory.
#pragma once
#include <stdint.h>

namespace bbtc {

// The count-phase arrays of a plan in host memory (layout as GraphView in
// bbtc_internal.h, resident form: absolute positions and indices).
struct HostTables {
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

// The triangles of task {i,j,k} (i <= j <= k).
uint64_t cpu_count_task(const HostTables& t, int32_t i, int32_t j, int32_t k);

}  // namespace bbtc
