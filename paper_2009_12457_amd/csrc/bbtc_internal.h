// Internal declarations shared by the host runtime and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bbtc.h"

namespace bbtc {

constexpr int kMaxP = 2048;         // largest supported blocks-per-side
constexpr int kPrepRows = 256;      // rows per workgroup in the block-index kernels
constexpr int kThreads = 256;       // workgroup size of every kernel
constexpr int kRadixItems = 16;     // keys per thread per radix tile
constexpr int kRadixTile = kThreads * kRadixItems;
constexpr int kScanItems = 8;
constexpr int kScanTile = kThreads * kScanItems;

// One task {i,j,k} as the counting kernels see it; `out` is its slot in the
// per-task output array.
struct DevTask {
  int32_t i, j, k, out;
};

// One unit of persistent work: rows [lo, hi) of the active-row list of block
// (i,j) of task `task` of plan `plan` (plan is 0 for single-plan launches).
struct DevItem {
  int32_t plan;
  int32_t task;
  uint32_t lo, hi;
};

// Device view of the blocked graph (stripe layout plus block row index).
//   ocol  : oriented CSR columns in rank space, every row ascending.
//   bot   : for a row u in part a, (p-a+1) absolute positions in ocol; entry
//           b-a is the first position of N(G,u) whose column is >= cuts[b],
//           so N(G_ab,u) = ocol[bot[b-a] .. bot[b-a+1]).  Rows of part a start
//           at element botp[a] and are (p-a+1) entries apart.
//   arow  : per block (a,b), the rows u of V_a with N(G_ab,u) non-empty, in
//           increasing order, starting at arp[bid(a,b)].
struct GraphView {
  int32_t p;
  uint32_t m;  // entries of ocol
  const int32_t* cuts;
  const uint64_t* botp;
  const uint32_t* bot;
  const int32_t* ocol;
  const uint64_t* arp;
  const int32_t* arow;
};

// Everything a counting kernel needs about one plan.
struct PlanCtx {
  GraphView g;
  const DevTask* tasks;
  uint64_t* per_task;
  uint64_t* total;
  int32_t wave_min;
  int32_t hash_min;  // < 0: never
};

struct CountParams {
  PlanCtx one;            // the plan of a single-plan launch
  const PlanCtx* many;    // device array, indexed by DevItem::plan (multi-plan launch)
  const DevItem* items;
  uint32_t nitems;
  uint32_t* cursor;
};

__host__ __device__ inline int64_t block_id(int64_t p, int64_t a, int64_t b) {
  return a * p - a * (a - 1) / 2 + (b - a);
}

// ---- launchers (kernels_prep.hip) ----
hipError_t launch_validate(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, int64_t nnz,
                           int symmetric, uint32_t* err, hipStream_t s);
hipError_t launch_degkey(const void* rowptr, int rp64, int64_t n, int idbits, uint64_t* keys, hipStream_t s);
// Sorts keys[0..count) by their low `bits` bits; the result ends in *result
// (one of a or b).  hist/partial are scratch sized by radix_scratch_*().
size_t radix_hist_entries(uint64_t count);
size_t scan_partial_entries(uint64_t count);
hipError_t radix_sort_u64(uint64_t* a, uint64_t* b, uint64_t count, int bits, uint32_t* hist,
                          uint32_t* partial, uint64_t** result, hipStream_t s);
// out[0..count] = exclusive scan of in[0..count), out[count] = total.
hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint64_t count, uint32_t* partial, hipStream_t s);
hipError_t launch_perm(const uint64_t* keys, int64_t n, int idbits, int32_t* order, int32_t* perm, hipStream_t s);
hipError_t launch_outdeg(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, const int32_t* perm,
                         uint32_t* od, hipStream_t s);
hipError_t launch_fill(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, const int32_t* perm,
                       const uint32_t* orow, int idbits, uint64_t* keys, uint64_t cap, hipStream_t s);
hipError_t launch_unpack(const uint64_t* keys, uint64_t m, int idbits, int32_t* ocol, hipStream_t s);
hipError_t launch_cuts(const uint32_t* orow, int64_t n, int32_t p, int mode, int32_t* cuts, hipStream_t s);

struct BlockBuild {
  int32_t p;
  int32_t nchunks;           // total row chunks (kPrepRows rows each, within one part)
  const int32_t* cuts;       // p+1
  const int32_t* chunk0;     // p+1: first chunk of each part
  const uint64_t* ccbase;    // p: start of part a's chunk counters
  const uint32_t* orow;
  const int32_t* ocol;
  const uint64_t* botp;
  uint32_t* bot;
  unsigned long long* bnnz;  // nb
  unsigned long long* bnzr;  // nb
  uint32_t* ccnt;            // per (part a, block b, chunk) active-row counts
  uint32_t* dmax_block;
  const uint32_t* ccoff;     // exclusive scan of ccnt (for the fill)
  int32_t* arow;
};
hipError_t launch_bot(const BlockBuild& bb, hipStream_t s);
hipError_t launch_arow(const BlockBuild& bb, hipStream_t s);

// ---- launchers (kernels_count.hip) ----
hipError_t launch_reset(uint64_t* per_task, int64_t ntasks, uint64_t* total, uint32_t* cursor, hipStream_t s);
hipError_t launch_count_task(const CountParams& cp, int32_t task, uint32_t nrows, hipStream_t s);
hipError_t launch_count_persistent(const CountParams& cp, int grid, bool multi, hipStream_t s);
int count_persistent_blocks_per_cu();

}  // namespace bbtc
