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

// One unit of persistent work of plan-order task `task` of its plan:
//   v < 0 : entries [lo, hi) of the active-column list of block (i,j);
//   v >= 0: in-neighbours [lo, hi) (relative to the start of the in-slice)
//           of one column v of G_ij whose in-slice is longer than the split
//           threshold; such columns are skipped by column-range items.
struct DevItem {
  int32_t task;
  uint32_t lo, hi;
  int32_t v;
};

// A column v of block (a,b) whose in-slice from V_a has more than `split`
// entries (collected while the active columns are written).
struct HeavyCol {
  uint32_t cid;  // column-major block id of (a,b)
  int32_t v;
  uint32_t cnt;  // in-slice length
};

// Device view of the blocked graph (stripe layout plus block row index).
//   ocol  : oriented CSR columns in rank space, every row ascending.
//   bot   : for a row u in part a, (p-a+1) absolute positions in ocol; entry
//           b-a is the first position of N(G,u) whose column is >= cuts[b],
//           so N(G_ab,u) = ocol[bot[b-a] .. bot[b-a+1]).  Rows of part a start
//           at element botp[a] and are (p-a+1) entries apart.
//   icol  : in-rows: for each rank v, the ranks u < v adjacent to v, ascending.
//   tbot  : for v in part b, (b+2) positions in icol; entry a is the first
//           in-neighbour of rank >= cuts[a], so the in-slice of v in block
//           (a,b) is icol[tbot[a] .. tbot[a+1]).  Part b starts at tbotp[b].
//   acol  : per block (a,b), the columns v of V_b with a non-empty in-slice
//           in increasing order, starting at acp[cid(a,b)], cid = b(b+1)/2+a.
struct GraphView {
  int32_t p;
  uint32_t m;  // entries of ocol (and of icol)
  // Streamed launches cover the tasks of one block pair (gi, gj) and read the
  // rows of parts gi and gj from cached stripes: colI/colJ/icolJ are shifted
  // so that the absolute positions held in bot/tbot index them, botI/botJ and
  // tbotJ point at the first block-boundary row of the part.  gi < 0: the
  // whole graph is resident and the fields below are used instead.
  int32_t gi, gj;
  const int32_t* colI;
  const int32_t* colJ;
  const int32_t* icolJ;
  const uint32_t* botI;
  const uint32_t* botJ;
  const uint32_t* tbotJ;
  const int32_t* cuts;
  const uint64_t* botp;
  const uint32_t* bot;
  const int32_t* ocol;
  const uint64_t* tbotp;
  const uint32_t* tbot;
  const int32_t* icol;
  const uint64_t* acp;   // column-major block order
  const int32_t* acol;
};

// Everything a counting kernel needs about one plan.
struct PlanCtx {
  GraphView g;
  const DevTask* tasks;
  int64_t ntasks;
  uint64_t* per_task;
  uint64_t* total;
  int32_t wave_min;
  int32_t hash_min;  // < 0: never
  uint32_t split;    // columns with longer in-slices come as split items
  int32_t pad;
  const DevItem* items;  // the plan's work items on the device (multi-plan launches)
};

// Work queues of a persistent launch: one per XCD (8 on MI355X, each with its
// own L2); a workgroup drains the queue of its own XCD first, then the others.
constexpr int kMaxQueues = 8;

struct CountParams {
  PlanCtx one;            // the plan of a single-plan launch
  // multi-plan launch: many[q] holds the items [plan_off[q], plan_off[q+1])
  // of the combined index space (nplans entries, non-decreasing from 0)
  const PlanCtx* many;
  const uint32_t* plan_off;
  int32_t nplans;
  const DevItem* items;
  uint32_t nitems;
  uint32_t* cursor;       // kMaxQueues claim counters, zeroed by the reset kernels
  uint32_t nq;            // queues in use, 1..kMaxQueues
  uint32_t qbeg[kMaxQueues];  // queue x = items[qbeg[x], qbeg[x] + qlen[x])
  uint32_t qlen[kMaxQueues];
};

__host__ __device__ inline int64_t block_id(int64_t p, int64_t a, int64_t b) {
  return a * p - a * (a - 1) / 2 + (b - a);
}
__host__ __device__ inline int64_t col_block_id(int64_t a, int64_t b) { return b * (b + 1) / 2 + a; }

// ---- launchers (kernels_prep.hip) ----
// Row kernels take two scratch lists (n entries each) with zeroed counters:
// rows longer than a lane handles, and huge rows cut into chunks (hpref:
// n+1 scratch words for the chunk prefix); launch_fill reuses the lists and
// prefix of launch_degs.
hipError_t launch_validate(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, int64_t nnz,
                           int symmetric, uint32_t* err, uint32_t* list, uint32_t* nlist, uint32_t* hlist,
                           uint32_t* nhlist, uint32_t* hpref, hipStream_t s);
hipError_t launch_degkey(const void* rowptr, int rp64, int64_t n, int idbits, uint64_t* keys, hipStream_t s);
// Stable sort of keys[0..count) by their bits [lo, hi) (LSD, 8 bits a pass);
// the result ends in *result (one of a or b).  hist/partial are scratch
// sized by radix_hist_entries() and scan_partial_entries().
size_t radix_hist_entries(uint64_t count);
size_t scan_partial_entries(uint64_t count);
hipError_t radix_sort_u64(uint64_t* a, uint64_t* b, uint64_t count, int lo, int hi, uint32_t* hist,
                          uint32_t* partial, uint64_t** result, hipStream_t s);
// out[0..count] = exclusive scan of in[0..count), out[count] = total.
hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint64_t count, uint32_t* partial, hipStream_t s);
hipError_t launch_perm(const uint64_t* keys, int64_t n, int idbits, int32_t* order, int32_t* perm, hipStream_t s);
hipError_t launch_degs(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, int64_t nnz,
                       const int32_t* perm, uint32_t* od, uint32_t* idg, uint32_t* list, uint32_t* nlist,
                       uint32_t* hlist, uint32_t* nhlist, uint32_t* hpref, uint32_t* err, int check, hipStream_t s);
// cur_o/cur_i: zeroed fill cursors of the huge rows (indexed by position in hlist).
hipError_t launch_fill(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, const int32_t* perm,
                       const uint32_t* orow, const uint32_t* irow, int32_t* ocol, int32_t* icol, const uint32_t* list,
                       const uint32_t* nlist, const uint32_t* hlist, const uint32_t* nhlist, const uint32_t* hpref,
                       uint32_t* cur_o, uint32_t* cur_i, hipStream_t s);
// Sorts every row of a CSR in place; values have at most `bits` bits.
// longrows and hugerows need nrows entries each, q[0..1] must be zero, and
// scratch needs rp[nrows] entries.
hipError_t launch_segsort(const uint32_t* rp, int32_t* col, int64_t nrows, int bits, uint32_t* midrows,
                          uint32_t* longrows, uint32_t* hugerows, uint32_t* q, int32_t* scratch, hipStream_t s);
// In-rows grouped by part: short rows fully sorted (launch_inrows_sort, which
// lists the long and huge rows and counts them in q[0], q[1], q[2]), long
// and huge ones by a counting pass over the parts of cuts[0..p] with
// scratch[] (m words) (launch_inrows_group).
hipError_t launch_inrows_sort(const uint32_t* rp, int32_t* col, int64_t nrows, uint32_t* midrows, uint32_t* longrows,
                              uint32_t* hugerows, uint32_t* q, hipStream_t s);
hipError_t launch_inrows_group(const uint32_t* rp, int32_t* col, const uint32_t* longrows, const uint32_t* hugerows,
                               const uint32_t* q, int32_t* scratch, const int32_t* cuts, int32_t p, hipStream_t s);
hipError_t launch_cuts(const uint32_t* orow, int64_t n, int32_t p, int mode, int32_t* cuts, hipStream_t s);

struct BlockBuild {
  int32_t p;
  int32_t nchunks;           // total row chunks (kPrepRows rows each, within one part)
  const int32_t* cuts;       // p+1
  const int32_t* chunk0;     // p+1: first chunk of each part
  const uint64_t* ccbase;    // p+1: start of part b's chunk counters (in side)
  const uint32_t* orow;
  const int32_t* ocol;
  const uint64_t* botp;
  uint32_t* bot;
  const uint32_t* irow;
  const int32_t* icol;
  const uint64_t* tbotp;
  uint32_t* tbot;
  unsigned long long* bnnz;  // nb, row-major block order
  unsigned long long* bnzr;  // nb, row-major block order
  unsigned long long* bnzc;  // nb, column-major block order cid(a,b) = b(b+1)/2 + a
  uint32_t* ccnt;            // per (part b, block (a,b), chunk) active-column counts
  uint32_t* dmax_block;      // [0] longest block slice, [1] longest oriented row
  const uint32_t* ccoff;     // exclusive scan of ccnt
  int32_t* acol;             // active columns, column-major block order
  uint32_t split;            // in-slice length above which a column is recorded as heavy
  HeavyCol* heavy;           // room for m/split + 1 records
  uint32_t* nheavy;
  uint32_t heavy_cap;
};
hipError_t launch_bot(const BlockBuild& bb, hipStream_t s);
hipError_t launch_tbot(const BlockBuild& bb, hipStream_t s);
hipError_t launch_acol(const BlockBuild& bb, hipStream_t s);

// Work-item emission on the device.  A run sends items [r0, r0 + n) of
// plan-order task `task` to out[dst, dst + n); the runs are sorted by dst,
// non-empty, and tile [0, nitems).  Item r of a task is its r-th hub chunk
// while r < nhub (chunks of `chunk` in-neighbours, hub records of block cid
// in hrec[hstart[cid], hstart[cid+1]) with their first chunk numbers in
// hcum), else active columns [(r - nhub) * nper, +nper) clipped to cols.
struct ItemRun {
  int32_t task;
  uint32_t r0, n, dst;
};
struct TaskItems {
  uint32_t nhub, nper, cols, cid;
};
hipError_t launch_emit_items(const ItemRun* runs, int32_t nruns, const TaskItems* ti, const uint32_t* hstart,
                             const HeavyCol* hrec, const uint32_t* hcum, uint32_t chunk, DevItem* out,
                             uint32_t nitems, hipStream_t s);

// ---- launchers (kernels_count.hip) ----
hipError_t launch_reset(uint64_t* per_task, int64_t ntasks, uint64_t* total, uint32_t* cursor, hipStream_t s);
// Zeroes the outputs of every plan of a multi-plan launch and the cursor.
hipError_t launch_reset_multi(const PlanCtx* ctxs, int32_t nplans, uint32_t* cursor, hipStream_t s);
hipError_t launch_count_persistent(const CountParams& cp, int grid, bool multi, hipStream_t s);
// Items [first, first+count) of cp.items, one workgroup each.
hipError_t launch_count_items(const CountParams& cp, uint32_t first, uint32_t count, hipStream_t s);
int count_persistent_blocks_per_cu();

}  // namespace bbtc
