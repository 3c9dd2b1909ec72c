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
//           of the hub column with absolute active-column index v (its
//           in-slice is longer than the split threshold); such columns are
//           skipped by column-range items.
struct DevItem {
  int32_t task;
  uint32_t lo, hi;
  int32_t v;
};

// An active column of block (a,b) whose in-slice from V_a has more than
// `split` entries (collected while the active columns are written).
struct HeavyCol {
  uint32_t cid;  // column-major block id of (a,b)
  uint32_t x;    // absolute active-column index (acol[x] is the vertex)
  uint32_t cnt;  // in-slice length
};

// Device view of the blocked graph (stripe layout plus block row index).
//   orow/ocol : oriented CSR in rank space, every row ascending; ocol is
//           16-byte aligned on absolute positions and padded by four
//           entries, so rows can be read in aligned 16-byte blocks.
//   rT    : ranks below rT (undirected degree <= the plan's bound_min_deg,
//           a prefix of the degree order) have no stored boundaries; their
//           block slices are found by scanning the row.  A part a stores
//           rows max(cuts[a], rT) .. cuts[a+1]-1.
//   bot   : for a stored row u in part a, (p-a+1) absolute positions in
//           ocol; entry b-a is the first position of N(G,u) whose column is
//           >= cuts[b], so N(G_ab,u) = ocol[bot[b-a] .. bot[b-a+1]).  Stored
//           rows of part a start at element botp[a], (p-a+1) entries apart.
//   acol  : per block (a,b), the columns v of V_b with a non-empty in-slice
//           in increasing order, starting at acp[cid(a,b)], cid = b(b+1)/2+a
//           (column-major block order).
//   aoff/icol : the in-side, block-major: active column x's in-slice (its
//           in-neighbours in V_a) is icol[aoff[x] .. aoff[x+1]).
struct GraphView {
  int32_t p;
  uint32_t m;  // entries of ocol (and of icol)
  int32_t rT;
  int32_t pad;
  const uint32_t* orow;
  // Streamed launches cover the tasks of one block pair (gi, gj) and read the
  // out-rows of parts gi and gj from cached stripes and block (gi,gj)'s
  // in-side from a staged copy: colI/colJ are shifted so that the absolute
  // positions of orow and bot index them, botI/botJ point at the first stored
  // boundary row of the part, acolJ/aoffJ/icolJ are shifted so that absolute
  // active-column indices and entry positions index them.  gi < 0: the whole
  // graph is resident and the fields below are used instead.
  int32_t gi, gj;
  const int32_t* colI;
  const int32_t* colJ;
  const uint32_t* botI;
  const uint32_t* botJ;
  const int32_t* acolJ;
  const uint32_t* aoffJ;
  const int32_t* icolJ;
  const int32_t* cuts;
  const uint64_t* botp;
  const uint32_t* bot;
  const int32_t* ocol;
  // ocol16[e] = ocol[e] - c_k for the part k holding ocol[e] (16 bits; used
  // only for parts of at most 65536 vertices), same positions, padded to a
  // multiple of 8 entries; nullptr: not built (streamed plans)
  const uint16_t* ocol16;
  const uint64_t* acp;
  const int32_t* acol;
  const uint32_t* aoff;
  const int32_t* icol;
  // Dense slices as bitmaps (resident plans): for the rows u >= dense_u0 (the
  // last parts, at most kDenseRows vertices) and the blocks k >= dense_k0,
  // dslot[(u - dense_u0) * (p - dense_k0) + (k - dense_k0)] is 0, or 1 + the
  // word offset in dbits of N(G_ik,u) as a bitmap over V_k (bit x of word
  // x / 32 for vertex c_k + x; ceil(|V_k|/32) words rounded up to 8, zero
  // padded) when the slice holds at least |V_k|/16 entries.  dslot null: none.
  int32_t dense_u0, dense_k0;
  const uint32_t* dslot;
  const uint32_t* dbits;
};
constexpr int64_t kDenseRows = 65536;

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
// A range of input rows for the degree and fill passes: local row x is
// original vertex x0 + x; the graph has ntot vertices; the range's row
// pointers lie in [nnz_lo, nnz_hi]; the fill writes only rows whose rank is
// in [rlo, rhi).
struct RowRange {
  int64_t x0, ntot, nnz_lo, nnz_hi;
  int32_t rlo, rhi;
};
inline RowRange whole_rows(int64_t n, int64_t nnz) { return RowRange{0, n, 0, nnz, 0, (int32_t)n}; }
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
// od == nullptr: list the long and huge rows only (no degrees).  rc (may be
// null): receives, at each input position, the rank of that entry's vertex,
// which the fill then reads instead of gathering it again.
hipError_t launch_degs(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, const RowRange& rr,
                       const int32_t* perm, uint32_t* od, uint32_t* idg, uint32_t* list, uint32_t* nlist,
                       uint32_t* hlist, uint32_t* nhlist, uint32_t* hpref, uint32_t* err, int check, int32_t* rc,
                       hipStream_t s);
// cur_o/cur_i: zeroed fill cursors of the huge rows (indexed by position in
// hlist); rc: the ranks written by launch_degs over the same rows, or null.
hipError_t launch_fill(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, const RowRange& rr,
                       const int32_t* perm,
                       const uint32_t* orow, const uint32_t* irow, int32_t* ocol, int32_t* icol, const uint32_t* list,
                       const uint32_t* nlist, const uint32_t* hlist, const uint32_t* nhlist, const uint32_t* hpref,
                       uint32_t* cur_o, uint32_t* cur_i, const int32_t* rc, hipStream_t s);
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
// The first `cap` rows of the combined list (huge rows, then long ones) are
// grouped in chunks spread over the chip: chunks holds room for m / 4096 +
// cap entries, *nchunks is zero on entry, cnt has room for cap * p words.
// cap = 0: every listed row by one workgroup.
struct GroupChunks {
  uint32_t cap;
  uint2* chunks;
  uint32_t* nchunks;
  uint32_t* cnt;
  uint32_t* rowmap;  // n words: rowmap[row] = its combined list index, for the rows taken
  uint32_t max_chunks;  // bound on the chunks (sizes the launches)
  bool all_taken;       // cap holds every row the lists can have (the per-row kernels are skipped)
};
constexpr uint32_t kGroupChunkEntries = 4096;
hipError_t launch_inrows_group(const uint32_t* rp, int32_t* col, const uint32_t* longrows, const uint32_t* hugerows,
                               const uint32_t* q, int32_t* scratch, const int32_t* cuts, int32_t p,
                               const GroupChunks& gc, hipStream_t s);
// Four degree thresholds (a negative one counts no rank).
struct DegThresholds {
  int64_t t[4];
};
// *wedges += sum over r < n of od[r] * idg[r] (the wedge count W) and
// nshort[q] += #{r : od[r] + idg[r] <= th.t[q]} for q < 4.
hipError_t launch_degree_stats(const uint32_t* od, const uint32_t* idg, int64_t n, const DegThresholds& th,
                               unsigned long long* wedges, uint32_t* nshort, hipStream_t s);
hipError_t launch_cuts(const uint32_t* orow, int64_t n, int32_t p, int mode, int32_t* cuts, hipStream_t s);
// ocol16[e] = ocol[e] - (first vertex of the part holding ocol[e]) for e < m,
// zero up to the next multiple of 8.
// Dense slices as bitmaps (see GraphView): one wavefront per (row, block)
// pair of the rows [cuts[k0], n) and blocks [k0, p); words of dbits are
// handed out from nwords[0] up to cap, nwords[1] counts the dense slices.
hipError_t launch_dense_build(const uint32_t* orow, const int32_t* ocol, const uint16_t* ocol16, const uint32_t* bot,
                              const uint64_t* botp, const int32_t* cuts, int32_t p, int32_t rT, int32_t k0, int64_t n,
                              int64_t npairs, uint32_t* dslot, uint32_t* dbits, uint32_t* nwords, uint64_t cap,
                              hipStream_t s);
hipError_t launch_ocol16(const int32_t* ocol, uint64_t m, const int32_t* cuts, int32_t p, uint16_t* ocol16,
                         hipStream_t s);

struct BlockBuild {
  int32_t p;
  int32_t rT;                // first rank with stored boundaries (see GraphView)
  int32_t nchunks;           // total row chunks (kPrepRows rows each, within one part)
  int32_t chunk_base;        // chunk of the launch's first workgroup
  const int32_t* cuts;       // p+1
  const int32_t* chunk0;     // p+1: first chunk of each part
  const uint64_t* ccbase;    // p+1: start of part b's chunk counters (in side)
  const uint32_t* orow;
  const int32_t* ocol;
  const uint64_t* botp;
  uint32_t* bot;
  const uint32_t* irow;       // in-rows (grouped by part) of the columns built
  const int32_t* icol;
  unsigned long long* bnnz;  // nb, row-major block order
  unsigned long long* bnzr;  // nb, row-major block order
  unsigned long long* bnzc;  // nb, column-major block order cid(a,b) = b(b+1)/2 + a
  uint32_t* ccnt;            // per (part b, block (a,b), chunk) active-column counts
  uint32_t* ecnt;            // the same for their in-slice entries
  uint32_t* dmax_block;      // [0] longest block slice, [1] longest oriented row
  const uint32_t* ccoff;     // exclusive scans of ccnt and ecnt (indexed like them)
  const uint32_t* ecoff;
  int32_t* acol;             // active columns, column-major block order (indexed by ccoff)
  uint32_t* aoff;            // their in-slice offsets in the block-major in-side
  uint32_t* asrc;            // their in-slice starts in icol
  uint32_t ebase;            // block-major entry offset of the first column built
  uint64_t xbase;            // absolute active-column index of acol[0]
  uint32_t split;            // in-slice length above which a column is recorded as heavy
  HeavyCol* heavy;           // room for m/split + 1 records
  uint32_t* nheavy;
  uint32_t heavy_cap;
  // In-rows grouped in chunks (launch_inrows_group): rowmap[v] is the
  // combined list index of row v when it was (checked against the lists,
  // the value is stale otherwise), gcnt + index * p the ends of its part runs
  // relative to the row start; rowmap null: none.
  const uint32_t* rowmap;
  const uint32_t* gcnt;
  const uint32_t* glong;
  const uint32_t* ghuge;
  const uint32_t* gq;
  uint32_t gcap;
};
// Chunks [bb.chunk_base, bb.chunk_base + nchunks) of the parts.
hipError_t launch_bot(const BlockBuild& bb, int nchunks, hipStream_t s);
hipError_t launch_acount(const BlockBuild& bb, int nchunks, hipStream_t s);
hipError_t launch_acol(const BlockBuild& bb, int nchunks, hipStream_t s);
// Copies the in-slices of *ncolsp active columns (at most ncols_max;
// aoff/asrc/icol/icolb shifted as in k_acol) into the block-major in side;
// hub records [h0, min(*h1p, cap)) (absolute indices, xbase = absolute index
// of aoff[0]) by one workgroup each.
hipError_t launch_icolb(const uint32_t* aoff, const uint32_t* asrc, const int32_t* icol, int32_t* icolb,
                        const uint32_t* ncolsp, uint64_t ncols_max, uint32_t split, const HeavyCol* heavy, uint32_t h0,
                        const uint32_t* h1p, uint32_t cap, uint64_t xbase, hipStream_t s);
// arr[*idx] = value (one thread).
hipError_t launch_set_at(uint32_t* arr, const uint32_t* idx, uint32_t value, hipStream_t s);

// Work-item emission on the device.  A run sends items [r0, r0 + n) of
// plan-order task `task` to out[dst, dst + n); the runs are sorted by dst,
// non-empty, and tile [0, nitems).  Item r of a task is its r-th hub chunk
// while r < nhub (chunks of `chunk` in-neighbours, hub records of block cid
// in hrec[hstart[cid], hstart[cid+1]) with their first chunk numbers in
// hcum; the item's v is the record's active-column index), else active
// columns [(r - nhub) * nper, +nper) clipped to cols.
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
// *x += v (one thread).
hipError_t launch_add_u64(uint64_t* x, uint64_t v, hipStream_t s);

}  // namespace bbtc
