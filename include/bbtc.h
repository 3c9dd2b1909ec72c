/*
 * bbtc.h -- C ABI of the MI355X block-based triangle counting library.
 *
 * Method: Yasar, Rajamanickam, Berry, Catalyurek, "Block-Based Triangle
 * Counting Algorithm for Heterogeneous Environments" (arXiv 2009.12457).
 *
 *   - Vertices are renumbered in non-decreasing degree order and every edge
 *     is kept once, from the lower to the higher rank (Sec. 2 and 4.1).
 *   - The rank range is cut into p contiguous parts V_0..V_{p-1} with one cut
 *     vector for rows and columns (symmetric rectilinear partition, Sec. 4.1);
 *     block G_ab holds the edges from V_a to V_b, a <= b.
 *   - Every triple i <= j <= k is a task over the blocks G_ij, G_jk, G_ik
 *     (Sec. 4.2, Alg. 4), |T| = p(p+1)(p+2)/6.
 *   - A task counts, for each u in V_i and each v in N(G_ij,u), the common
 *     elements of N(G_ik,u) and N(G_jk,v) (Sec. 4.3, the Intersect and HMap
 *     per-task algorithms).  Each triangle is counted by exactly one task, so
 *     the total is the sum of the per-task counts.
 *
 * All counting is exact 64-bit integer arithmetic.
 *
 * Conventions for every entry point:
 *   - No exception crosses this boundary; every call returns a status and a
 *     failing call leaves a message for bbtc_last_error() on that thread.
 *   - Input buffers stay owned by the caller and may be freed as soon as the
 *     call returns (the library copies what it keeps).
 *   - A plan owns all of its host and device memory; it is used by one stream
 *     at a time.  Different plans may be used concurrently.
 *   - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *     null stream).
 */
#ifndef BBTC_H_
#define BBTC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bbtc_status;
#define BBTC_OK 0
#define BBTC_EINVAL (-1)  /* malformed graph, options or arguments */
#define BBTC_ENOMEM (-2)  /* a host or device allocation failed */
#define BBTC_EBUDGET (-3) /* the device budget cannot hold even one unit of work */
#define BBTC_EDEVICE (-4) /* a HIP call failed */
#define BBTC_ESTATE (-5)  /* the call does not fit the plan's state */

/* bbtc_csr.flags */
#define BBTC_CSR_DEVICE 1u  /* rowptr/colidx are device pointers (else host) */
#define BBTC_CSR_TRUSTED 2u /* skip the O(nnz log d) symmetry check */

/*
 * A simple undirected graph G=(V,E) (Sec. 2) as a symmetric CSR: both
 * directions of every edge are stored, each row strictly increasing, no
 * self-loops.  n = |V| < 2^31; nnz = 2|E| and |E| < 2^32.
 * rowptr has n+1 entries of rowptr_bits (32 or 64) bits, rowptr[0] = 0 and
 * rowptr[n] = nnz.  colidx has nnz entries in [0, n).
 * Host inputs are validated on the host before any device call (with
 * BBTC_CSR_TRUSTED only their rowptr; their entries are then checked by a
 * kernel right after the upload); device inputs are validated by a kernel.
 * Either way a violation returns BBTC_EINVAL.
 */
typedef struct bbtc_csr {
  int64_t n;
  int64_t nnz;
  const void* rowptr;
  int32_t rowptr_bits;
  uint32_t flags;
  const int32_t* colidx;
} bbtc_csr;

/* bbtc_options.mode */
#define BBTC_MODE_PERSISTENT 0      /* one work-stealing launch over all tasks */
#define BBTC_MODE_PLAIN_INTERSECT 1 /* one launch per task, every list probed by
                                       binary search in a sorted LDS copy */
#define BBTC_MODE_PLAIN_HMAP 2      /* one launch per task, every list staged
                                       alone as an LDS bitmap or hash (wave_min
                                       and hash_min are ignored) */

/* bbtc_options.cut_mode */
#define BBTC_CUT_BALANCED 0 /* parts of ~m/p oriented entries each */
#define BBTC_CUT_UNIFORM 1  /* parts of ~n/p vertices each */

/*
 * Tuning knobs.  None of them changes any result: every choice counts each
 * triangle exactly once.  Zero selects the library default.
 *   p             blocks per side, 1 <= p <= min(n, 2048); 0 = p from the
 *                 average degree (Sec. 7.3 suggests p near the average degree).
 *   wave_min      a column v of G_ij whose list N(G_jk,v) has at least
 *                 wave_min entries (default 32; capped at the 512-word
 *                 wavefront stage) is staged alone and
 *                 probed by a whole 64-lane wavefront; shorter lists of the
 *                 columns a workgroup holds are staged together, sorted, and
 *                 probed by binary search by all its lanes.
 *   hash_min      wavefront columns with |N(G_jk,v)| >= hash_min stage it as an
 *                 LDS bitmap over V_k or an LDS hash (the HMap form); shorter
 *                 ones as a sorted LDS copy probed by binary search (the
 *                 Intersect form).  -1 = never.
 *   grid          workgroups of the persistent launch; 0 = by occupancy.
 *   item_rows     active columns of G_ij per persistent work item.
 *   graph         0: the persistent count (reset + launch) is captured once
 *                 in a hipGraph and replayed; -1: launched directly.
 *   device_budget_bytes  upper bound on the device memory a plan holds for
 *                 the count (0 = none).  A plan over the budget keeps its
 *                 count-phase arrays in pinned host memory and streams, per
 *                 block pair (i,j), what its tasks read (Sec. 4.1: a task
 *                 needs only its three blocks): the out-rows of V_i and V_j
 *                 with their stored block boundaries (two out-stripes, cached
 *                 least recently used first) and block (i,j)'s in side.  When
 *                 the resident partition itself would not fit, bbtc_partition
 *                 builds the plan in pieces (input rows in chunks, parts in
 *                 groups as large as the budget allows) straight into pinned
 *                 host memory.  BBTC_EBUDGET when the budget cannot hold the
 *                 degree order, the build of a single part, or two out-stripes
 *                 beside two in-block slots.
 *   bound_min_deg the block row index (Sec. 4.1) stores, for a vertex of
 *                 undirected degree above bound_min_deg, the position of each
 *                 block's slice in its out-row; rows of lower degree (a
 *                 prefix of the degree order) store nothing and the counting
 *                 kernels find their slices by scanning the short row.  The
 *                 stored index then stays small for any p.  0 = automatic:
 *                 the smallest of {0, 8, 16, 32} whose stored boundaries take
 *                 at most 4m bytes (the size of the out-rows), else 32 (and
 *                 32 for plans partitioned in pieces within a device budget,
 *                 whose boundaries stream with the out-rows); -1 = store
 *                 every row.
 *   dense         plans held on the device keep the dense slices of their
 *                 last parts as bitmaps too (see bbtc_partition): 0 = for
 *                 graphs of at least 2^22 edges, 1 = always, -1 = never.
 */
typedef struct bbtc_options {
  int32_t p;
  int32_t cut_mode;
  int32_t mode;
  int32_t wave_min;
  int32_t hash_min;
  int32_t grid;
  int32_t item_rows;
  int32_t graph;
  int64_t device_budget_bytes;
  int32_t bound_min_deg;
  int32_t dense;
} bbtc_options;

/* Task kinds: EMPTY tasks have an empty block and count 0 without work. */
#define BBTC_TASK_EMPTY 0
#define BBTC_TASK_WORK 1

/*
 * One task {i,j,k}, i <= j <= k (Sec. 4.2).  `est` is the workload estimate
 * |E(G_ij)| * max(delta(G_ik), delta(G_jk)) with delta(G_ab) = |E(G_ab)|/|V_a|
 * (Sec. 5), used only to order the work (non-increasing, ties by (i,j,k)).
 */
typedef struct bbtc_task {
  int32_t i, j, k;
  int32_t kind;
  double est;
} bbtc_task;

/* Plan statistics (the quantities of the complexity analysis, Sec. 4.4). */
typedef struct bbtc_stats {
  int64_t n, m, p;
  int64_t ntasks, work_tasks, nitems;
  int64_t m_max;        /* largest block |E(G_ab)| */
  double m_avg;         /* 2m / (p(p+1)) */
  double lambda;        /* m_max / m_avg */
  int64_t d_max;        /* largest oriented degree */
  int64_t d_max_block;  /* largest partial degree d(G_ab,u) */
  double c;             /* d_max / d_max_block */
  int64_t wedges;       /* sum over oriented edges (u,v) of d(G,v): the probe volume */
  int64_t bytes_colidx; /* 4 * (p+2) * m: each task's three blocks read once */
  int64_t bytes_rowidx; /* block row-index bytes the tasks read */
  int64_t bytes_total;  /* bytes_colidx + bytes_rowidx + 8 |T| */
  int64_t footprint;    /* device bytes held by the plan */
  double partition_ms;  /* wall time of the last bbtc_partition */
  int64_t streamed;     /* 1: over the device budget, stripes stream from pinned host memory */
  int64_t stripe_slots; /* stripes the device cache holds (streamed plans) */
  int64_t stripe_bytes; /* bytes per stripe slot */
  int64_t stripe_uploads; /* stripe and block uploads by the last bbtc_count (streamed plans) */
  int64_t resident_bytes; /* device bytes of the count phase with every stripe and block resident */
  int64_t stored_rows;    /* rows with stored block boundaries (ranks n - stored_rows .. n-1) */
  int64_t bound_bytes;    /* bytes of the stored block boundaries */
  int64_t dense_slices;   /* slices N(G_ik,u) also held as bitmaps over V_k (see bbtc_partition) */
  int64_t dense_bytes;    /* bytes of those bitmaps */
} bbtc_stats;

typedef struct bbtc_plan bbtc_plan;

/* Fills `opt` with the defaults (all knobs 0 = automatic, persistent mode). */
void bbtc_options_default(bbtc_options* opt);

/*
 * Degree ordering, orientation, symmetric rectilinear cut, block row
 * indices and the task list (Sec. 4.1, 4.2, 5), all computed on the device.
 * If *plan is NULL a new plan is created, otherwise it is rebuilt in place,
 * reusing its device buffers when they are large enough.  Returns when the
 * plan is ready (the call synchronises `stream`).  On failure *plan is left
 * as it was (a new plan is not created).  A plan held on the device of a
 * graph of at least 2^22 edges (bbtc_options.dense) also keeps, for the
 * rows of its last parts (at most 65536 vertices) and the
 * blocks of those parts, every slice N(G_ik,u) with at least |V_k|/16
 * entries as a bitmap over V_k as well (no larger than the 16-bit list);
 * the count probes such a slice word by word against a column's staged
 * bitmap (bbtc_stats.dense_slices).
 */
bbtc_status bbtc_partition(const bbtc_csr* g, const bbtc_options* opt, void* stream, bbtc_plan** plan);

/*
 * Counts every task of the plan (Sec. 4.3) and the total.  d_per_task is
 * device memory for ntasks uint64 in the order of bbtc_plan_tasks; d_total
 * is device memory for one uint64.  Both are overwritten.  Asynchronous:
 * results are valid once `stream` has completed the enqueued work.
 */
bbtc_status bbtc_count(bbtc_plan* plan, void* stream, uint64_t* d_per_task, uint64_t* d_total);

/*
 * Several plans counted by shared persistent launches (continuous batching).
 * d_per_task[q] and d_totals + q receive plan q's results, exactly as
 * bbtc_count would.  The launch reads every plan's own device buffers (its
 * work items included), so plans must not be in use on another stream or
 * re-partitioned until `stream` has completed it.  BBTC_ESTATE for a plan
 * that is not ready or that streams under a device budget; BBTC_EINVAL for
 * null arguments or more than 2^32 - 1 work items in total.  Asynchronous,
 * like bbtc_count.
 */
bbtc_status bbtc_count_multi(bbtc_plan* const* plans, int32_t nplans, void* stream,
                             uint64_t* const* d_per_task, uint64_t* d_totals);

/*
 * Hybrid execution (Sec. 5, Alg. 5-7; Sec. 7.8): the GPU and host threads
 * count the plan's tasks together.  Tasks are in the plan's order
 * (non-increasing estimate); the GPU counts the tasks before `cutoff` (plan
 * order index) with the persistent kernel, host threads take tasks one at a
 * time from the back of the list and never below `cutoff`, and once its
 * first share is done the GPU claims half of the tasks still between the two
 * sides at a time until they meet.  Host threads count by list intersection
 * (Alg. 1) over host copies of the plan's tables, made on the first call
 * for a plan build (O(m) host memory).  cutoff -1 = |T|/2; cutoff |T| = the
 * GPU alone.  cpu_threads 0 = the hardware threads minus one, at most 16.  Results as
 * bbtc_count, but the call is synchronous: it returns when they are in
 * d_per_task/d_total (`stream` is synchronised).  Not for streamed plans
 * (BBTC_ESTATE).  `stats` (may be NULL) reports the split.
 */
typedef struct bbtc_hybrid_stats {
  int64_t gpu_tasks, cpu_tasks;  /* non-empty tasks counted by each side */
  int64_t gpu_launches;          /* persistent launches of the GPU side */
  int64_t cutoff;                /* the cut-off used */
  int64_t split;                 /* the host threads counted tasks [split, |T|) */
  int32_t cpu_threads;
  int32_t pad;
  double cpu_ms;                 /* longest busy time of a host thread */
  double total_ms;               /* wall time of the call */
  uint64_t cpu_triangles;        /* triangles counted by the host threads */
} bbtc_hybrid_stats;
bbtc_status bbtc_count_hybrid(bbtc_plan* plan, void* stream, uint64_t* d_per_task, uint64_t* d_total,
                              int32_t cpu_threads, int64_t cutoff, bbtc_hybrid_stats* stats);

/*
 * For callers that cannot allocate memory (code under stream capture, tight
 * serving loops, harnesses that forbid allocation): bbtc_count_multi with
 * the state of the shared launch (the plans' kernel contexts, their item
 * offsets and the work-queue cursors) kept in a fixed device array of the
 * library (BBTC_STATIC_BYTES per device, held until the process ends)
 * instead of memory allocated per call.  The successful path calls no
 * allocating routine (no hipMalloc/hipFree, no pinned host memory, no
 * events, no host heap).  At most BBTC_STATIC_MAX_PLANS plans per call,
 * else BBTC_EINVAL.  Every call on a device shares that device's array, and
 * each call rewrites it: calls that overlap on one device (on different
 * streams, or before an earlier call's work on another stream has
 * completed) race and give wrong results; calls in order on one stream are
 * safe.  Arguments, results and the other errors as bbtc_count_multi.
 */
#define BBTC_STATIC_MAX_PLANS 64
#define BBTC_STATIC_BYTES 32768
bbtc_status bbtc_count_multi_static(bbtc_plan* const* plans, int32_t nplans, void* stream,
                                    uint64_t* const* d_per_task, uint64_t* d_totals);

/*
 * Autotuner.  Picks p, wave_min and hash_min for this graph by timing the
 * persistent count (HIP events on `stream`, median of `reps` launches after
 * one warm-up) by coordinate descent: first p over {p0/4, p0/2, p0, 2*p0}
 * (p0 = base->p, or the average degree when base->p is 0: Sec. 7.3 of the
 * paper suggests p near the average degree), continuing by halving below
 * p0/4 (doubling above 2*p0) while the count gets faster, then wave_min over
 * {16, 32, 64, 128, 256, 512}, then hash_min over {-1, 1, 32, 256}; a threshold
 * leaves its current value only for a candidate more than 3% faster (so that
 * timing noise does not decide between near-equal values).  The other fields of
 * *base are kept.  Every candidate gives identical counts; only time differs.
 * On success *out holds the chosen options and *best_ms (if not NULL) the
 * count time with them.  Synchronises `stream`.
 */
bbtc_status bbtc_autotune(const bbtc_csr* g, const bbtc_options* base, int32_t reps, void* stream,
                          bbtc_options* out, double* best_ms);

/* Borrowed host views, valid until the plan is rebuilt or destroyed. */
bbtc_status bbtc_plan_tasks(const bbtc_plan* plan, const bbtc_task** tasks, int64_t* ntasks);
bbtc_status bbtc_plan_cuts(const bbtc_plan* plan, const int32_t** cuts, int32_t* p);
/* Block sizes |E(G_ab)|, a <= b, row-major: p(p+1)/2 entries. */
bbtc_status bbtc_plan_block_nnz(const bbtc_plan* plan, const int64_t** nnz, int64_t* nblocks);
bbtc_status bbtc_plan_stats(const bbtc_plan* plan, bbtc_stats* out);

/*
 * Copies of device-resident plan arrays into caller memory (host or device),
 * enqueued on `stream` and complete when it is.
 *   perm: n int32, the rank of each original vertex id.
 *   orow: n+1 uint32 and ocol: m int32, the oriented CSR in rank space.
 */
bbtc_status bbtc_plan_copy_perm(const bbtc_plan* plan, int32_t* dst, void* stream);
bbtc_status bbtc_plan_copy_oriented(const bbtc_plan* plan, uint32_t* orow, int32_t* ocol, void* stream);

void bbtc_plan_destroy(bbtc_plan* plan);

/*
 * Diagnostics: consistency of the block tables the counting kernels index
 * (Sec. 4.1's blocks in the layout described below), checked on the host
 * against their definitions from the oriented CSR.
 *
 * bbtc_tables: host arrays of one plan.  n vertices, m oriented edges, p
 * parts, cut vector cuts[p+1]; out-rows orow[n+1]/ocol[m] (ranks above the
 * row's rank, ascending).  Ranks below rT store no block boundaries; part a
 * stores the s_a = cuts[a+1] - max(cuts[a], rT) rows max(cuts[a], rT) ..
 * cuts[a+1]-1, p-a+1 positions per stored row, column-major from botp[a] on:
 * entry b-a of stored row r (the first position of the out-row with a column
 * >= cuts[b]; entry p-a = the row end) at botp[a] + (b-a) s_a + r.  The in side is
 * block-major: per block (a,b) in column-major order cid = b(b+1)/2 + a,
 * acol lists from acp[cid] on the columns v of V_b with an in-neighbour in
 * V_a, ascending, and active column x's in-neighbours in V_a (in any order)
 * are icolb[aoff[x] .. aoff[x+1]); the slices lie back to back from 0 to m.
 * Returns BBTC_OK, or BBTC_EINVAL with the first violation in
 * bbtc_last_error().  Pure host code: no device is needed.
 */
typedef struct bbtc_tables {
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
} bbtc_tables;
bbtc_status bbtc_check_tables(const bbtc_tables* tables);

/*
 * Copies a plan's tables and work items to the host (synchronising `stream`)
 * and checks them: the tables as bbtc_check_tables, every dense slice's
 * bitmap against its slice (and that exactly the slices with at least
 * |V_k|/16 entries have one), and every work item within its task's active
 * columns or hub in-slice, the items of each task covering its columns
 * exactly once.  BBTC_EDEVICE names the first violation.  O(m + p^2 + items
 * + bitmap words) host work, for tests and debugging.
 */
bbtc_status bbtc_plan_verify(const bbtc_plan* plan, void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* bbtc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BBTC_H_ */
