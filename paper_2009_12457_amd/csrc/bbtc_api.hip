// Host runtime of the C ABI declared in include/bbtc.h.
//
// bbtc_partition runs the preprocessing kernels (validation, degree order,
// orientation, cut vector, block row index) and composes the task list
// (arXiv 2009.12457, Alg. 4) with the workload estimate of Sec. 5 on the
// host from the p(p+1)/2 block sizes.  bbtc_count enqueues the counting
// kernels: one work-stealing launch (persistent mode) or one launch per task
// on four side streams (plain modes, the paper's per-task execution with
// n_s = 4 streams per GPU, Sec. 5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <condition_variable>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "bbtc_internal.h"
#include "cpu_count.h"
#include "plan_check.h"

using namespace bbtc;

namespace {

thread_local std::string g_err;

bbtc_status fail(bbtc_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

bbtc_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(BBTC_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
  return fail(BBTC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call, what)                      \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

template <typename T>
struct DevBuf;
template <typename T>
hipError_t ensure_pow2(DevBuf<T>& b, size_t n);

template <typename T>
struct DevBuf {
  T* ptr = nullptr;
  size_t cap = 0;  // elements
  hipError_t ensure(size_t n) {
    if (n == 0) n = 1;
    if (ptr && n <= cap) return hipSuccess;
    release();
    hipError_t e = hipMalloc((void**)&ptr, n * sizeof(T));
    if (e != hipSuccess) {
      ptr = nullptr;
      cap = 0;
      return e;
    }
    cap = n;
    return hipSuccess;
  }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    cap = 0;
  }
  size_t bytes() const { return cap * sizeof(T); }
};

// ensure() rounded up to a power of two: for the buffers whose size follows
// each graph (a plan rebuilt for graphs of many sizes, as in serving, then
// rarely reallocates, and hipFree waits for the whole device)
template <typename T>
hipError_t ensure_pow2(DevBuf<T>& b, size_t n) {
  if (b.ptr && n <= b.cap) return hipSuccess;
  size_t r = 1;
  while (r < n) r <<= 1;
  return b.ensure(r);
}

int bits_for(uint64_t maxval) {  // bits to hold values 0..maxval
  int b = 1;
  while (b < 63 && (maxval >> b) != 0) ++b;
  return b;
}

}  // namespace

// Pinned host staging for the small transfers of a partition (sizes, cut
// vector, block statistics, task list): copies to and from pinned memory
// are asynchronous DMA, copies to pageable memory each cost a round trip.
struct PinnedStage {
  char* ptr = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes) {
    if (ptr && bytes <= cap) return hipSuccess;
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    cap = 0;
    const size_t want = std::max<size_t>(bytes, 1 << 16);
    hipError_t e = hipHostMalloc((void**)&ptr, want, hipHostMallocDefault);
    if (e == hipSuccess) cap = want; else ptr = nullptr;
    return e;
  }
  ~PinnedStage() {
    if (ptr) (void)hipHostFree(ptr);
  }
};

struct bbtc_plan {
  int64_t n = 0, m = 0;
  int32_t p = 0;
  bbtc_options opt{};
  int idbits = 1;
  int64_t rT = 0;  // first rank with stored block boundaries
  bool ready = false;
  // device
  DevBuf<char> in_rowptr;
  DevBuf<int32_t> in_col;
  DevBuf<uint64_t> keys_a, keys_b;
  DevBuf<uint32_t> hist, partial;
  DevBuf<int32_t> perm, order, ocol, icol, cuts, acol;
  DevBuf<uint32_t> od, idg, orow, irow, midrows, longrows, hugerows, bot, ccnt, ccoff, cursor, err, aoff, asrc;
  DevBuf<int32_t> icolb;  // the block-major in side (icol is the vertex-major one it is built from)
  DevBuf<uint16_t> ocol16;  // out-rows relative to the part of each entry (resident plans)
  DevBuf<int32_t> rc;       // rank of each input entry's vertex, between the degree pass and the fill
  DevBuf<uint64_t> acp;
  // Per-part index tables (uploaded together) and per-block statistics with
  // their counters (cleared and read back together), in one allocation:
  // chunk0[p+1] | ccbase, botp [p+1] | head[4] = {hub records, dmax x2,
  // -} | bnnz, bnzr, bnzc [nb]
  DevBuf<char> blk;
  int32_t* chunk0 = nullptr;
  uint64_t *ccbase = nullptr, *botp = nullptr;
  uint32_t* head = nullptr;
  unsigned long long *bnnz = nullptr, *bnzr = nullptr, *bnzc = nullptr;
  DevBuf<DevTask> tasks;
  DevBuf<DevItem> items;
  DevBuf<DevItem> xitems;          // the same items as per-XCD queues (persistent launches)
  DevBuf<HeavyCol> heavy;
  DevBuf<char> emit;               // inputs of the item-emission kernel
  DevBuf<char> grp;                // chunk list and part counters of the chunked in-row grouping (partition only)
  // dense slices of the last parts as bitmaps (GraphView::dslot, dbits) and
  // their counters {words handed out, slices}
  DevBuf<uint32_t> dslot, dbits, dcount;
  int32_t dense_k0 = 0;            // first block with dense slices (p: none)
  int64_t dense_slices = 0, dense_words = 0;
  // host
  std::vector<int32_t> h_cuts;
  std::vector<int64_t> h_nnz, h_nzr, h_nzc;  // nzc in column-major block order
  std::vector<bbtc_task> h_tasks;  // plan order (LPT)
  std::vector<DevTask> h_dtasks;   // same order
  std::vector<int32_t> h_work;     // plan-order indices of WORK tasks
  std::vector<DevItem> h_items;
  PinnedStage stage;
  PinnedStage cstage;              // the cut vector, read back while the rows are sorted
  std::vector<ItemRun> h_runs;     // the per-XCD queues as runs of task items (sorted by position)
  uint32_t nq = 1, qbeg[kMaxQueues] = {0}, qlen[kMaxQueues] = {0};
  std::vector<HeavyCol> h_heavy;   // hub columns, sorted by (block, column)
  std::vector<int64_t> h_hub_first, h_hub_count;  // per plan-order task: its range of h_items
  // per plan-order task: work items, columns per range item, hub-chunk items;
  // hub records per block
  std::vector<uint32_t> h_nitem, h_nper, h_nhub;
  std::vector<int64_t> h_hstart;
  size_t nitems = 0;                // work items of the plan (either layout)
  double est_sum = 0;               // sum of the task estimates (orders plans in shared launches)
  uint32_t split = 0;              // in-slice length above which a column is a hub
  int64_t ccount = 0;              // number of chunk counters
  int ncu = 0, blocks_per_cu = 0;
  hipStream_t side[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_cuts = nullptr;  // the cut vector has reached the host (cstage)
  // ---- budgeted streaming of the count phase (see stream_setup)
  bool streamed = false;
  // pinned host copies of the count-phase arrays: out-rows and their stored
  // boundaries, the block-major in side with its active columns
  int32_t* h_ocol = nullptr;
  uint32_t* h_bot = nullptr;
  uint32_t* h_orow = nullptr;
  int32_t* h_acol = nullptr;
  uint32_t* h_aoff = nullptr;
  int32_t* h_icolb = nullptr;
  std::vector<uint64_t> h_botp, ocut, h_acp;  // part offsets; orow at the cuts; active-column offsets
  DevBuf<char> cache;            // out-stripe slots, then the two in-block slots
  size_t slot_bytes = 0, block_bytes = 0;
  struct Slot {
    int key = -1;                // out-stripe of part `key` (block slots: unused)
    uint64_t last = 0;
    bool used = false;           // a kernel has read it (released is recorded)
    hipEvent_t ready = nullptr, released = nullptr;
  };
  std::vector<Slot> slots;       // out-stripe slots
  Slot bslot[2];                 // in-block slots, alternating between block pairs
  uint64_t clock = 0;
  std::vector<std::pair<int32_t, int32_t>> groups;  // block pairs (i,j) in the walk order (stream_finish)
  std::vector<std::vector<int64_t>> stripe_uses;    // per part: the walk positions of the pairs reading it
  std::vector<int64_t> group_first, group_count;    // their ranges of the item list
  int64_t copies = 0;            // stripe and block uploads by the last streamed count
  int64_t resident_bytes = 0;    // count-phase bytes with every stripe and block resident
  void drop_stream() {
    for (auto& s : slots) {
      if (s.ready) (void)hipEventDestroy(s.ready);
      if (s.released) (void)hipEventDestroy(s.released);
    }
    slots.clear();
    for (auto& s : bslot) {
      if (s.ready) (void)hipEventDestroy(s.ready);
      if (s.released) (void)hipEventDestroy(s.released);
      s = Slot();
    }
    cache.release();
    for (void* h : {(void*)h_ocol, (void*)h_bot, (void*)h_orow, (void*)h_acol, (void*)h_aoff, (void*)h_icolb})
      if (h) (void)hipHostFree(h);
    h_ocol = h_acol = h_icolb = nullptr;
    h_bot = h_orow = h_aoff = nullptr;
    streamed = false;
  }
  // ---- hybrid execution (see count_hybrid_impl): host copies of the
  // count-phase tables and the plan-order work items, made on first use
  struct HybridHost {
    bool ready = false;
    std::vector<uint32_t> orow, bot, aoff;
    std::vector<int32_t> ocol, acol, icolb;
    std::vector<uint64_t> botp, acp;
    std::vector<int64_t> istart;  // plan-order item index of each task, |T|+1
    HostTables t{};
  } hy;
  bool plan_order_items = false;  // `items` holds the plan-order layout
  // captured persistent count, valid for the output pointers it was made with
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  uint64_t* g_per = nullptr;
  uint64_t* g_tot = nullptr;
  // outputs of the last direct launch since the graph was dropped: a graph is
  // captured only once the same outputs are counted into a second time
  uint64_t* d_per = nullptr;
  uint64_t* d_tot = nullptr;
  bbtc_stats stats{};

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    g_per = g_tot = nullptr;
    d_per = d_tot = nullptr;
  }

  ~bbtc_plan() {
    drop_graph();
    drop_stream();
    for (int q = 0; q < 4; ++q) {
      if (side[q]) (void)hipStreamDestroy(side[q]);
      if (ev_join[q]) (void)hipEventDestroy(ev_join[q]);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_cuts) (void)hipEventDestroy(ev_cuts);
    in_rowptr.release(); in_col.release(); keys_a.release(); keys_b.release(); hist.release(); partial.release();
    perm.release(); order.release(); ocol.release(); icol.release(); cuts.release(); blk.release();
    acol.release(); od.release(); idg.release(); orow.release(); irow.release(); midrows.release();
    longrows.release();
    hugerows.release();
    bot.release(); ccnt.release(); ccoff.release(); cursor.release(); aoff.release(); asrc.release(); icolb.release();
    ocol16.release(); rc.release();
    err.release(); acp.release(); tasks.release(); items.release(); xitems.release(); heavy.release();
    emit.release(); grp.release(); dslot.release(); dbits.release(); dcount.release();
  }

  size_t footprint() const {
    return in_rowptr.bytes() + in_col.bytes() + keys_a.bytes() + keys_b.bytes() + hist.bytes() + partial.bytes() +
           perm.bytes() + order.bytes() + ocol.bytes() + icol.bytes() + cuts.bytes() + blk.bytes() +
           acol.bytes() + od.bytes() + idg.bytes() + orow.bytes() + irow.bytes() + midrows.bytes() + longrows.bytes() +
           hugerows.bytes() + bot.bytes() +
           ccnt.bytes() + ccoff.bytes() + cursor.bytes() + err.bytes() + acp.bytes() + aoff.bytes() + asrc.bytes() +
           icolb.bytes() + ocol16.bytes() + rc.bytes() +
           tasks.bytes() + items.bytes() + xitems.bytes() + heavy.bytes() + emit.bytes() + grp.bytes() +
           dslot.bytes() + dbits.bytes() + dcount.bytes() +
           cache.bytes();
  }
};

namespace {

// ------------------------------------------------------------ host validation
// rows == false: only rowptr (O(n)); the entries are then checked by the
// device validation kernels after the upload.
template <typename RP>
bbtc_status validate_host(const RP* rowptr, const int32_t* col, int64_t n, int64_t nnz, bool symmetric,
                          bool rows = true) {
  if ((int64_t)rowptr[0] != 0) return fail(BBTC_EINVAL, "rowptr[0] must be 0");
  if ((int64_t)rowptr[n] != nnz) return fail(BBTC_EINVAL, "rowptr[n] must equal nnz");
  for (int64_t x = 0; x < n; ++x)
    if ((int64_t)rowptr[x + 1] < (int64_t)rowptr[x]) return fail(BBTC_EINVAL, "rowptr must be non-decreasing");
  if (!rows) return BBTC_OK;
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 100000) nt = 1;
  std::vector<uint32_t> bad(nt, 0);
  auto work = [&](unsigned t) {
    uint32_t e = 0;
    for (int64_t x = (int64_t)t; x < n; x += nt) {
      const int64_t b = rowptr[x], en = rowptr[x + 1];
      for (int64_t q = b; q < en; ++q) {
        const int32_t y = col[q];
        if (y < 0 || y >= n) { e |= 1; continue; }
        if (y == x) e |= 4;
        if (q > b && col[q - 1] >= y) e |= 2;
        if (symmetric) {
          const int32_t* rb = col + (int64_t)rowptr[y];
          const int32_t* re = col + (int64_t)rowptr[y + 1];
          const int32_t* it = std::lower_bound(rb, re, (int32_t)x);
          if (it == re || *it != (int32_t)x) e |= 16;
        }
      }
    }
    bad[t] = e;
  };
  if (nt == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) th.emplace_back(work, t);
    for (auto& t : th) t.join();
  }
  uint32_t e = 0;
  for (auto v : bad) e |= v;
  if (e & 1) return fail(BBTC_EINVAL, "column index out of range");
  if (e & 2) return fail(BBTC_EINVAL, "rows must be strictly increasing (sorted, no duplicates)");
  if (e & 4) return fail(BBTC_EINVAL, "self-loop in input");
  if (e & 16) return fail(BBTC_EINVAL, "input is not symmetric");
  return BBTC_OK;
}

bbtc_status decode_device_err(uint32_t e) {
  if (e & 8) return fail(BBTC_EINVAL, "rowptr malformed (not 0..nnz, or decreasing)");
  if (e & 1) return fail(BBTC_EINVAL, "column index out of range");
  if (e & 2) return fail(BBTC_EINVAL, "rows must be strictly increasing (sorted, no duplicates)");
  if (e & 4) return fail(BBTC_EINVAL, "self-loop in input");
  if (e & 16) return fail(BBTC_EINVAL, "input is not symmetric");
  return BBTC_OK;
}

bool is_device_pointer(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

void fill_defaults(bbtc_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->mode = BBTC_MODE_PERSISTENT;
  o->cut_mode = BBTC_CUT_BALANCED;
}

constexpr int kDefaultWaveMin = 32;
constexpr int kDefaultHashMin = 16;
constexpr int kDefaultItemRows = 256;
constexpr uint32_t kHubSplit = 256;   // in-slice length above which a column is split
constexpr unsigned kHybridMaxThreads = 16;  // default host threads of the hybrid count, at most
constexpr double kTuneMargin = 0.97;        // the autotuner's thresholds change for a gain above 3% only
constexpr uint32_t kHubChunk = 1024;  // in-neighbours per hub work item
constexpr int kItemsPerBlock = 20;    // work items per resident workgroup (by estimated work)
constexpr int64_t kGroupRowCap = 1 << 17;      // long/huge in-rows grouped in chunks, at most
// Below this many edges a graph's hubs are small enough for one workgroup
// per row, and the chunked grouping and the dense bitmaps cost more (fixed
// launches, in many concurrent partitions when serving) than they save.
constexpr uint64_t kLargeGraphEdges = 1ull << 22;
constexpr uint64_t kGroupCounters = 1u << 22;  // their per-part counters, at most (words)

// The plain HMap mode is the paper's per-task HMap throughout: every live
// column stages its list alone as a bitmap or hash (no shared sorted stage).
int eff_wave_min(const bbtc_options& o) {
  if (o.mode == BBTC_MODE_PLAIN_HMAP) return 1;
  return o.wave_min > 0 ? o.wave_min : kDefaultWaveMin;
}
// Rows of undirected degree at most the threshold keep no stored block
// boundaries.  Automatic (bound_min_deg 0): the smallest of kAutoBound whose
// stored boundaries take at most the 4m bytes of the out-rows (a probe of a
// row with stored boundaries reads one cache line of them; a short row
// without them is scanned, which reads its row pointers and the row), else
// the largest.
constexpr int kAutoBound[4] = {0, 8, 16, 32};
DegThresholds bound_thresholds(const bbtc_options& o) {
  DegThresholds th;
  for (int q = 0; q < 4; ++q) th.t[q] = o.bound_min_deg == 0 ? kAutoBound[q] : (int64_t)o.bound_min_deg;
  return th;
}
// Bytes of stored boundaries when ranks from rT on store them.
uint64_t bound_bytes(const std::vector<int32_t>& cuts, int32_t p, int64_t rT) {
  uint64_t b = 0;
  for (int32_t a = 0; a < p; ++a) {
    const int64_t sa = std::max<int64_t>(0, cuts[a + 1] - std::max<int64_t>(cuts[a], rT));
    b += 4ull * (uint64_t)(p - a + 1) * (uint64_t)sa;
  }
  return b;
}
// The first rank with stored boundaries, from the four counts of
// k_degree_stats and the cut vector.  Plans built within a device budget
// stream their out-stripes with the boundaries, so there the automatic
// threshold stays at the largest candidate.
int64_t choose_rT(const bbtc_options& o, const uint32_t cnt[4], const std::vector<int32_t>& cuts, int32_t p,
                  uint64_t m, bool budgeted) {
  if (o.bound_min_deg != 0) return cnt[0];
  if (budgeted) return cnt[3];
  for (int q = 0; q < 4; ++q)
    if (bound_bytes(cuts, p, cnt[q]) <= 4 * m) return cnt[q];
  return cnt[3];
}

int eff_hash_min(const bbtc_options& o) {
  if (o.mode == BBTC_MODE_PLAIN_INTERSECT) return -1;
  if (o.mode == BBTC_MODE_PLAIN_HMAP) return 1;
  if (o.hash_min < 0) return -1;
  return o.hash_min > 0 ? o.hash_min : kDefaultHashMin;
}

PlanCtx plan_ctx(const bbtc_plan* pl, uint64_t* per_task, uint64_t* total) {
  PlanCtx c;
  c.g.p = pl->p;
  c.g.m = (uint32_t)pl->m;
  c.g.gi = c.g.gj = -1;
  c.g.rT = (int32_t)pl->rT;
  c.g.pad = 0;
  c.g.orow = pl->orow.ptr;
  c.g.colI = c.g.colJ = c.g.icolJ = nullptr;
  c.g.acolJ = nullptr;
  c.g.aoffJ = nullptr;
  c.g.botI = c.g.botJ = nullptr;
  c.g.cuts = pl->cuts.ptr;
  c.g.botp = pl->botp;
  c.g.bot = pl->bot.ptr;
  c.g.ocol = pl->ocol.ptr;
  c.g.ocol16 = pl->streamed ? nullptr : pl->ocol16.ptr;
  const bool dense = !pl->streamed && pl->ocol16.ptr != nullptr && pl->dense_k0 < pl->p && pl->dslot.ptr != nullptr;
  c.g.dense_k0 = dense ? pl->dense_k0 : pl->p;
  c.g.dense_u0 = dense ? pl->h_cuts[pl->dense_k0] : 0;
  c.g.dslot = dense ? pl->dslot.ptr : nullptr;
  c.g.dbits = dense ? pl->dbits.ptr : nullptr;
  c.g.acp = pl->acp.ptr;
  c.g.acol = pl->acol.ptr;
  c.g.aoff = pl->aoff.ptr;
  c.g.icol = pl->icolb.ptr;
  c.tasks = pl->tasks.ptr;
  c.ntasks = (int64_t)pl->h_tasks.size();
  c.items = pl->opt.mode == BBTC_MODE_PERSISTENT && !pl->streamed ? pl->xitems.ptr : pl->items.ptr;
  c.per_task = per_task;
  c.total = total;
  c.wave_min = eff_wave_min(pl->opt);
  c.hash_min = eff_hash_min(pl->opt);
  c.split = pl->split;
  c.pad = 0;
  return c;
}

// ------------------------------------------------------------ task list
// Alg. 4 order, the Sec. 5 estimate, kinds, and the non-increasing order by
// estimate (ties kept in Alg. 4 order); the number of work items per task.
void compose_tasks(bbtc_plan* pl) {
  const int64_t p = pl->p;
  std::vector<bbtc_task> all;
  all.reserve((size_t)(p * (p + 1) * (p + 2) / 6));
  for (int32_t i = 0; i < p; ++i)
    for (int32_t j = i; j < p; ++j)
      for (int32_t k = j; k < p; ++k) {
        bbtc_task t;
        t.i = i; t.j = j; t.k = k;
        const int64_t nij = pl->h_nnz[block_id(p, i, j)], nik = pl->h_nnz[block_id(p, i, k)],
                      njk = pl->h_nnz[block_id(p, j, k)];
        const double vi = (double)(pl->h_cuts[i + 1] - pl->h_cuts[i]);
        const double vj = (double)(pl->h_cuts[j + 1] - pl->h_cuts[j]);
        t.kind = (nij > 0 && nik > 0 && njk > 0) ? BBTC_TASK_WORK : BBTC_TASK_EMPTY;
        t.est = (double)nij * std::max((double)nik / vi, (double)njk / vj);
        if (t.kind == BBTC_TASK_EMPTY) t.est = 0.0;
        all.push_back(t);
      }
  std::vector<int64_t> idx(all.size());
  for (size_t q = 0; q < idx.size(); ++q) idx[q] = (int64_t)q;
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return all[a].est > all[b].est; });
  pl->h_tasks.resize(all.size());
  pl->h_dtasks.resize(all.size());
  pl->h_work.clear();
  pl->h_items.clear();
  pl->h_hub_first.clear();
  pl->h_hub_count.clear();
  for (size_t q = 0; q < idx.size(); ++q) {
    const bbtc_task& t = all[idx[q]];
    pl->h_tasks[q] = t;
    pl->h_dtasks[q] = DevTask{t.i, t.j, t.k, (int32_t)q};
    if (t.kind == BBTC_TASK_WORK) pl->h_work.push_back((int32_t)q);
  }
  // hub columns of each block
  const int64_t nb = p * (p + 1) / 2;
  pl->h_hstart.assign((size_t)nb + 1, 0);
  for (const HeavyCol& hc : pl->h_heavy) pl->h_hstart[hc.cid + 1]++;
  for (int64_t b = 0; b < nb; ++b) pl->h_hstart[b + 1] += pl->h_hstart[b];
  {  // group the hub records by block (counting sort; their order inside a block is free)
    std::vector<HeavyCol> g(pl->h_heavy.size());
    std::vector<int64_t> at(pl->h_hstart.begin(), pl->h_hstart.end() - 1);
    for (const HeavyCol& hc : pl->h_heavy) g[(size_t)at[hc.cid]++] = hc;
    pl->h_heavy.swap(g);
  }
  // Work items per task (emitted later, in the layout the launch needs): the
  // task's hub chunks, then its active columns in ranges sized by the task's
  // estimated work per column so that dense tasks spread over many
  // workgroups (at most item_rows columns per range).
  const uint32_t step = (uint32_t)(pl->opt.item_rows > 0 ? pl->opt.item_rows : kDefaultItemRows);
  double est_sum = 0;
  for (int32_t q : pl->h_work) est_sum += pl->h_tasks[q].est;
  pl->est_sum = est_sum;
  const double target = est_sum / (double)std::max<int64_t>(1, (int64_t)pl->blocks_per_cu * pl->ncu * kItemsPerBlock);
  pl->h_nitem.assign(all.size(), 0);
  pl->h_nper.assign(all.size(), 0);
  pl->h_nhub.assign(all.size(), 0);
  pl->nitems = 0;
  for (int32_t q : pl->h_work) {
    const bbtc_task& t = pl->h_tasks[q];
    const int64_t cid = col_block_id(t.i, t.j);
    uint32_t c = 0;
    for (int64_t r = pl->h_hstart[cid]; r < pl->h_hstart[cid + 1]; ++r)
      c += (pl->h_heavy[r].cnt + kHubChunk - 1) / kHubChunk;
    pl->h_nhub[q] = c;
    const uint32_t cols = (uint32_t)pl->h_nzc[cid];
    const double per_col = cols ? t.est / (double)cols : 0.0;
    uint32_t nper = step;
    if (per_col > 0 && target > 0) nper = (uint32_t)std::max(1.0, std::min((double)step, target / per_col));
    c += (cols + nper - 1) / nper;
    pl->h_nitem[q] = c;
    pl->h_nper[q] = nper;
    pl->nitems += c;
  }
}

// Writes the work items of plan-order task q to out (h_nitem[q] of them).
void emit_items(const bbtc_plan* pl, int32_t q, DevItem* out) {
  const bbtc_task& t = pl->h_tasks[q];
  const int64_t cid = col_block_id(t.i, t.j);
  size_t at = 0;
  for (int64_t r = pl->h_hstart[cid]; r < pl->h_hstart[cid + 1]; ++r) {
    const HeavyCol& hc = pl->h_heavy[r];
    for (uint32_t lo = 0; lo < hc.cnt; lo += kHubChunk)
      out[at++] = DevItem{q, lo, std::min(hc.cnt, lo + kHubChunk), (int32_t)hc.x};
  }
  const uint32_t cols = (uint32_t)pl->h_nzc[cid], nper = pl->h_nper[q];
  for (uint32_t lo = 0; lo < cols; lo += nper) out[at++] = DevItem{q, lo, std::min(cols, lo + nper), -1};
}

// The items in plan order, each task's contiguous (the plain launches and the
// streamed walk use this layout).
void compose_plan_order(bbtc_plan* pl) {
  pl->h_items.resize(pl->nitems);
  pl->plan_order_items = false;  // set once they are uploaded to `items`
  pl->h_hub_first.assign(pl->h_tasks.size(), 0);
  pl->h_hub_count.assign(pl->h_tasks.size(), 0);
  size_t at = 0;
  for (int32_t q : pl->h_work) {
    pl->h_hub_first[q] = (int64_t)at;
    pl->h_hub_count[q] = pl->h_nitem[q];
    emit_items(pl, q, pl->h_items.data() + at);
    at += pl->h_nitem[q];
  }
}

// The persistent launch walks the same work items as kMaxQueues queues, one
// per XCD (each XCD has its own L2).  The probes of task (i,j,k) gather rows
// of G_ik, so the tasks sharing (i,k) stay on one XCD and run back to back
// there: groups go, heaviest first, to the least loaded queue.  A task heavier
// than half a queue's fair share has its items dealt over all queues instead.
// Workgroups drain their own XCD's queue and then help the others, so the
// split changes only locality, never what is counted.
bbtc_status compose_queues(bbtc_plan* pl) {
  const int X = kMaxQueues;
  const int64_t p = pl->p;
  double total = 0;
  for (int32_t q : pl->h_work) total += pl->h_tasks[q].est;
  const double fair = total / X;
  std::vector<double> load(X, 0.0);
  auto least = [&]() { return (int)(std::min_element(load.begin(), load.end()) - load.begin()); };
  std::vector<size_t> wide_cnt(X, 0), group_cnt(X, 0);
  std::vector<int32_t> wide;  // tasks dealt over all queues, plan order
  std::vector<std::array<uint32_t, kMaxQueues>> wshare;  // their items per queue
  std::vector<int64_t> gfirst((size_t)(p * (p + 1) / 2), -1), gnext(pl->h_tasks.size(), -1);
  std::vector<int64_t> glast(gfirst.size(), -1);
  std::vector<double> gload(gfirst.size(), 0.0);
  std::vector<size_t> gitems(gfirst.size(), 0);
  for (int32_t q : pl->h_work) {  // plan order: heaviest first
    const bbtc_task& t = pl->h_tasks[q];
    const uint32_t c = pl->h_nitem[q];
    if (t.est > fair / 2 && c > 1) {
      // the items in about 64 equal pieces, each to the least loaded queue
      wide.push_back(q);
      const double w = t.est / (double)c;
      const uint32_t piece = std::max<uint32_t>(1, c / 64);
      std::array<uint32_t, kMaxQueues> sh{};
      for (uint32_t r = 0; r < c; r += piece) {
        const uint32_t k = std::min(piece, c - r);
        const int x = least();
        sh[x] += k;
        wide_cnt[x] += k;
        load[x] += w * k;
      }
      wshare.push_back(sh);
    } else {  // chain the task into its (i,k) group, keeping plan order
      const int64_t g = block_id(p, t.i, t.k);
      if (gfirst[g] < 0) gfirst[g] = q; else gnext[glast[g]] = q;
      glast[g] = q;
      gload[g] += t.est;
      gitems[g] += c;
    }
  }
  std::vector<int64_t> gs;
  for (size_t g = 0; g < gfirst.size(); ++g)
    if (gfirst[g] >= 0) gs.push_back((int64_t)g);
  std::stable_sort(gs.begin(), gs.end(), [&](int64_t a, int64_t b) { return gload[a] > gload[b]; });
  std::vector<int> gq(gfirst.size(), 0);
  for (int64_t g : gs) {
    const int x = least();
    gq[g] = x;
    group_cnt[x] += gitems[g];
    load[x] += gload[g];
  }
  // queue x: its share of the wide tasks' items, then its groups in order
  std::vector<size_t> at(2 * X, 0);
  size_t pos = 0;
  pl->nq = X;
  for (int x = 0; x < X; ++x) {
    pl->qbeg[x] = (uint32_t)pos;
    at[x] = pos;
    pos += wide_cnt[x];
    at[x + X] = pos;
    pos += group_cnt[x];
    pl->qlen[x] = (uint32_t)(pos - pl->qbeg[x]);
  }
  // The queues as runs of task items, queue by queue (so the runs come in
  // position order); a wide task's share of a queue is one contiguous piece.
  std::vector<std::vector<ItemRun>> qr(X);
  for (size_t h = 0; h < wide.size(); ++h) {
    const int32_t q = wide[h];
    uint32_t r0 = 0;
    for (int x = 0; x < X; ++x)
      if (wshare[h][x]) {
        qr[x].push_back(ItemRun{q, r0, wshare[h][x], (uint32_t)at[x]});
        at[x] += wshare[h][x];
        r0 += wshare[h][x];
      }
  }
  for (int64_t g : gs)
    for (int64_t q = gfirst[g]; q >= 0; q = gnext[q]) {
      const int x = gq[g];
      if (pl->h_nitem[q] == 0) continue;
      qr[x].push_back(ItemRun{(int32_t)q, 0, pl->h_nitem[q], (uint32_t)at[x + X]});
      at[x + X] += pl->h_nitem[q];
    }
  pl->h_runs.clear();
  for (int x = 0; x < X; ++x) pl->h_runs.insert(pl->h_runs.end(), qr[x].begin(), qr[x].end());
  return BBTC_OK;
}

// A launch over items[0, nitems) as a single queue.
void one_queue(CountParams& cp) {
  cp.nq = 1;
  for (int x = 0; x < kMaxQueues; ++x) cp.qbeg[x] = cp.qlen[x] = 0;
  cp.qlen[0] = cp.nitems;
}

// ------------------------------------------------------------ streaming
// The tasks of block pair (i,j) read the out-rows of V_i and V_j with their
// stored block boundaries (two out-stripes) and the in side of block (i,j)
// (its active columns, in-slice offsets and in-slices), nothing else.  When
// the plan exceeds the device budget these arrays live in pinned host
// memory; the device keeps a cache of out-stripe slots (the stripe needed
// farthest ahead goes) and two in-block slots, and bbtc_count walks the block pairs in
// column chunks that the cache holds (stream_finish), uploading on a side
// stream gated by events, ahead of the kernels.
template <typename T>
bbtc_status to_pinned(T** dst, const T* src, size_t n, hipStream_t s) {
  HIP_TRY(hipHostMalloc((void**)dst, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault), "pinned alloc");
  if (n) HIP_TRY(hipMemcpyAsync(*dst, src, n * sizeof(T), hipMemcpyDeviceToHost, s), "D2H");
  return BBTC_OK;
}

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// An out-stripe starts (ocut & 3) words into its slot, so that positions that
// are multiples of 4 in the whole oriented CSR stay 16-byte aligned (the
// counting kernels read out-rows in aligned 16-byte blocks); its rows are
// padded to a multiple of 16 bytes, then come the part's stored boundaries.
size_t out_head(const bbtc_plan* pl, int a) { return (size_t)(pl->ocut[a] & 3); }

size_t stripe_bytes(const bbtc_plan* pl, int a) {
  return align16(4 * (out_head(pl, a) + pl->ocut[a + 1] - pl->ocut[a])) + 4 * (pl->h_botp[a + 1] - pl->h_botp[a]);
}

// In-block slot of block cid: active columns | in-slice offsets (one more) |
// in-slices, each padded to 16 bytes.
struct BlockSpan {
  uint64_t x0, nx, e0, ne;  // active columns [x0, x0+nx), entries [e0, e0+ne)
  size_t o_aoff, o_icol, bytes;
};
BlockSpan block_span(const bbtc_plan* pl, int64_t cid) {
  BlockSpan b;
  b.x0 = pl->h_acp[cid];
  b.nx = pl->h_acp[cid + 1] - b.x0;
  b.e0 = pl->h_aoff[b.x0];
  b.ne = pl->h_aoff[b.x0 + b.nx] - b.e0;
  b.o_aoff = align16(4 * b.nx);
  b.o_icol = b.o_aoff + align16(4 * (b.nx + 1));
  b.bytes = b.o_icol + align16(4 * b.ne);
  return b;
}

// Sizes the slots within the budget, then groups the plan-order work items
// by block pair in the walk order.  The walk takes the columns j in chunks
// of S = slots - 1 parts: a chunk's out-stripes stay cached while i runs over
// every part up to the chunk's end (one more slot holds the stripe of an i
// outside the chunk), so each stripe is uploaded about once per chunk to its
// right plus once for its own chunk, instead of once per row pass.  Needs
// the pinned arrays in place.
bbtc_status stream_finish(bbtc_plan* pl, hipStream_t s) {
  const int32_t p = pl->p;
  const int64_t nb = (int64_t)p * (p + 1) / 2;
  pl->h_acp.assign((size_t)nb + 1, 0);
  for (int64_t b = 0; b < nb; ++b) pl->h_acp[b + 1] = pl->h_acp[b] + (uint64_t)pl->h_nzc[b];
  pl->heavy.release();  // the hub records were read back by the partition
  if (pl->h_items.size() != pl->nitems) compose_plan_order(pl);
  // slot sizes: the largest out-stripe, the largest in-block of a pair with work
  size_t slot = 16, blk = 16;
  for (int a = 0; a < p; ++a) slot = std::max(slot, stripe_bytes(pl, a));
  for (int32_t q : pl->h_work) {
    const bbtc_task& t = pl->h_tasks[q];
    blk = std::max(blk, block_span(pl, col_block_id(t.i, t.j)).bytes);
  }
  pl->slot_bytes = align16(slot);
  pl->block_bytes = align16(blk);
  pl->xitems.release();  // streamed launches walk the plan order, pair by pair
  {  // every stripe and block resident
    int64_t all = (int64_t)pl->footprint();
    for (int a = 0; a < p; ++a) all += (int64_t)stripe_bytes(pl, a);
    for (int64_t c = 0; c < nb; ++c) all += (int64_t)block_span(pl, c).bytes;
    pl->resident_bytes = all;
  }
  // the cache takes what the budget leaves: two block slots, then out-stripes
  // (with the item list as it will be once uploaded below)
  const size_t items_after = pl->items.ptr && pl->items.cap >= pl->nitems
                                 ? pl->items.bytes()
                                 : sizeof(DevItem) * std::max<size_t>(pl->nitems, 1);
  const int64_t fixed = (int64_t)(pl->footprint() - pl->items.bytes() + items_after);
  const int64_t room = pl->opt.device_budget_bytes - fixed - 2 * (int64_t)pl->block_bytes;
  const int64_t nslots = room > 0 ? room / (int64_t)pl->slot_bytes : 0;
  if (nslots < 2)
    return fail(BBTC_EBUDGET, "device budget holds " + std::to_string(nslots) + " out-stripe slots of " +
                                  std::to_string(pl->slot_bytes) + " B besides two block slots of " +
                                  std::to_string(pl->block_bytes) + " B and " + std::to_string(fixed) +
                                  " B of resident data; a block pair needs 2");
  const int64_t use = std::min<int64_t>(nslots, p);
  const int64_t chunk = std::max<int64_t>(1, use - 1);
  std::vector<DevItem> items = pl->h_items;
  // walk order: column chunk, then i ascending, then j ascending
  auto walk_key = [&](const DevItem& it) {
    const bbtc_task& t = pl->h_tasks[it.task];
    return ((int64_t)(t.j / chunk) * p + t.i) * p + t.j;
  };
  std::stable_sort(items.begin(), items.end(),
                   [&](const DevItem& x, const DevItem& y) { return walk_key(x) < walk_key(y); });
  pl->groups.clear();
  pl->group_first.clear();
  pl->group_count.clear();
  int64_t last = -1;
  for (size_t q = 0; q < items.size(); ++q) {
    const int64_t key = walk_key(items[q]);
    if (key != last) {
      const bbtc_task& t = pl->h_tasks[items[q].task];
      pl->groups.push_back({t.i, t.j});
      pl->group_first.push_back((int64_t)q);
      pl->group_count.push_back(0);
      last = key;
    }
    pl->group_count.back()++;
  }
  pl->stripe_uses.assign((size_t)p, {});
  for (size_t g = 0; g < pl->groups.size(); ++g) {
    pl->stripe_uses[(size_t)pl->groups[g].first].push_back((int64_t)g);
    if (pl->groups[g].second != pl->groups[g].first) pl->stripe_uses[(size_t)pl->groups[g].second].push_back((int64_t)g);
  }
  pl->h_items = items;
  HIP_TRY(pl->items.ensure(items.size()), "alloc items");
  if (!items.empty())
    HIP_TRY(hipMemcpyAsync(pl->items.ptr, items.data(), sizeof(DevItem) * items.size(), hipMemcpyHostToDevice, s),
            "H2D");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  HIP_TRY(pl->cache.ensure((size_t)use * pl->slot_bytes + 2 * pl->block_bytes), "alloc stripe cache");
  pl->slots.assign((size_t)use, bbtc_plan::Slot());
  for (auto& sl : pl->slots) {
    HIP_TRY(hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming), "event");
    HIP_TRY(hipEventCreateWithFlags(&sl.released, hipEventDisableTiming), "event");
  }
  for (auto& sl : pl->bslot) {
    HIP_TRY(hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming), "event");
    HIP_TRY(hipEventCreateWithFlags(&sl.released, hipEventDisableTiming), "event");
  }
  pl->streamed = true;
  return BBTC_OK;
}

// A resident build over the budget: the count-phase arrays move to pinned
// host memory and every device array the count does not read is released.
bbtc_status stream_setup(bbtc_plan* pl, hipStream_t s) {
  const int32_t p = pl->p;
  const int64_t n = pl->n, nb = (int64_t)p * (p + 1) / 2;
  std::vector<uint32_t> oro(n + 1);
  HIP_TRY(hipMemcpyAsync(oro.data(), pl->orow.ptr, 4 * (n + 1), hipMemcpyDeviceToHost, s), "D2H");
  pl->h_botp.assign(p + 1, 0);
  HIP_TRY(hipMemcpyAsync(pl->h_botp.data(), pl->botp, 8 * (p + 1), hipMemcpyDeviceToHost, s), "D2H");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  pl->ocut.assign(p + 1, 0);
  for (int32_t a = 0; a <= p; ++a) pl->ocut[a] = oro[pl->h_cuts[a]];
  size_t ncols = 0;
  for (int64_t b = 0; b < nb; ++b) ncols += (size_t)pl->h_nzc[b];
  bbtc_status st;
  if ((st = to_pinned(&pl->h_ocol, pl->ocol.ptr, (size_t)pl->m, s)) != BBTC_OK) return st;
  if ((st = to_pinned(&pl->h_bot, pl->bot.ptr, (size_t)pl->h_botp[p], s)) != BBTC_OK) return st;
  if ((st = to_pinned(&pl->h_orow, pl->orow.ptr, (size_t)n + 1, s)) != BBTC_OK) return st;
  if ((st = to_pinned(&pl->h_acol, pl->acol.ptr, ncols, s)) != BBTC_OK) return st;
  if ((st = to_pinned(&pl->h_aoff, pl->aoff.ptr, ncols + 1, s)) != BBTC_OK) return st;
  if ((st = to_pinned(&pl->h_icolb, pl->icolb.ptr, (size_t)pl->m, s)) != BBTC_OK) return st;
  HIP_TRY(hipStreamSynchronize(s), "sync");
  // release everything the count phase does not read (the out-row pointers
  // stay: the slices of rows without stored boundaries are found by scanning)
  pl->ocol.release(); pl->icol.release(); pl->bot.release(); pl->acol.release(); pl->aoff.release();
  pl->asrc.release(); pl->icolb.release(); pl->irow.release(); pl->ocol16.release(); pl->rc.release();
  pl->keys_a.release(); pl->keys_b.release(); pl->hist.release(); pl->partial.release();
  pl->od.release(); pl->idg.release(); pl->order.release();
  pl->longrows.release(); pl->hugerows.release(); pl->midrows.release(); pl->ccnt.release(); pl->ccoff.release();
  pl->in_rowptr.release(); pl->in_col.release(); pl->heavy.release(); pl->emit.release(); pl->grp.release();
  pl->dslot.release(); pl->dbits.release(); pl->dcount.release();
  pl->dense_k0 = pl->p;
  return stream_finish(pl, s);
}

// Enqueues on `cs` the upload of `bytes` host bytes into a slot once the
// kernels that read the slot's previous contents are done.
hipError_t upload_after(bbtc_plan::Slot& sl, hipStream_t cs) {
  return sl.used ? hipStreamWaitEvent(cs, sl.released, 0) : hipSuccess;
}

// Returns the slot holding out-stripe a for the pair at walk position g,
// uploading it (on `cs`) if needed, never evicting a slot listed in `keep`.
// The victim is the stripe whose next use in the walk is farthest away (the
// whole walk is known in advance), ties broken by least recent use.  -1 if
// every slot is kept.
int stripe_slot(bbtc_plan* pl, int a, int64_t g, const std::vector<int>& keep, hipStream_t cs, bbtc_status* st) {
  *st = BBTC_OK;
  int victim = -1;
  for (size_t q = 0; q < pl->slots.size(); ++q)
    if (pl->slots[q].key == a) {
      pl->slots[q].last = ++pl->clock;
      return (int)q;
    }
  auto next_use = [&](int key) -> int64_t {
    if (key < 0) return INT64_MAX;  // empty slot
    const std::vector<int64_t>& u = pl->stripe_uses[(size_t)key];
    const auto it = std::lower_bound(u.begin(), u.end(), g);
    return it == u.end() ? INT64_MAX : *it;
  };
  int64_t far = -1;
  for (size_t q = 0; q < pl->slots.size(); ++q) {
    if (std::find(keep.begin(), keep.end(), (int)q) != keep.end()) continue;
    const int64_t nu = next_use(pl->slots[q].key);
    if (victim < 0 || nu > far || (nu == far && pl->slots[q].last < pl->slots[victim].last)) {
      victim = (int)q;
      far = nu;
    }
  }
  if (victim < 0) return -1;
  bbtc_plan::Slot& sl = pl->slots[victim];
  hipError_t e = upload_after(sl, cs);
  char* base = pl->cache.ptr + (size_t)victim * pl->slot_bytes;
  const size_t nc = pl->ocut[a + 1] - pl->ocut[a], nb = pl->h_botp[a + 1] - pl->h_botp[a];
  const size_t hd = out_head(pl, a);
  if (e == hipSuccess && nc)
    e = hipMemcpyAsync(base + 4 * hd, pl->h_ocol + pl->ocut[a], 4 * nc, hipMemcpyHostToDevice, cs);
  if (e == hipSuccess && nb)
    e = hipMemcpyAsync(base + align16(4 * (hd + nc)), pl->h_bot + pl->h_botp[a], 4 * nb, hipMemcpyHostToDevice, cs);
  if (e == hipSuccess) e = hipEventRecord(sl.ready, cs);
  if (e != hipSuccess) {
    *st = hip_fail(e, "stripe upload");
    return -1;
  }
  sl.key = a;
  sl.last = ++pl->clock;
  pl->copies++;
  return victim;
}

// Uploads block cid's in side into block slot r (on `cs`).
bbtc_status block_upload(bbtc_plan* pl, int r, int64_t cid, hipStream_t cs) {
  bbtc_plan::Slot& sl = pl->bslot[r];
  const BlockSpan b = block_span(pl, cid);
  char* base = pl->cache.ptr + pl->slots.size() * pl->slot_bytes + (size_t)r * pl->block_bytes;
  HIP_TRY(upload_after(sl, cs), "wait");
  if (b.nx) {
    HIP_TRY(hipMemcpyAsync(base, pl->h_acol + b.x0, 4 * b.nx, hipMemcpyHostToDevice, cs), "block upload");
    HIP_TRY(hipMemcpyAsync(base + b.o_aoff, pl->h_aoff + b.x0, 4 * (b.nx + 1), hipMemcpyHostToDevice, cs),
            "block upload");
  }
  if (b.ne) HIP_TRY(hipMemcpyAsync(base + b.o_icol, pl->h_icolb + b.e0, 4 * b.ne, hipMemcpyHostToDevice, cs), "block upload");
  HIP_TRY(hipEventRecord(sl.ready, cs), "event");
  sl.key = (int)cid;
  pl->copies++;
  return BBTC_OK;
}

bbtc_status count_streamed(bbtc_plan* pl, hipStream_t s, uint64_t* d_per_task, uint64_t* d_total) {
  const int64_t nt = (int64_t)pl->h_tasks.size();
  HIP_TRY(launch_reset(d_per_task, nt, d_total, pl->cursor.ptr, s), "reset");
  hipStream_t cs = pl->side[1];
  pl->copies = 0;
  // uploads start after the reset (and anything earlier on s) is enqueued
  HIP_TRY(hipEventRecord(pl->ev_fork, s), "event");
  HIP_TRY(hipStreamWaitEvent(cs, pl->ev_fork, 0), "wait");
  const int grid_max = pl->blocks_per_cu * pl->ncu;
  for (size_t g = 0; g < pl->groups.size(); ++g) {
    const int32_t i = pl->groups[g].first, j = pl->groups[g].second;
    const int64_t cid = col_block_id(i, j);
    std::vector<int> keep;
    int slot[2];
    const int need[2] = {i, j};
    bbtc_status st = BBTC_OK;
    for (int q = 0; q < 2; ++q) {
      slot[q] = stripe_slot(pl, need[q], (int64_t)g, keep, cs, &st);
      if (st != BBTC_OK) return st;
      if (slot[q] < 0) return fail(BBTC_EBUDGET, "stripe cache too small for one block pair");
      keep.push_back(slot[q]);
    }
    const int r = (int)(g & 1);
    if ((st = block_upload(pl, r, cid, cs)) != BBTC_OK) return st;
    for (int q = 0; q < 2; ++q) HIP_TRY(hipStreamWaitEvent(s, pl->slots[slot[q]].ready, 0), "wait");
    HIP_TRY(hipStreamWaitEvent(s, pl->bslot[r].ready, 0), "wait");
    CountParams cp;
    std::memset(&cp, 0, sizeof(cp));
    cp.one = plan_ctx(pl, d_per_task, d_total);
    cp.one.g.gi = i;
    cp.one.g.gj = j;
    auto base = [&](int q) { return pl->cache.ptr + (size_t)slot[q] * pl->slot_bytes; };
    const size_t nci = pl->ocut[i + 1] - pl->ocut[i], ncj = pl->ocut[j + 1] - pl->ocut[j];
    const size_t hi = out_head(pl, i), hj = out_head(pl, j);
    // shifted so that absolute positions and indices land in the slots
    cp.one.g.colI = (const int32_t*)base(0) + hi - pl->ocut[i];
    cp.one.g.botI = (const uint32_t*)(base(0) + align16(4 * (hi + nci)));
    cp.one.g.colJ = (const int32_t*)base(1) + hj - pl->ocut[j];
    cp.one.g.botJ = (const uint32_t*)(base(1) + align16(4 * (hj + ncj)));
    const BlockSpan b = block_span(pl, cid);
    const char* bb = pl->cache.ptr + pl->slots.size() * pl->slot_bytes + (size_t)r * pl->block_bytes;
    cp.one.g.acolJ = (const int32_t*)bb - b.x0;
    cp.one.g.aoffJ = (const uint32_t*)(bb + b.o_aoff) - b.x0;
    cp.one.g.icolJ = (const int32_t*)(bb + b.o_icol) - b.e0;
    cp.items = pl->items.ptr + pl->group_first[g];
    cp.nitems = (uint32_t)pl->group_count[g];
    cp.cursor = pl->cursor.ptr;
    one_queue(cp);
    HIP_TRY(launch_reset(nullptr, 0, nullptr, pl->cursor.ptr, s), "cursor");  // cursor only
    const int grid = (int)std::min<int64_t>(grid_max, (int64_t)cp.nitems);
    HIP_TRY(launch_count_persistent(cp, grid, false, s), "count");
    for (int q = 0; q < 2; ++q) {
      HIP_TRY(hipEventRecord(pl->slots[slot[q]].released, s), "event");
      pl->slots[slot[q]].used = true;
    }
    HIP_TRY(hipEventRecord(pl->bslot[r].released, s), "event");
    pl->bslot[r].used = true;
  }
  return BBTC_OK;
}

// Dense slices as bitmaps (resident plans with the 16-bit out-rows): the
// rows of the last parts, at most kDenseRows of them, against the blocks of
// those parts.  The bitmap words are bounded by half the entries of those
// blocks plus a segment's padding per slice (a dense slice has at least
// |V_k|/16 entries, i.e. at least two per word).
bbtc_status build_dense(bbtc_plan* pl, bool budgeted, hipStream_t s) {
  const int32_t p = pl->p;
  pl->dense_k0 = p;
  if (budgeted || pl->ocol16.ptr == nullptr || pl->opt.dense == -1) return BBTC_OK;
  if (pl->opt.dense == 0 && (uint64_t)pl->m < kLargeGraphEdges) return BBTC_OK;
  int32_t k0 = p;
  while (k0 > 0 && (int64_t)pl->h_cuts[p] - pl->h_cuts[k0 - 1] <= kDenseRows) --k0;
  if (k0 >= p) return BBTC_OK;
  const int64_t rows = (int64_t)pl->h_cuts[p] - pl->h_cuts[k0], nk = p - k0;
  uint64_t ent = 0;
  for (int32_t a = k0; a < p; ++a)
    for (int32_t k = a; k < p; ++k) ent += (uint64_t)pl->h_nnz[block_id(p, a, k)];
  const uint64_t cap = ent / 2 + 8 * (uint64_t)std::min<int64_t>(rows * nk, (int64_t)ent) + 8;
  HIP_TRY(ensure_pow2(pl->dslot, (size_t)(rows * nk)), "alloc dense slots");
  HIP_TRY(ensure_pow2(pl->dbits, (size_t)cap), "alloc dense bitmaps");
  HIP_TRY(pl->dcount.ensure(4), "alloc");
  HIP_TRY(hipMemsetAsync(pl->dcount.ptr, 0, 16, s), "memset");
  HIP_TRY(launch_dense_build(pl->orow.ptr, pl->ocol.ptr, pl->ocol16.ptr, pl->bot.ptr, pl->botp, pl->cuts.ptr, p,
                             (int32_t)pl->rT, k0, pl->n, rows * nk, pl->dslot.ptr, pl->dbits.ptr, pl->dcount.ptr, cap,
                             s),
          "dense slices");
  pl->dense_k0 = k0;
  return BBTC_OK;
}

// Block statistics and hub records from the device, the task list and work
// items (Alg. 4, Sec. 5's estimate), their upload and the plan statistics;
// then the streaming set-up of a plan over the device budget.  `budgeted`:
// the count-phase arrays are already in pinned host memory.
bbtc_status finish_partition(bbtc_plan* pl, hipStream_t s, uint64_t m, uint64_t wedges, uint64_t hcap, bool budgeted,
                             std::chrono::steady_clock::time_point t0) {
  const bbtc_options& opt = pl->opt;
  const int64_t n = pl->n;
  const int32_t p = pl->p;
  const int64_t nb = (int64_t)p * (p + 1) / 2;
  const size_t wb = sizeof(unsigned long long) * (size_t)nb;
  uint32_t hd[2] = {0, 0};
  uint32_t nheavy = 0;
  {  // block statistics through the pinned stage, one copy: [nheavy, dmax x2, -] then bnnz, bnzr, bnzc
    HIP_TRY(pl->stage.ensure(16 + 3 * wb), "pinned alloc");
    char* st = pl->stage.ptr;
    const uint32_t* sc = (const uint32_t*)st;
    const unsigned long long* sb = (const unsigned long long*)(st + 16);
    HIP_TRY(hipMemcpyAsync(st, pl->head, 16 + 3 * wb, hipMemcpyDeviceToHost, s), "D2H");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    nheavy = sc[0];
    hd[0] = sc[1];
    hd[1] = sc[2];
    pl->h_nnz.assign(sb, sb + nb);
    pl->h_nzr.assign(sb + nb, sb + 2 * nb);
    pl->h_nzc.assign(sb + 2 * nb, sb + 3 * nb);
  }
  if (nheavy > hcap) return fail(BBTC_EDEVICE, "hub column list overflow");
  {
    uint64_t ncols = 0;
    for (int64_t v : pl->h_nzc) ncols += (uint64_t)v;
    if (ncols >= (1ull << 31)) return fail(BBTC_EINVAL, "more than 2^31-1 active columns");
  }
  pl->h_heavy.resize(nheavy);
  if (nheavy) {
    HIP_TRY(pl->stage.ensure(sizeof(HeavyCol) * nheavy), "pinned alloc");
    HIP_TRY(hipMemcpyAsync(pl->stage.ptr, pl->heavy.ptr, sizeof(HeavyCol) * nheavy, hipMemcpyDeviceToHost, s), "D2H");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    std::memcpy(pl->h_heavy.data(), pl->stage.ptr, sizeof(HeavyCol) * nheavy);
  }

  // ---- tasks (Alg. 4) and work items ----
  std::vector<uint64_t> acp((size_t)nb + 1);
  acp[0] = 0;
  for (int64_t b = 0; b < nb; ++b) acp[b + 1] = acp[b] + (uint64_t)pl->h_nzc[b];
  compose_tasks(pl);
  {
    const bbtc_status dst = build_dense(pl, budgeted, s);
    if (dst != BBTC_OK) return dst;
  }
  // the persistent launch reads the per-XCD queues, the plain one the plan order
  const bool queued = opt.mode == BBTC_MODE_PERSISTENT && !budgeted;
  if (queued) {
    bbtc_status qst = compose_queues(pl);
    if (qst != BBTC_OK) return qst;
  } else {
    compose_plan_order(pl);
  }
  const int64_t nt = (int64_t)pl->h_tasks.size();
  HIP_TRY(pl->acp.ensure((size_t)nb + 1), "alloc");
  HIP_TRY(pl->tasks.ensure((size_t)nt), "alloc tasks");
  HIP_TRY((queued ? pl->xitems : pl->items).ensure(pl->nitems), "alloc items");
  HIP_TRY(pl->cursor.ensure(kMaxQueues), "alloc");
  {  // through the pinned stage; the final synchronisation below covers these copies
    const size_t wa = sizeof(uint64_t) * (size_t)(nb + 1), wt = sizeof(DevTask) * (size_t)nt;
    // persistent launches: the work items are written on the device from
    // runs of task items (a few per task) instead of being uploaded
    const size_t nr = queued ? pl->h_runs.size() : 0, nh = queued ? pl->h_heavy.size() : 0;
    const size_t o_runs = 0, o_ti = align16(o_runs + sizeof(ItemRun) * nr),
                 o_hs = align16(o_ti + sizeof(TaskItems) * (size_t)nt),
                 o_hr = align16(o_hs + sizeof(uint32_t) * (size_t)(nb + 1)),
                 o_hc = align16(o_hr + sizeof(HeavyCol) * nh), we = align16(o_hc + sizeof(uint32_t) * nh);
    const size_t e0 = align16(wa + wt);
    HIP_TRY(pl->stage.ensure(e0 + (queued ? we : 0)), "pinned alloc");
    char* st = pl->stage.ptr;
    std::memcpy(st, acp.data(), wa);
    std::memcpy(st + wa, pl->h_dtasks.data(), wt);
    HIP_TRY(hipMemcpyAsync(pl->acp.ptr, st, wa, hipMemcpyHostToDevice, s), "H2D");
    HIP_TRY(hipMemcpyAsync(pl->tasks.ptr, st + wa, wt, hipMemcpyHostToDevice, s), "H2D");
    if (queued && pl->nitems) {
      char* e = st + e0;
      std::memcpy(e + o_runs, pl->h_runs.data(), sizeof(ItemRun) * nr);
      TaskItems* ti = (TaskItems*)(e + o_ti);
      for (int64_t q = 0; q < nt; ++q) {
        const bbtc_task& t = pl->h_tasks[q];
        const int64_t cid = col_block_id(t.i, t.j);
        ti[q] = TaskItems{pl->h_nhub[q], pl->h_nper[q], (uint32_t)pl->h_nzc[cid], (uint32_t)cid};
      }
      uint32_t* hs = (uint32_t*)(e + o_hs);
      for (int64_t b = 0; b <= nb; ++b) hs[b] = (uint32_t)pl->h_hstart[b];
      std::memcpy(e + o_hr, pl->h_heavy.data(), sizeof(HeavyCol) * nh);
      uint32_t* hc = (uint32_t*)(e + o_hc);  // first chunk number of each record within its block
      for (int64_t b = 0; b < nb; ++b) {
        uint32_t c = 0;
        for (int64_t r = pl->h_hstart[b]; r < pl->h_hstart[b + 1]; ++r) {
          hc[r] = c;
          c += (pl->h_heavy[r].cnt + kHubChunk - 1) / kHubChunk;
        }
      }
      HIP_TRY(pl->emit.ensure(we), "alloc");
      HIP_TRY(hipMemcpyAsync(pl->emit.ptr, e, we, hipMemcpyHostToDevice, s), "H2D");
      const char* d = pl->emit.ptr;
      HIP_TRY(launch_emit_items((const ItemRun*)(d + o_runs), (int32_t)nr, (const TaskItems*)(d + o_ti),
                                (const uint32_t*)(d + o_hs), (const HeavyCol*)(d + o_hr), (const uint32_t*)(d + o_hc),
                                kHubChunk, pl->xitems.ptr, (uint32_t)pl->nitems, s),
              "emit work items");
    }
  }
  if (pl->nitems && !queued)
    HIP_TRY(hipMemcpyAsync(pl->items.ptr, pl->h_items.data(), sizeof(DevItem) * pl->h_items.size(),
                           hipMemcpyHostToDevice, s),
            "H2D");
  pl->plan_order_items = !queued;
  if (pl->dense_k0 < p)  // the dense-slice counters, through the (now free) cut stage
    HIP_TRY(hipMemcpyAsync(pl->cstage.ptr, pl->dcount.ptr, 8, hipMemcpyDeviceToHost, s), "D2H");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  pl->dense_words = pl->dense_k0 < p ? ((const uint32_t*)pl->cstage.ptr)[0] : 0;
  pl->dense_slices = pl->dense_k0 < p ? ((const uint32_t*)pl->cstage.ptr)[1] : 0;

  // ---- statistics (Sec. 4.4 quantities and the byte model) ----
  bbtc_stats& st = pl->stats;
  std::memset(&st, 0, sizeof(st));
  st.n = n;
  st.m = (int64_t)m;
  st.p = p;
  st.ntasks = nt;
  st.work_tasks = (int64_t)pl->h_work.size();
  st.nitems = (int64_t)pl->nitems;
  for (auto v : pl->h_nnz) st.m_max = std::max<int64_t>(st.m_max, v);
  st.m_avg = 2.0 * (double)m / ((double)p * (double)(p + 1));
  st.lambda = st.m_avg > 0 ? (double)st.m_max / st.m_avg : 0.0;
  st.d_max_block = hd[0];
  st.d_max = hd[1];
  st.c = st.d_max_block > 0 ? (double)st.d_max / (double)st.d_max_block : 0.0;
  st.wedges = (int64_t)wedges;
  st.stored_rows = n - pl->rT;
  st.bound_bytes = (int64_t)bound_bytes(pl->h_cuts, p, pl->rT);
  st.dense_slices = pl->dense_slices;
  st.dense_bytes = 4 * pl->dense_words;
  st.bytes_colidx = 4 * (int64_t)(p + 2) * (int64_t)m;
  int64_t rowidx = 0;
  for (const auto& t : pl->h_tasks)
    rowidx += 12 * (pl->h_nzr[block_id(p, t.i, t.j)] + pl->h_nzr[block_id(p, t.j, t.k)] +
                    pl->h_nzr[block_id(p, t.i, t.k)]);
  st.bytes_rowidx = rowidx;
  st.bytes_total = st.bytes_colidx + st.bytes_rowidx + 8 * nt;
  if (budgeted) {
    bbtc_status sst = stream_finish(pl, s);
    if (sst != BBTC_OK) return sst;
  } else if (opt.device_budget_bytes > 0 && (int64_t)pl->footprint() > opt.device_budget_bytes) {
    bbtc_status sst = stream_setup(pl, s);
    if (sst != BBTC_OK) return sst;
  }
  st.footprint = (int64_t)pl->footprint();
  st.partition_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  pl->ready = true;
  return BBTC_OK;
}

// ------------------------------------------------------------ budgeted partition
// A graph whose resident partition would exceed the device budget is
// partitioned from its CSR (host or device memory) in pieces, within the
// budget: the degree order from the row pointers; the out- and in-degrees
// chunk by chunk of input rows; then, group of parts by group of parts, the
// out-rows (sorted, with their stored block boundaries) and, separately, the
// in side (in-rows grouped by part, then the block-major in side), each
// group from one pass over the input chunks, copied to pinned host memory.
// Groups are as large as the budget allows; a single part whose build does
// not fit is BBTC_EBUDGET.  The count then streams (stream_finish).

// Upper bound of the device bytes of a resident partition.
int64_t resident_estimate(int64_t n, int64_t nnz, int32_t p, int64_t bound_deg, bool host_input, int64_t rpb) {
  const int64_t m = nnz / 2;
  const int64_t bd = bound_deg == 0 ? kAutoBound[3] : bound_deg;  // 0: automatic (at most 4m bytes, or as at 32)
  int64_t stored = bd < 0 ? n : std::min<int64_t>(n, nnz / (bd + 1));
  if (bound_deg == 0) stored = std::max<int64_t>(stored, m / (p + 1));
  int64_t b = (host_input ? rpb * (n + 1) + 4 * nnz : 0);
  b += 16 * n + 8 * n + 8 * n + 8 * (n + 1) + 12 * n;  // keys, perm/order, degrees, row pointers, row lists
  b += 4 * (m + 4) * 2 + 4 * m * 4 + 4 + 2 * (m + 16) + 4 * nnz;  // ocol, icol, acol, aoff, asrc, icolb, ocol16, ranks
  b += 4 * (int64_t)(p + 1) * stored;                  // stored block boundaries
  b += 16 * ((int64_t)p * (n / kPrepRows + p) + 1);    // chunk counters and their scans
  b += 12 * (m / 256 + 1) + (int64_t)p * (p + 1) * (p + 2) / 6 * 48 + (64 << 20);  // hubs, tasks, items, slack
  return b;
}

struct InChunk {
  int64_t x0, x1, e0, e1;
};

struct BudgetBuild {
  bbtc_plan* pl;
  const bbtc_csr* g;
  hipStream_t s;
  bool on_device;
  int rp64;
  size_t rpb;
  std::vector<int64_t> hrp;   // row pointers on the host (64-bit)
  std::vector<InChunk> chunks;
  DevBuf<char> crp;           // a chunk's row pointers (host input)
  DevBuf<int32_t> ccol;       // a chunk's entries (host input)
  DevBuf<uint32_t> hpref, cur_o, cur_i, q;
  uint64_t max_rows = 0, max_ent = 0;

  const int64_t* rp_host() const { return hrp.data(); }
  // Device pointers of chunk c: its row pointers (at row x0) and entries
  // (shifted so that absolute positions index them).
  bbtc_status load(size_t c, const void** rp, const int32_t** col) {
    const InChunk& k = chunks[c];
    if (on_device) {
      *rp = (const char*)g->rowptr + (size_t)k.x0 * rpb;
      *col = g->colidx;
      return BBTC_OK;
    }
    HIP_TRY(hipMemcpyAsync(crp.ptr, (const char*)g->rowptr + (size_t)k.x0 * rpb, (size_t)(k.x1 - k.x0 + 1) * rpb,
                           hipMemcpyHostToDevice, s),
            "H2D rows");
    if (k.e1 > k.e0)
      HIP_TRY(hipMemcpyAsync(ccol.ptr, g->colidx + k.e0, 4 * (size_t)(k.e1 - k.e0), hipMemcpyHostToDevice, s),
              "H2D entries");
    *rp = crp.ptr;
    *col = ccol.ptr - k.e0;
    return BBTC_OK;
  }
  // One pass of the degree kernels over every chunk: od != nullptr counts
  // the out-/in-degrees (with the entry checks of trusted input when check),
  // otherwise only the row lists are made and the fill of the ranks
  // [rlo, rhi) writes ocol/icol (either may be null).
  bbtc_status pass(uint32_t* od, uint32_t* idg, int check, int32_t rlo, int32_t rhi, int32_t* ocol, int32_t* icol) {
    bbtc_plan* P = pl;
    for (size_t c = 0; c < chunks.size(); ++c) {
      const InChunk& k = chunks[c];
      const void* rp;
      const int32_t* col;
      bbtc_status st = load(c, &rp, &col);
      if (st != BBTC_OK) return st;
      HIP_TRY(hipMemsetAsync(P->err.ptr + 4, 0, 8, s), "memset");
      const RowRange rr{k.x0, P->n, k.e0, k.e1, rlo, rhi};
      const int64_t nr = k.x1 - k.x0;
      HIP_TRY(launch_degs(rp, rp64, col, nr, rr, P->perm.ptr, od, idg, P->longrows.ptr, P->err.ptr + 4,
                          P->hugerows.ptr, P->err.ptr + 5, hpref.ptr, P->err.ptr, check, nullptr, s),
              "degrees");
      if (!od)
        HIP_TRY(launch_fill(rp, rp64, col, nr, rr, P->perm.ptr, P->orow.ptr, P->irow.ptr, ocol, icol, P->longrows.ptr,
                            P->err.ptr + 4, P->hugerows.ptr, P->err.ptr + 5, hpref.ptr, cur_o.ptr, cur_i.ptr, nullptr,
                            s),
                "fill");
    }
    return BBTC_OK;
  }
};

bbtc_status partition_budgeted(const bbtc_csr* g, hipStream_t s, bbtc_plan* pl,
                               std::chrono::steady_clock::time_point t0) {
  const bbtc_options& opt = pl->opt;
  const int64_t n = g->n, nnz = g->nnz, budget = opt.device_budget_bytes;
  BudgetBuild B;
  B.pl = pl;
  B.g = g;
  B.s = s;
  B.on_device = (g->flags & BBTC_CSR_DEVICE) != 0;
  B.rp64 = g->rowptr_bits == 64;
  B.rpb = B.rp64 ? 8 : 4;
  const bool symmetric_check = (g->flags & BBTC_CSR_TRUSTED) == 0;
  // row pointers on the host, chunks of input rows (at most max_ent entries
  // and max_rows rows each; a longer row is a chunk of its own)
  B.hrp.resize((size_t)n + 1);
  if (B.on_device) {
    std::vector<char> tmp((size_t)(n + 1) * B.rpb);
    HIP_TRY(hipMemcpy(tmp.data(), g->rowptr, tmp.size(), hipMemcpyDeviceToHost), "D2H rowptr");
    for (int64_t x = 0; x <= n; ++x)
      B.hrp[x] = B.rp64 ? ((const int64_t*)tmp.data())[x] : (int64_t)((const int32_t*)tmp.data())[x];
  } else {
    for (int64_t x = 0; x <= n; ++x)
      B.hrp[x] = B.rp64 ? ((const int64_t*)g->rowptr)[x] : (int64_t)((const int32_t*)g->rowptr)[x];
  }
  // a chunk's entries take at most 1/32 of the budget
  const uint64_t ent_cap = (uint64_t)std::max<int64_t>(4096, std::min<int64_t>(1 << 28, budget / 128));
  const uint64_t row_cap = std::min<uint64_t>(1 << 23, std::max<uint64_t>(4096, ent_cap / 4));
  for (int64_t x0 = 0; x0 < n;) {
    int64_t x1 = x0 + 1;
    while (x1 < n && (uint64_t)(x1 + 1 - x0) <= row_cap && (uint64_t)(B.hrp[x1 + 1] - B.hrp[x0]) <= ent_cap) ++x1;
    B.chunks.push_back(InChunk{x0, x1, B.hrp[x0], B.hrp[x1]});
    B.max_rows = std::max<uint64_t>(B.max_rows, (uint64_t)(x1 - x0));
    B.max_ent = std::max<uint64_t>(B.max_ent, (uint64_t)(B.hrp[x1] - B.hrp[x0]));
    x0 = x1;
  }
  if (!B.on_device) {
    HIP_TRY(B.crp.ensure((B.max_rows + 1) * B.rpb), "alloc chunk rows");
    HIP_TRY(B.ccol.ensure(B.max_ent), "alloc chunk entries");
  }
  HIP_TRY(pl->err.ensure(16), "alloc");
  HIP_TRY(pl->longrows.ensure(B.max_rows), "alloc");
  HIP_TRY(pl->hugerows.ensure(B.max_rows), "alloc");
  HIP_TRY(B.hpref.ensure(B.max_rows + 1), "alloc");
  HIP_TRY(B.cur_o.ensure(B.max_rows), "alloc");
  HIP_TRY(B.cur_i.ensure(B.max_rows), "alloc");
  HIP_TRY(hipMemsetAsync(pl->err.ptr, 0, 8 * sizeof(uint32_t), s), "memset");
  if (B.on_device && symmetric_check) {  // untrusted device input: the validation kernels, on the whole input
    HIP_TRY(pl->irow.ensure((size_t)n + 1), "alloc");
    DevBuf<uint32_t> l1, l2;
    HIP_TRY(l1.ensure((size_t)n), "alloc");
    HIP_TRY(l2.ensure((size_t)n), "alloc");
    HIP_TRY(launch_validate(g->rowptr, B.rp64, g->colidx, n, nnz, 1, pl->err.ptr, l1.ptr, pl->err.ptr + 4, l2.ptr,
                            pl->err.ptr + 5, pl->irow.ptr, s),
            "validate");
    uint32_t e = 0;
    HIP_TRY(hipMemcpyAsync(&e, pl->err.ptr, 4, hipMemcpyDeviceToHost, s), "D2H err");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    l1.release();
    l2.release();
    if (e) return decode_device_err(e);
    HIP_TRY(hipMemsetAsync(pl->err.ptr, 0, 8 * sizeof(uint32_t), s), "memset");
  }
  {  // (after validation, so that bad input is EINVAL whatever the budget) the
     // arrays of the degree order must fit at least: keys (two), perm,
     // order, the radix histogram and scan partials, the row pointers of
     // host input, and a little room for the small tables
    const uint64_t hist = radix_hist_entries((uint64_t)n);
    const uint64_t part = scan_partial_entries(std::max<uint64_t>(hist, (uint64_t)n + 1)) + 4096;
    const int64_t fixed = 24 * n + 4 * (int64_t)(hist + part) + (B.on_device ? 0 : (int64_t)B.rpb * (n + 1)) +
                          (1 << 20);
    if (fixed > budget)
      return fail(BBTC_EBUDGET, "device budget below the " + std::to_string(fixed) +
                                    " B that ordering the vertices needs");
  }
  // trusted input: the degree pass checks the entries (untrusted input was
  // checked above, on the host or by the validation kernels)
  const int check_in_degs = symmetric_check ? 0 : 1;

  // ---- degree order (Sec. 4.1) from the row pointers alone ----
  pl->idbits = bits_for((uint64_t)(n - 1));
  {
    DevBuf<char> drp;
    const void* rp = g->rowptr;
    if (!B.on_device) {
      HIP_TRY(drp.ensure((size_t)(n + 1) * B.rpb), "alloc rowptr");
      HIP_TRY(hipMemcpyAsync(drp.ptr, g->rowptr, (size_t)(n + 1) * B.rpb, hipMemcpyHostToDevice, s), "H2D rowptr");
      rp = drp.ptr;
    }
    HIP_TRY(pl->keys_a.ensure((size_t)n), "alloc keys");
    HIP_TRY(pl->keys_b.ensure((size_t)n), "alloc keys");
    HIP_TRY(pl->hist.ensure(radix_hist_entries((uint64_t)n)), "alloc hist");
    HIP_TRY(pl->partial.ensure(scan_partial_entries(std::max<uint64_t>(radix_hist_entries((uint64_t)n), (uint64_t)n + 1)) +
                               4096),
            "alloc partial");
    HIP_TRY(pl->perm.ensure((size_t)n), "alloc perm");
    HIP_TRY(pl->order.ensure((size_t)n), "alloc order");
    uint64_t* sorted = nullptr;
    HIP_TRY(launch_degkey(rp, B.rp64, n, pl->idbits, pl->keys_a.ptr, s), "degkey");
    HIP_TRY(radix_sort_u64(pl->keys_a.ptr, pl->keys_b.ptr, (uint64_t)n, pl->idbits, 2 * pl->idbits, pl->hist.ptr,
                           pl->partial.ptr, &sorted, s),
            "degree sort");
    HIP_TRY(launch_perm(sorted, n, pl->idbits, pl->order.ptr, pl->perm.ptr, s), "perm");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    pl->keys_a.release();
    pl->keys_b.release();
    pl->hist.release();
    pl->order.release();
  }

  // ---- out- and in-degrees, chunk by chunk ----
  HIP_TRY(pl->od.ensure((size_t)n), "alloc od");
  HIP_TRY(pl->idg.ensure((size_t)n), "alloc idg");
  bbtc_status st = B.pass(pl->od.ptr, pl->idg.ptr, check_in_degs, 0, (int32_t)n, nullptr, nullptr);
  if (st != BBTC_OK) return st;
  unsigned long long* d_wedges = (unsigned long long*)(pl->err.ptr + 6);
  HIP_TRY(hipMemsetAsync(pl->err.ptr + 8, 0, 16, s), "memset");
  HIP_TRY(launch_degree_stats(pl->od.ptr, pl->idg.ptr, n, bound_thresholds(opt), d_wedges, pl->err.ptr + 8, s),
          "degree statistics");
  HIP_TRY(pl->orow.ensure((size_t)n + 1), "alloc orow");
  HIP_TRY(pl->irow.ensure((size_t)n + 1), "alloc irow");
  HIP_TRY(scan_u32(pl->od.ptr, pl->orow.ptr, (uint64_t)n, pl->partial.ptr, s), "scan out-degrees");
  HIP_TRY(scan_u32(pl->idg.ptr, pl->irow.ptr, (uint64_t)n, pl->partial.ptr, s), "scan in-degrees");
  std::vector<uint32_t> horow((size_t)n + 1), hirow((size_t)n + 1);
  uint32_t eb[12] = {0};
  uint64_t wedges = 0;
  HIP_TRY(hipMemcpyAsync(horow.data(), pl->orow.ptr, 4 * (n + 1), hipMemcpyDeviceToHost, s), "D2H orow");
  HIP_TRY(hipMemcpyAsync(hirow.data(), pl->irow.ptr, 4 * (n + 1), hipMemcpyDeviceToHost, s), "D2H irow");
  HIP_TRY(hipMemcpyAsync(eb, pl->err.ptr, sizeof(eb), hipMemcpyDeviceToHost, s), "D2H err");
  HIP_TRY(hipMemcpyAsync(&wedges, d_wedges, 8, hipMemcpyDeviceToHost, s), "D2H wedges");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  if (eb[0]) return decode_device_err(eb[0]);
  const uint32_t* nshort = eb + 8;  // ranks at or below each degree threshold
  const uint64_t m = horow[n];
  if (m > (uint64_t)nnz / 2 || hirow[n] != horow[n]) return fail(BBTC_EINVAL, "input is not symmetric");
  pl->m = (int64_t)m;
  pl->od.release();
  pl->idg.release();
  // ---- cut vector (Sec. 4.1) ----
  int32_t p = opt.p;
  if (p == 0) {  // p near the average degree (Sec. 7.3)
    p = (int32_t)std::lround(2.0 * (double)m / (double)n);
    p = std::max(1, std::min<int32_t>(p, (int32_t)std::min<int64_t>(n, 256)));
  }
  pl->p = p;
  pl->opt.p = p;
  HIP_TRY(pl->cuts.ensure((size_t)p + 1), "alloc cuts");
  HIP_TRY(launch_cuts(pl->orow.ptr, n, p, opt.cut_mode, pl->cuts.ptr, s), "cuts");
  pl->h_cuts.assign((size_t)p + 1, 0);
  HIP_TRY(hipMemcpyAsync(pl->h_cuts.data(), pl->cuts.ptr, 4 * (p + 1), hipMemcpyDeviceToHost, s), "D2H cuts");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  pl->rT = choose_rT(opt, nshort, pl->h_cuts, p, m, true);
  HIP_TRY(hipStreamSynchronize(s), "sync");
  const std::vector<int32_t>& cuts = pl->h_cuts;
  const int64_t nb = (int64_t)p * (p + 1) / 2;
  pl->ocut.assign(p + 1, 0);
  std::vector<uint64_t> icut(p + 1, 0);
  for (int32_t a = 0; a <= p; ++a) {
    pl->ocut[a] = horow[cuts[a]];
    icut[a] = hirow[cuts[a]];
  }
  // chunk tables and stored-boundary offsets of every part (as partition_impl)
  std::vector<int32_t> chunk0((size_t)p + 1);
  std::vector<uint64_t> ccbase((size_t)p + 1), botp((size_t)p + 1);
  int64_t nch = 0;
  uint64_t cc = 0, bp = 0;
  for (int32_t a = 0; a < p; ++a) {
    const int64_t va = cuts[a + 1] - cuts[a];
    const int64_t ca = (va + kPrepRows - 1) / kPrepRows;
    const int64_t sa = std::max<int64_t>(0, cuts[a + 1] - std::max<int64_t>(cuts[a], pl->rT));
    chunk0[a] = (int32_t)nch;
    ccbase[a] = cc;
    botp[a] = bp;
    nch += ca;
    cc += (uint64_t)(a + 1) * (uint64_t)ca;
    bp += (uint64_t)(p - a + 1) * (uint64_t)sa;
  }
  chunk0[p] = (int32_t)nch;
  ccbase[p] = cc;
  botp[p] = bp;
  pl->ccount = (int64_t)cc;
  pl->h_botp = botp;
  const size_t w8 = sizeof(uint64_t) * (size_t)(p + 1), wb = sizeof(unsigned long long) * (size_t)nb;
  const size_t o_cb = align16(sizeof(int32_t) * (size_t)(p + 1)), o_hd = align16(o_cb + 2 * w8);
  HIP_TRY(pl->blk.ensure(o_hd + 16 + 3 * wb), "alloc");
  pl->chunk0 = (int32_t*)pl->blk.ptr;
  pl->ccbase = (uint64_t*)(pl->blk.ptr + o_cb);
  pl->botp = pl->ccbase + (p + 1);
  pl->head = (uint32_t*)(pl->blk.ptr + o_hd);
  pl->bnnz = (unsigned long long*)(pl->blk.ptr + o_hd + 16);
  pl->bnzr = pl->bnnz + nb;
  pl->bnzc = pl->bnzr + nb;
  {
    HIP_TRY(pl->stage.ensure(std::max(o_hd, 16 + 3 * wb)), "pinned alloc");
    char* stg = pl->stage.ptr;
    std::memcpy(stg, chunk0.data(), sizeof(int32_t) * (p + 1));
    std::memcpy(stg + o_cb, ccbase.data(), w8);
    std::memcpy(stg + o_cb + w8, botp.data(), w8);
    HIP_TRY(hipMemcpyAsync(pl->blk.ptr, stg, o_hd, hipMemcpyHostToDevice, s), "H2D");
    HIP_TRY(hipMemsetAsync(pl->head, 0, 16 + 3 * wb, s), "memset");
    HIP_TRY(hipStreamSynchronize(s), "sync");
  }
  pl->split = kHubSplit;
  const uint64_t hcap = m / kHubSplit + 1;
  HIP_TRY(pl->heavy.ensure((size_t)hcap), "alloc");
  // pinned host arrays of the count phase (active columns: at most m)
  HIP_TRY(hipHostMalloc((void**)&pl->h_ocol, 4 * std::max<uint64_t>(m, 1), hipHostMallocDefault), "pinned alloc");
  HIP_TRY(hipHostMalloc((void**)&pl->h_bot, 4 * std::max<uint64_t>(bp, 1), hipHostMallocDefault), "pinned alloc");
  HIP_TRY(hipHostMalloc((void**)&pl->h_orow, 4 * ((size_t)n + 1), hipHostMallocDefault), "pinned alloc");
  HIP_TRY(hipHostMalloc((void**)&pl->h_acol, 4 * std::max<uint64_t>(m, 1), hipHostMallocDefault), "pinned alloc");
  HIP_TRY(hipHostMalloc((void**)&pl->h_aoff, 4 * (m + 1), hipHostMallocDefault), "pinned alloc");
  HIP_TRY(hipHostMalloc((void**)&pl->h_icolb, 4 * std::max<uint64_t>(m, 1), hipHostMallocDefault), "pinned alloc");
  std::memcpy(pl->h_orow, horow.data(), 4 * ((size_t)n + 1));

  BlockBuild bb;
  std::memset(&bb, 0, sizeof(bb));
  bb.p = p;
  bb.rT = (int32_t)pl->rT;
  bb.nchunks = (int32_t)nch;
  bb.cuts = pl->cuts.ptr;
  bb.chunk0 = pl->chunk0;
  bb.ccbase = pl->ccbase;
  bb.orow = pl->orow.ptr;
  bb.botp = pl->botp;
  bb.irow = pl->irow.ptr;
  bb.bnnz = pl->bnnz;
  bb.bnzr = pl->bnzr;
  bb.bnzc = pl->bnzc;
  bb.dmax_block = pl->head + 1;
  bb.split = pl->split;
  bb.heavy = pl->heavy.ptr;
  bb.nheavy = pl->head;
  bb.heavy_cap = (uint32_t)hcap;
  HIP_TRY(B.q.ensure(4), "alloc");
  // what stays on the device meanwhile; groups take the rest of the budget
  auto room = [&]() { return budget - (int64_t)pl->footprint() - (int64_t)(B.crp.bytes() + B.ccol.bytes() +
                                                                          B.hpref.bytes() + B.cur_o.bytes() +
                                                                          B.cur_i.bytes() + B.q.bytes()); };
  DevBuf<int32_t> ga, gb;  // group rows and scratch
  DevBuf<uint32_t> gbot, gacol, gaoff, gasrc, gcc;

  // ---- out side, group by group: out-rows sorted, stored boundaries ----
  // group buffers (rows, scratch, boundaries) and the row lists of a group
  // are allocated per group and released after it, so each group may use
  // all of room()
  auto drop_lists = [&]() {
    pl->midrows.release();
    pl->longrows.release();
    pl->hugerows.release();
  };
  for (int32_t a0 = 0; a0 < p;) {
    int32_t a1 = a0;
    int64_t need = 0;
    drop_lists();
    const int64_t avail = room();
    while (a1 < p) {
      const int64_t e = (int64_t)(pl->ocut[a1 + 1] - pl->ocut[a0]), rows = cuts[a1 + 1] - cuts[a0];
      const int64_t want = 8 * (e + 8) + 4 * (int64_t)(botp[a1 + 1] - botp[a0]) + 12 * rows + 1024;
      if (a1 > a0 && want > avail) break;
      need = want;
      ++a1;
    }
    if (need > avail)
      return fail(BBTC_EBUDGET, "device budget too small to build the out-rows of part " + std::to_string(a0) + " (" +
                                    std::to_string(need) + " B needed, " + std::to_string(room()) + " B free)");
    const int64_t R0 = cuts[a0], R1 = cuts[a1];
    const uint64_t o0 = pl->ocut[a0], ne = pl->ocut[a1] - o0;
    HIP_TRY(ga.ensure(ne + 8), "alloc group rows");
    HIP_TRY(gb.ensure(ne + 8), "alloc group scratch");
    HIP_TRY(gbot.ensure(botp[a1] - botp[a0]), "alloc group boundaries");
    HIP_TRY(pl->midrows.ensure((size_t)(R1 - R0)), "alloc");
    HIP_TRY(pl->longrows.ensure(std::max<size_t>((size_t)(R1 - R0), B.max_rows)), "alloc");
    HIP_TRY(pl->hugerows.ensure(std::max<size_t>((size_t)(R1 - R0), B.max_rows)), "alloc");
    if ((st = B.pass(nullptr, nullptr, 0, (int32_t)R0, (int32_t)R1, ga.ptr - o0, nullptr)) != BBTC_OK) return st;
    HIP_TRY(hipMemsetAsync(B.q.ptr, 0, 16, s), "memset");
    HIP_TRY(launch_segsort(pl->orow.ptr + R0, ga.ptr - o0, R1 - R0, pl->idbits, pl->midrows.ptr, pl->longrows.ptr,
                           pl->hugerows.ptr, B.q.ptr, gb.ptr - o0, s),
            "sort out-rows");
    bb.chunk_base = chunk0[a0];
    bb.ocol = ga.ptr - o0;
    bb.bot = gbot.ptr - botp[a0];
    HIP_TRY(launch_bot(bb, chunk0[a1] - chunk0[a0], s), "block row index");
    if (ne) HIP_TRY(hipMemcpyAsync(pl->h_ocol + o0, ga.ptr, 4 * ne, hipMemcpyDeviceToHost, s), "D2H");
    if (botp[a1] > botp[a0])
      HIP_TRY(hipMemcpyAsync(pl->h_bot + botp[a0], gbot.ptr, 4 * (botp[a1] - botp[a0]), hipMemcpyDeviceToHost, s),
              "D2H");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    ga.release();
    gb.release();
    gbot.release();
    a0 = a1;
  }

  // ---- in side, group by group: in-rows grouped by part, block-major ----
  uint64_t xbase = 0;
  uint32_t hdone = 0;  // hub records written by earlier groups
  for (int32_t a0 = 0; a0 < p;) {
    int32_t a1 = a0;
    int64_t need = 0;
    drop_lists();
    const int64_t avail = room();
    while (a1 < p) {
      const int64_t e = (int64_t)(icut[a1 + 1] - icut[a0]), rows = cuts[a1 + 1] - cuts[a0];
      const int64_t cols = std::min<int64_t>(e, rows * (int64_t)(a1 + 1));  // active columns, at most
      const int64_t want =
          8 * (e + 8) + 12 * (cols + 1) + 12 * rows + 16 * (int64_t)(ccbase[a1 + 1] - ccbase[a0] + 1) + 1024;
      if (a1 > a0 && want > avail) break;
      need = want;
      ++a1;
    }
    if (need > avail)
      return fail(BBTC_EBUDGET, "device budget too small to build the in side of part " + std::to_string(a0) + " (" +
                                    std::to_string(need) + " B needed, " + std::to_string(room()) + " B free)");
    const int64_t R0 = cuts[a0], R1 = cuts[a1];
    const uint64_t i0 = icut[a0], ne = icut[a1] - i0, c0 = ccbase[a0], ncc = ccbase[a1] - c0;
    HIP_TRY(ga.ensure(ne + 8), "alloc group in-rows");
    HIP_TRY(gb.ensure(ne + 8), "alloc group scratch");
    HIP_TRY(gcc.ensure(4 * (ncc + 1)), "alloc group counters");
    HIP_TRY(pl->midrows.ensure((size_t)(R1 - R0)), "alloc");
    HIP_TRY(pl->longrows.ensure(std::max<size_t>((size_t)(R1 - R0), B.max_rows)), "alloc");
    HIP_TRY(pl->hugerows.ensure(std::max<size_t>((size_t)(R1 - R0), B.max_rows)), "alloc");
    if (pl->partial.cap < scan_partial_entries(ncc)) HIP_TRY(pl->partial.ensure(scan_partial_entries(ncc) + 4096), "alloc");
    if ((st = B.pass(nullptr, nullptr, 0, (int32_t)R0, (int32_t)R1, nullptr, ga.ptr - i0)) != BBTC_OK) return st;
    HIP_TRY(hipMemsetAsync(B.q.ptr, 0, 16, s), "memset");
    HIP_TRY(launch_inrows_sort(pl->irow.ptr + R0, ga.ptr - i0, R1 - R0, pl->midrows.ptr, pl->longrows.ptr,
                               pl->hugerows.ptr, B.q.ptr, s),
            "sort in-rows");
    HIP_TRY(launch_inrows_group(pl->irow.ptr + R0, ga.ptr - i0, pl->longrows.ptr, pl->hugerows.ptr, B.q.ptr,
                                gb.ptr - i0, pl->cuts.ptr, p, GroupChunks{0, nullptr, nullptr, nullptr, nullptr, 0, false},
                                s),
            "group in-rows");
    uint32_t* ccnt = gcc.ptr;                   // [ncc] column counts, [ncc] entry counts,
    uint32_t* ecnt = gcc.ptr + (ncc + 1);       // then their scans
    uint32_t* ccoff = gcc.ptr + 2 * (ncc + 1);
    uint32_t* ecoff = gcc.ptr + 3 * (ncc + 1);
    bb.chunk_base = chunk0[a0];
    bb.icol = ga.ptr - i0;
    bb.ccnt = ccnt - c0;
    bb.ecnt = ecnt - c0;
    HIP_TRY(launch_acount(bb, chunk0[a1] - chunk0[a0], s), "active-column counts");
    HIP_TRY(scan_u32(ccnt, ccoff, ncc, pl->partial.ptr, s), "scan column counters");
    HIP_TRY(scan_u32(ecnt, ecoff, ncc, pl->partial.ptr, s), "scan entry counters");
    uint32_t ncols = 0;
    HIP_TRY(hipMemcpyAsync(&ncols, ccoff + ncc, 4, hipMemcpyDeviceToHost, s), "D2H");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    HIP_TRY(gacol.ensure((size_t)ncols + 1), "alloc group active columns");
    HIP_TRY(gaoff.ensure((size_t)ncols + 1), "alloc group offsets");
    HIP_TRY(gasrc.ensure((size_t)ncols + 1), "alloc group sources");
    bb.ccoff = ccoff - c0;
    bb.ecoff = ecoff - c0;
    bb.acol = (int32_t*)gacol.ptr;
    bb.aoff = gaoff.ptr;
    bb.asrc = gasrc.ptr;
    bb.ebase = (uint32_t)i0;
    bb.xbase = xbase;
    HIP_TRY(launch_acol(bb, chunk0[a1] - chunk0[a0], s), "active columns");
    HIP_TRY(launch_set_at(gaoff.ptr, ccoff + ncc, (uint32_t)icut[a1], s), "in-slice sentinel");
    HIP_TRY(launch_icolb(gaoff.ptr, gasrc.ptr, ga.ptr - i0, gb.ptr - i0, ccoff + ncc, ncols, pl->split,
                         pl->heavy.ptr, hdone, pl->head, (uint32_t)hcap, xbase, s),
            "block-major in side");
    if (ncols) {
      HIP_TRY(hipMemcpyAsync(pl->h_acol + xbase, gacol.ptr, 4 * (size_t)ncols, hipMemcpyDeviceToHost, s), "D2H");
      HIP_TRY(hipMemcpyAsync(pl->h_aoff + xbase, gaoff.ptr, 4 * ((size_t)ncols + 1), hipMemcpyDeviceToHost, s), "D2H");
    }
    if (ne) HIP_TRY(hipMemcpyAsync(pl->h_icolb + i0, gb.ptr, 4 * ne, hipMemcpyDeviceToHost, s), "D2H");
    HIP_TRY(hipMemcpyAsync(&hdone, pl->head, 4, hipMemcpyDeviceToHost, s), "D2H");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    hdone = std::min<uint32_t>(hdone, (uint32_t)hcap);
    xbase += ncols;
    ga.release();
    gb.release();
    gacol.release();
    gaoff.release();
    gasrc.release();
    gcc.release();
    a0 = a1;
  }
  pl->h_aoff[xbase] = (uint32_t)m;
  // only what the count reads stays on the device: perm, orow, the plan
  // tables; the rest is released
  pl->irow.release();
  pl->midrows.release();
  pl->longrows.release();
  pl->hugerows.release();
  pl->partial.release();
  B.crp.release();
  B.ccol.release();
  B.hpref.release();
  B.cur_o.release();
  B.cur_i.release();
  B.q.release();
  return finish_partition(pl, s, m, wedges, hcap, true, t0);
}

bbtc_status partition_impl(const bbtc_csr* g, const bbtc_options* optp, hipStream_t s, bbtc_plan* pl) {
  auto t0 = std::chrono::steady_clock::now();
  bbtc_options opt;
  if (optp) opt = *optp; else fill_defaults(&opt);
  const int64_t n = g->n, nnz = g->nnz;
  if (n < 1 || n > 2147483647LL) return fail(BBTC_EINVAL, "n must be in [1, 2^31-1]");
  if (g->rowptr_bits != 32 && g->rowptr_bits != 64) return fail(BBTC_EINVAL, "rowptr_bits must be 32 or 64");
  if (!g->rowptr || (nnz > 0 && !g->colidx)) return fail(BBTC_EINVAL, "null rowptr/colidx");
  if (nnz < 0 || (nnz & 1)) return fail(BBTC_EINVAL, "nnz must be even and non-negative (both directions stored)");
  if (g->rowptr_bits == 32 && nnz > 2147483647LL) return fail(BBTC_EINVAL, "nnz needs 64-bit rowptr");
  if (nnz / 2 >= (1LL << 32) - 1) return fail(BBTC_EINVAL, "more than 2^32-2 edges");
  if (opt.p < 0 || opt.p > kMaxP || opt.p > n) return fail(BBTC_EINVAL, "p must be in [0, min(n, 2048)]");
  if (opt.cut_mode != BBTC_CUT_BALANCED && opt.cut_mode != BBTC_CUT_UNIFORM) return fail(BBTC_EINVAL, "bad cut_mode");
  if (opt.mode < BBTC_MODE_PERSISTENT || opt.mode > BBTC_MODE_PLAIN_HMAP) return fail(BBTC_EINVAL, "bad mode");
  if (opt.wave_min < 0 || opt.grid < 0 || opt.item_rows < 0 || opt.device_budget_bytes < 0 || opt.hash_min < -1 ||
      opt.bound_min_deg < -1)
    return fail(BBTC_EINVAL, "negative option");
  if (opt.graph != 0 && opt.graph != -1) return fail(BBTC_EINVAL, "graph must be 0 or -1");
  if (opt.dense < -1 || opt.dense > 1) return fail(BBTC_EINVAL, "dense must be -1, 0 or 1");
  const bool on_device = (g->flags & BBTC_CSR_DEVICE) != 0;
  const bool symmetric_check = (g->flags & BBTC_CSR_TRUSTED) == 0;
  const int rp64 = g->rowptr_bits == 64;
  if (!on_device) {
    // trusted host input: rowptr here, the entries on the device after the upload
    const bool rows = symmetric_check;
    bbtc_status st = rp64 ? validate_host((const int64_t*)g->rowptr, g->colidx, n, nnz, symmetric_check, rows)
                          : validate_host((const int32_t*)g->rowptr, g->colidx, n, nnz, symmetric_check, rows);
    if (st != BBTC_OK) return st;
  } else if (!is_device_pointer(g->rowptr) || (nnz > 0 && !is_device_pointer(g->colidx))) {
    return fail(BBTC_EINVAL, "BBTC_CSR_DEVICE set but rowptr/colidx are not device memory");
  }

  pl->ready = false;
  pl->drop_graph();
  pl->drop_stream();
  pl->hy = bbtc_plan::HybridHost();
  pl->plan_order_items = false;
  pl->opt = opt;
  pl->n = n;
  if (!pl->ncu) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    pl->ncu = prop.multiProcessorCount;
    pl->blocks_per_cu = count_persistent_blocks_per_cu();
    for (int q = 0; q < 4; ++q) {
      HIP_TRY(hipStreamCreateWithFlags(&pl->side[q], hipStreamNonBlocking), "hipStreamCreate");
      HIP_TRY(hipEventCreateWithFlags(&pl->ev_join[q], hipEventDisableTiming), "hipEventCreate");
    }
    HIP_TRY(hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming), "hipEventCreate");
    HIP_TRY(hipEventCreateWithFlags(&pl->ev_cuts, hipEventDisableTiming), "hipEventCreate");
  }
  // over the device budget even to partition: partition in pieces
  if (opt.device_budget_bytes > 0) {
    const int32_t pe = opt.p > 0 ? opt.p : 256;
    if (resident_estimate(n, nnz, pe, opt.bound_min_deg, !on_device, rp64 ? 8 : 4) > opt.device_budget_bytes) {
      pl->ocol16.release();  // streamed counts read the four-byte rows
      pl->rc.release();
      return partition_budgeted(g, s, pl, t0);
    }
  }

  const size_t rp_bytes = (size_t)(n + 1) * (rp64 ? 8 : 4);
  const void* rowptr = g->rowptr;
  const int32_t* col = g->colidx;
  if (!on_device) {
    HIP_TRY(pl->in_rowptr.ensure(rp_bytes), "alloc input rowptr");
    HIP_TRY(pl->in_col.ensure((size_t)nnz), "alloc input colidx");
    HIP_TRY(hipMemcpyAsync(pl->in_rowptr.ptr, g->rowptr, rp_bytes, hipMemcpyHostToDevice, s), "H2D rowptr");
    if (nnz > 0)
      HIP_TRY(hipMemcpyAsync(pl->in_col.ptr, g->colidx, (size_t)nnz * 4, hipMemcpyHostToDevice, s), "H2D colidx");
    rowptr = pl->in_rowptr.ptr;
    col = pl->in_col.ptr;
  }
  // Untrusted device input: the validation kernels (with the symmetry check).
  // Trusted input (host or device): the degree pass checks the rest below.
  const int check_in_degs = symmetric_check ? 0 : 1;
  if (on_device && symmetric_check) {
    HIP_TRY(pl->err.ensure(16), "alloc");
    HIP_TRY(pl->longrows.ensure((size_t)n), "alloc");
    HIP_TRY(pl->hugerows.ensure((size_t)n), "alloc");
    HIP_TRY(pl->irow.ensure((size_t)n + 1), "alloc");  // chunk-prefix scratch for the validation kernels
    HIP_TRY(hipMemsetAsync(pl->err.ptr, 0, 8 * sizeof(uint32_t), s), "memset");
    HIP_TRY(launch_validate(rowptr, rp64, col, n, nnz, symmetric_check, pl->err.ptr, pl->longrows.ptr, pl->err.ptr + 4,
                            pl->hugerows.ptr, pl->err.ptr + 5, pl->irow.ptr, s),
            "validate");
    uint32_t e = 0;
    HIP_TRY(hipMemcpyAsync(&e, pl->err.ptr, 4, hipMemcpyDeviceToHost, s), "D2H err");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (e) return decode_device_err(e);
  }

  // ---- degree order (Sec. 4.1): sort keys (degree, id) ----
  pl->idbits = bits_for((uint64_t)(n - 1));
  const uint64_t mmax = (uint64_t)nnz / 2;
  HIP_TRY(pl->keys_a.ensure((size_t)n), "alloc keys");
  HIP_TRY(pl->keys_b.ensure((size_t)n), "alloc keys");
  HIP_TRY(pl->hist.ensure(radix_hist_entries((uint64_t)n)), "alloc hist");
  HIP_TRY(pl->partial.ensure(scan_partial_entries(std::max<uint64_t>(radix_hist_entries((uint64_t)n), (uint64_t)n + 1)) +
                             4096),
          "alloc partial");
  HIP_TRY(pl->perm.ensure((size_t)n), "alloc perm");
  HIP_TRY(pl->order.ensure((size_t)n), "alloc order");
  HIP_TRY(pl->od.ensure((size_t)n), "alloc od");
  HIP_TRY(pl->idg.ensure((size_t)n), "alloc idg");
  HIP_TRY(pl->orow.ensure((size_t)n + 1), "alloc orow");
  HIP_TRY(pl->irow.ensure((size_t)n + 1), "alloc irow");
  HIP_TRY(pl->longrows.ensure((size_t)n), "alloc");
  HIP_TRY(pl->hugerows.ensure((size_t)n), "alloc");
  HIP_TRY(pl->err.ensure(16), "alloc");
  HIP_TRY(hipMemsetAsync(pl->err.ptr, 0, 8 * sizeof(uint32_t), s), "memset");
  uint64_t* sorted = nullptr;
  HIP_TRY(launch_degkey(rowptr, rp64, n, pl->idbits, pl->keys_a.ptr, s), "degkey");
  // the keys start in id order and the sort is stable: the degree bits alone decide
  HIP_TRY(radix_sort_u64(pl->keys_a.ptr, pl->keys_b.ptr, (uint64_t)n, pl->idbits, 2 * pl->idbits, pl->hist.ptr,
                         pl->partial.ptr, &sorted, s),
          "degree sort");
  HIP_TRY(launch_perm(sorted, n, pl->idbits, pl->order.ptr, pl->perm.ptr, s), "perm");

  // ---- orientation: out-rows (higher ranks) and in-rows (lower ranks) ----
  // err[4]: rows too long for one lane, listed in longrows by launch_degs
  // err[4], err[5]: rows too long for one lane / huge rows, listed by launch_degs
  // the rank of every entry's vertex, gathered once here and read by the fill
  HIP_TRY(pl->rc.ensure((size_t)nnz), "alloc entry ranks");
  HIP_TRY(launch_degs(rowptr, rp64, col, n, whole_rows(n, nnz), pl->perm.ptr, pl->od.ptr, pl->idg.ptr, pl->longrows.ptr,
                      pl->err.ptr + 4, pl->hugerows.ptr, pl->err.ptr + 5, (uint32_t*)pl->keys_b.ptr, pl->err.ptr,
                      check_in_degs, pl->rc.ptr, s),
          "degrees");
  // while od/idg are degrees: the wedge count W (Sec. 4.4's work measure)
  // and the first rank whose block boundaries are stored
  unsigned long long* d_wedges = (unsigned long long*)(pl->err.ptr + 6);
  HIP_TRY(hipMemsetAsync(pl->err.ptr + 8, 0, 16, s), "memset");
  HIP_TRY(launch_degree_stats(pl->od.ptr, pl->idg.ptr, n, bound_thresholds(opt), d_wedges, pl->err.ptr + 8, s),
          "degree statistics");
  HIP_TRY(scan_u32(pl->od.ptr, pl->orow.ptr, (uint64_t)n, pl->partial.ptr, s), "scan out-degrees");
  HIP_TRY(scan_u32(pl->idg.ptr, pl->irow.ptr, (uint64_t)n, pl->partial.ptr, s), "scan in-degrees");
  HIP_TRY(pl->stage.ensure(64), "pinned alloc");
  uint32_t* mm = (uint32_t*)pl->stage.ptr;
  HIP_TRY(hipMemcpyAsync(&mm[0], pl->orow.ptr + n, 4, hipMemcpyDeviceToHost, s), "D2H m");
  HIP_TRY(hipMemcpyAsync(&mm[1], pl->irow.ptr + n, 4, hipMemcpyDeviceToHost, s), "D2H m");
  HIP_TRY(hipMemcpyAsync(&mm[2], pl->err.ptr, 4, hipMemcpyDeviceToHost, s), "D2H err");
  HIP_TRY(hipMemcpyAsync(&mm[4], d_wedges, 8, hipMemcpyDeviceToHost, s), "D2H wedges");
  HIP_TRY(hipMemcpyAsync(&mm[8], pl->err.ptr + 8, 16, hipMemcpyDeviceToHost, s), "D2H short rows");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  if (mm[2]) return decode_device_err(mm[2]);
  uint32_t nshort[4];  // ranks at or below each degree threshold
  std::memcpy(nshort, &mm[8], sizeof(nshort));
  uint64_t wedges = 0;
  std::memcpy(&wedges, &mm[4], 8);
  const uint64_t m = mm[0];
  if (m > mmax || mm[1] != mm[0]) return fail(BBTC_EINVAL, "input is not symmetric");
  pl->m = (int64_t)m;
  // + 4: the counting kernels read out-rows in aligned 16-byte blocks
  HIP_TRY(pl->ocol.ensure((size_t)m + 4), "alloc ocol");
  HIP_TRY(pl->icol.ensure((size_t)m + 4), "alloc icol");
  // od/idg are consumed (scanned): their first entries become the huge rows'
  // fill cursors (zeroed by launch_fill)
  HIP_TRY(launch_fill(rowptr, rp64, col, n, whole_rows(n, nnz), pl->perm.ptr, pl->orow.ptr, pl->irow.ptr, pl->ocol.ptr, pl->icol.ptr,
                      pl->longrows.ptr, pl->err.ptr + 4, pl->hugerows.ptr, pl->err.ptr + 5,
                      (const uint32_t*)pl->keys_b.ptr, pl->od.ptr, pl->idg.ptr, pl->rc.ptr, s),
          "fill");
  // ---- cut vector (Sec. 4.1): it needs only orow ----
  int32_t p = opt.p;
  if (p == 0) {  // p near the average degree (Sec. 7.3)
    double avg = 2.0 * (double)m / (double)n;
    p = (int32_t)std::lround(avg);
    p = std::max(1, std::min<int32_t>(p, (int32_t)std::min<int64_t>(n, 256)));
  }
  pl->p = p;
  pl->opt.p = p;
  HIP_TRY(pl->cuts.ensure((size_t)p + 1), "alloc cuts");
  HIP_TRY(launch_cuts(pl->orow.ptr, n, p, opt.cut_mode, pl->cuts.ptr, s), "cuts");
  // the cut vector goes to the host at once: the block tables it sizes are
  // computed while the rows are sorted
  HIP_TRY(pl->cstage.ensure(sizeof(int32_t) * (p + 1)), "pinned alloc");
  HIP_TRY(hipMemcpyAsync(pl->cstage.ptr, pl->cuts.ptr, sizeof(int32_t) * (p + 1), hipMemcpyDeviceToHost, s),
          "D2H cuts");
  HIP_TRY(hipEventRecord(pl->ev_cuts, s), "event");

  // ---- rows: out-rows sorted on s, in-rows grouped by part on side[2], at once ----
  // acol is not built yet: its m entries serve as the long/huge-row scratch of
  // both chains, one after the other.  The in-row lists use od, idg and keys_a
  // (free after the fill) and the counters err[5..7].
  HIP_TRY(pl->acol.ensure((size_t)m), "alloc active columns");
  HIP_TRY(pl->midrows.ensure((size_t)n), "alloc");
  hipStream_t si = pl->side[2];
  HIP_TRY(hipMemsetAsync(pl->err.ptr, 0, 32, s), "memset");
  HIP_TRY(hipEventRecord(pl->ev_fork, s), "event");
  HIP_TRY(hipStreamWaitEvent(si, pl->ev_fork, 0), "wait");
  HIP_TRY(launch_inrows_sort(pl->irow.ptr, pl->icol.ptr, n, pl->od.ptr, pl->idg.ptr, (uint32_t*)pl->keys_a.ptr,
                             pl->err.ptr + 5, si),
          "sort in-rows");
  HIP_TRY(launch_segsort(pl->orow.ptr, pl->ocol.ptr, n, pl->idbits, pl->midrows.ptr, pl->longrows.ptr,
                         pl->hugerows.ptr, pl->err.ptr, pl->acol.ptr, s),
          "sort out-rows");
  HIP_TRY(hipEventRecord(pl->ev_join[0], s), "event");  // the out-rows are done with the scratch
  HIP_TRY(hipStreamWaitEvent(si, pl->ev_join[0], 0), "wait");
  GroupChunks gc{0, nullptr, nullptr, nullptr, nullptr, 0, false};
  if ((uint64_t)m >= kLargeGraphEdges) {  // the first rows of the long/huge list are grouped in chunks over the whole chip
    gc.cap = (uint32_t)std::min<int64_t>(kGroupRowCap, (int64_t)(kGroupCounters / (uint64_t)p));
    // a listed row has more than 1024 entries: at most m / 1024 of them
    const uint64_t maxrows = (uint64_t)m / 1024;
    gc.all_taken = maxrows <= gc.cap;
    const size_t nck = (size_t)(m / kGroupChunkEntries) + std::min<uint64_t>(gc.cap, maxrows) + 1;
    gc.max_chunks = (uint32_t)std::min<size_t>(nck, 0xFFFFFFFFu);
    const size_t o_cnt = align16(8 * nck + 16), bytes = o_cnt + 4 * (size_t)gc.cap * (size_t)p;
    HIP_TRY(ensure_pow2(pl->grp, bytes), "alloc in-row chunks");
    gc.chunks = (uint2*)pl->grp.ptr;
    gc.nchunks = (uint32_t*)(pl->grp.ptr + 8 * nck);
    gc.cnt = (uint32_t*)(pl->grp.ptr + o_cnt);
    gc.rowmap = pl->od.ptr;  // free once the in-row sort has used it as a row list
    HIP_TRY(hipMemsetAsync(gc.nchunks, 0, 16, si), "memset");  // k_gchunk_list clears the counters it uses
  }
  HIP_TRY(launch_inrows_group(pl->irow.ptr, pl->icol.ptr, pl->idg.ptr, (const uint32_t*)pl->keys_a.ptr,
                              pl->err.ptr + 5, pl->acol.ptr, pl->cuts.ptr, p, gc, si),
          "group in-rows");
  HIP_TRY(hipEventSynchronize(pl->ev_cuts), "sync");
  pl->h_cuts.assign((const int32_t*)pl->cstage.ptr, (const int32_t*)pl->cstage.ptr + p + 1);
  pl->rT = choose_rT(opt, nshort, pl->h_cuts, p, m, false);

  // ---- block row index (out side, on s after the out-row sort) and the
  // block-major in side (on side[2] after the in-row grouping) ----
  const int64_t nb = (int64_t)p * (p + 1) / 2;
  std::vector<int32_t> chunk0((size_t)p + 1);
  std::vector<uint64_t> ccbase((size_t)p + 1), botp((size_t)p + 1);
  int64_t nch = 0;
  uint64_t cc = 0, bp = 0;
  for (int32_t a = 0; a < p; ++a) {
    const int64_t va = pl->h_cuts[a + 1] - pl->h_cuts[a];
    const int64_t ca = (va + kPrepRows - 1) / kPrepRows;
    // stored rows of part a: max(c_a, rT) .. c_{a+1}-1
    const int64_t sa = std::max<int64_t>(0, pl->h_cuts[a + 1] - std::max<int64_t>(pl->h_cuts[a], pl->rT));
    chunk0[a] = (int32_t)nch;
    ccbase[a] = cc;
    botp[a] = bp;
    nch += ca;
    cc += (uint64_t)(a + 1) * (uint64_t)ca;
    bp += (uint64_t)(p - a + 1) * (uint64_t)sa;
  }
  chunk0[p] = (int32_t)nch;
  ccbase[p] = cc;
  botp[p] = bp;
  pl->ccount = (int64_t)cc;
  const size_t w8 = sizeof(uint64_t) * (size_t)(p + 1), wb = sizeof(unsigned long long) * (size_t)nb;
  const size_t o_cb = align16(sizeof(int32_t) * (size_t)(p + 1)), o_hd = align16(o_cb + 2 * w8);
  HIP_TRY(pl->blk.ensure(o_hd + 16 + 3 * wb), "alloc");
  pl->chunk0 = (int32_t*)pl->blk.ptr;
  pl->ccbase = (uint64_t*)(pl->blk.ptr + o_cb);
  pl->botp = pl->ccbase + (p + 1);
  pl->head = (uint32_t*)(pl->blk.ptr + o_hd);
  pl->bnnz = (unsigned long long*)(pl->blk.ptr + o_hd + 16);
  pl->bnzr = pl->bnnz + nb;
  pl->bnzc = pl->bnzr + nb;
  HIP_TRY(pl->bot.ensure((size_t)bp), "alloc block row index");
  HIP_TRY(pl->ccnt.ensure(2 * ((size_t)cc + 1)), "alloc");   // column counts, then entry counts
  HIP_TRY(pl->ccoff.ensure(2 * ((size_t)cc + 1)), "alloc");  // their scans
  HIP_TRY(pl->aoff.ensure((size_t)m + 1), "alloc in-slice offsets");
  HIP_TRY(pl->asrc.ensure((size_t)m), "alloc");
  HIP_TRY(pl->icolb.ensure((size_t)m), "alloc block-major in side");
  uint32_t* ecnt = pl->ccnt.ptr + cc + 1;
  uint32_t* ecoff = pl->ccoff.ptr + cc + 1;
  if (pl->partial.cap < scan_partial_entries(cc)) HIP_TRY(pl->partial.ensure(scan_partial_entries(cc) + 4096), "alloc");
  {  // the index tables through the pinned stage, one copy (the D2H below is ordered after it on s;
     // the stage is sized for that D2H too, so it is not reallocated under this copy)
    HIP_TRY(pl->stage.ensure(std::max(o_hd, 16 + 3 * wb)), "pinned alloc");
    char* st = pl->stage.ptr;
    std::memcpy(st, chunk0.data(), sizeof(int32_t) * (p + 1));
    std::memcpy(st + o_cb, ccbase.data(), w8);
    std::memcpy(st + o_cb + w8, botp.data(), w8);
    HIP_TRY(hipMemcpyAsync(pl->blk.ptr, st, o_hd, hipMemcpyHostToDevice, s), "H2D");
  }
  HIP_TRY(hipMemsetAsync(pl->head, 0, 16 + 3 * wb, s), "memset");  // counters and block statistics
  BlockBuild bb;
  std::memset(&bb, 0, sizeof(bb));
  bb.p = p;
  bb.rT = (int32_t)pl->rT;
  bb.nchunks = (int32_t)nch;
  bb.chunk_base = 0;
  bb.cuts = pl->cuts.ptr;
  bb.chunk0 = pl->chunk0;
  bb.ccbase = pl->ccbase;
  bb.orow = pl->orow.ptr;
  bb.ocol = pl->ocol.ptr;
  bb.botp = pl->botp;
  bb.bot = pl->bot.ptr;
  bb.irow = pl->irow.ptr;
  bb.icol = pl->icol.ptr;
  bb.bnnz = pl->bnnz;
  bb.bnzr = pl->bnzr;
  bb.bnzc = pl->bnzc;
  bb.ccnt = pl->ccnt.ptr;
  bb.ecnt = ecnt;
  bb.dmax_block = pl->head + 1;
  bb.ccoff = pl->ccoff.ptr;
  bb.ecoff = ecoff;
  bb.acol = pl->acol.ptr;
  bb.aoff = pl->aoff.ptr;
  bb.asrc = pl->asrc.ptr;
  bb.ebase = 0;
  bb.xbase = 0;
  pl->split = kHubSplit;
  const uint64_t hcap = m / kHubSplit + 1;
  HIP_TRY(pl->heavy.ensure((size_t)hcap), "alloc");
  bb.split = pl->split;
  bb.heavy = pl->heavy.ptr;
  bb.nheavy = pl->head;
  bb.heavy_cap = (uint32_t)hcap;
  // the slices of the in-rows grouped in chunks come from their part counters
  bb.rowmap = gc.rowmap;
  bb.gcnt = gc.cnt;
  bb.glong = pl->idg.ptr;
  bb.ghuge = (const uint32_t*)pl->keys_a.ptr;
  bb.gq = pl->err.ptr + 5;
  bb.gcap = gc.cap;
  // block boundaries on s; the active-column counts, then the 16-bit
  // out-rows on side[2] meanwhile
  HIP_TRY(pl->ocol16.ensure((size_t)((m + 7) / 8 * 8 + 8)), "alloc 16-bit out-rows");
  HIP_TRY(hipEventRecord(pl->ev_fork, s), "event");
  HIP_TRY(hipStreamWaitEvent(si, pl->ev_fork, 0), "wait");
  HIP_TRY(launch_acount(bb, (int)nch, si), "active-column counts");
  HIP_TRY(launch_ocol16(pl->ocol.ptr, m, pl->cuts.ptr, p, pl->ocol16.ptr, si), "16-bit out-rows");
  HIP_TRY(launch_bot(bb, (int)nch, s), "block row index");
  HIP_TRY(hipEventRecord(pl->ev_join[2], si), "event");
  HIP_TRY(hipStreamWaitEvent(s, pl->ev_join[2], 0), "wait");
  HIP_TRY(scan_u32(pl->ccnt.ptr, pl->ccoff.ptr, cc, pl->partial.ptr, s), "scan column counters");
  HIP_TRY(scan_u32(ecnt, ecoff, cc, pl->partial.ptr, s), "scan entry counters");
  HIP_TRY(launch_acol(bb, (int)nch, s), "active columns");
  // aoff[number of active columns] = m closes the last slice; then the slices
  HIP_TRY(launch_set_at(pl->aoff.ptr, pl->ccoff.ptr + cc, (uint32_t)m, s), "in-slice sentinel");
  HIP_TRY(launch_icolb(pl->aoff.ptr, pl->asrc.ptr, pl->icol.ptr, pl->icolb.ptr, pl->ccoff.ptr + cc, (uint64_t)m,
                       pl->split, pl->heavy.ptr, 0, pl->head, (uint32_t)hcap, 0, s),
          "block-major in side");
  return finish_partition(pl, s, m, wedges, hcap, false, t0);
}

// State of multi-plan launches: device copies of the plan contexts (each
// pointing at its plan's own device work items) and of their item offsets in
// the combined index space, filled from pinned host staging.  A ring of slots
// lets several shared launches be in flight at once (on different streams); a
// slot is reused only after the launch that last used it has finished.
struct MultiSlot {
  DevBuf<char> dev;  // PlanCtx[nplans], then uint32_t plan_off[nplans]
  DevBuf<uint32_t> cursor;
  char* h = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};
constexpr int kMultiSlots = 8;
struct MultiState {
  std::mutex mu;
  MultiSlot slot[kMultiSlots];
  int next = 0;
};
MultiState g_multi;

bbtc_status count_multi_impl(bbtc_plan* const* plans, int32_t nplans, hipStream_t s, uint64_t* const* d_per_task,
                             uint64_t* d_totals) {
  MultiState& M = g_multi;
  std::lock_guard<std::mutex> lock(M.mu);
  MultiSlot& S = M.slot[M.next];
  M.next = (M.next + 1) % kMultiSlots;
  if (!S.done) HIP_TRY(hipEventCreateWithFlags(&S.done, hipEventDisableTiming), "hipEventCreate");
  if (S.used) HIP_TRY(hipEventSynchronize(S.done), "event sync");  // staging and buffers are free again
  size_t nitems = 0;
  for (int32_t q = 0; q < nplans; ++q) nitems += plans[q]->nitems;
  if (nitems > 0xFFFFFFFFull) return fail(BBTC_EINVAL, "too many work items for one shared launch");
  const size_t wc = align16(sizeof(PlanCtx) * (size_t)nplans), wbytes = wc + sizeof(uint32_t) * (size_t)nplans;
  if (S.cap < wbytes) {
    if (S.h) (void)hipHostFree(S.h);
    S.h = nullptr;
    S.cap = 0;
    HIP_TRY(hipHostMalloc((void**)&S.h, wbytes, hipHostMallocDefault), "pinned alloc");
    S.cap = wbytes;
  }
  // heavier plans first (sum of task estimates), each plan's items in its own order
  std::vector<std::pair<double, int32_t>> order;
  for (int32_t q = 0; q < nplans; ++q) {
    double w = 0;
    for (const auto& t : plans[q]->h_tasks) w += t.est;
    order.push_back({-w, q});
  }
  std::stable_sort(order.begin(), order.end());
  PlanCtx* hc = (PlanCtx*)S.h;
  uint32_t* ho = (uint32_t*)(S.h + wc);
  uint32_t at = 0;
  for (int32_t r = 0; r < nplans; ++r) {
    const int32_t q = order[r].second;
    hc[r] = plan_ctx(plans[q], d_per_task[q], d_totals + q);
    ho[r] = at;
    at += (uint32_t)plans[q]->nitems;
  }
  HIP_TRY(S.dev.ensure(wbytes), "alloc");
  HIP_TRY(S.cursor.ensure(kMaxQueues), "alloc");
  HIP_TRY(hipMemcpyAsync(S.dev.ptr, S.h, wbytes, hipMemcpyHostToDevice, s), "H2D");
  const PlanCtx* d_ctx = (const PlanCtx*)S.dev.ptr;
  HIP_TRY(launch_reset_multi(d_ctx, nplans, S.cursor.ptr, s), "reset");
  if (nitems) {
    CountParams cp;
    std::memset(&cp, 0, sizeof(cp));
    cp.many = d_ctx;
    cp.plan_off = (const uint32_t*)(S.dev.ptr + wc);
    cp.nplans = nplans;
    cp.items = nullptr;
    cp.nitems = (uint32_t)nitems;
    cp.cursor = S.cursor.ptr;
    one_queue(cp);
    const int ncu = plans[0]->ncu, bpc = plans[0]->blocks_per_cu;
    int grid = (int)std::min<int64_t>((int64_t)bpc * ncu, (int64_t)nitems);
    HIP_TRY(launch_count_persistent(cp, grid, true, s), "count");
  }
  HIP_TRY(hipEventRecord(S.done, s), "event");
  S.used = true;
  return BBTC_OK;
}

// ------------------------------------------------------------ hybrid execution
// Sec. 5 (Alg. 5-7): the tasks are in non-increasing order of their estimate;
// the GPU takes heavy tasks from the front, host threads light ones from the
// back, towards each other, and the host threads never go below the cut-off.
// Here the GPU's share is counted by the persistent kernel over contiguous
// task ranges (plan-order items are contiguous per task): first the tasks
// below the cut-off, then, in competition with the host threads, half of
// what is left at a time.  The host threads claim one task at a time from the
// back and count it with the Intersect form (cpu_count_task) over host
// copies of the plan's tables.  The host threads' tasks form the tail
// [back, |T|); their counts are copied into the per-task output at the end.
bbtc_status hybrid_prepare(bbtc_plan* pl, hipStream_t s) {
  auto& h = pl->hy;
  if (h.ready) return BBTC_OK;
  const int64_t n = pl->n, m = pl->m, p = pl->p, nb = p * (p + 1) / 2, nt = (int64_t)pl->h_tasks.size();
  if (!pl->plan_order_items) {
    compose_plan_order(pl);
    HIP_TRY(pl->items.ensure(pl->nitems), "alloc items");
    if (pl->nitems)
      HIP_TRY(hipMemcpyAsync(pl->items.ptr, pl->h_items.data(), sizeof(DevItem) * pl->nitems, hipMemcpyHostToDevice, s),
              "H2D");
    pl->plan_order_items = true;
  }
  h.istart.assign((size_t)nt + 1, 0);
  for (int64_t q = 0; q < nt; ++q)
    h.istart[q + 1] = h.istart[q] + (pl->h_tasks[q].kind == BBTC_TASK_WORK ? (int64_t)pl->h_nitem[q] : 0);
  h.botp.resize(p + 1);
  h.acp.resize(nb + 1);
  h.orow.resize(n + 1);
  HIP_TRY(hipMemcpyAsync(h.botp.data(), pl->botp, 8 * (p + 1), hipMemcpyDeviceToHost, s), "D2H");
  HIP_TRY(hipMemcpyAsync(h.acp.data(), pl->acp.ptr, 8 * (nb + 1), hipMemcpyDeviceToHost, s), "D2H");
  HIP_TRY(hipMemcpyAsync(h.orow.data(), pl->orow.ptr, 4 * (n + 1), hipMemcpyDeviceToHost, s), "D2H");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  h.ocol.resize(m + 1);
  h.icolb.resize(m + 1);
  h.bot.resize(h.botp[p] + 1);
  h.acol.resize(h.acp[nb] + 1);
  h.aoff.resize(h.acp[nb] + 1);
  HIP_TRY(hipMemcpyAsync(h.ocol.data(), pl->ocol.ptr, 4 * m, hipMemcpyDeviceToHost, s), "D2H");
  HIP_TRY(hipMemcpyAsync(h.icolb.data(), pl->icolb.ptr, 4 * m, hipMemcpyDeviceToHost, s), "D2H");
  HIP_TRY(hipMemcpyAsync(h.bot.data(), pl->bot.ptr, 4 * h.botp[p], hipMemcpyDeviceToHost, s), "D2H");
  HIP_TRY(hipMemcpyAsync(h.acol.data(), pl->acol.ptr, 4 * h.acp[nb], hipMemcpyDeviceToHost, s), "D2H");
  HIP_TRY(hipMemcpyAsync(h.aoff.data(), pl->aoff.ptr, 4 * (h.acp[nb] + 1), hipMemcpyDeviceToHost, s), "D2H");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  h.t = HostTables{(int32_t)p, (int32_t)pl->rT, pl->h_cuts.data(), h.orow.data(), h.ocol.data(), h.botp.data(),
                   h.bot.data(), h.acp.data(), h.acol.data(), h.aoff.data(), h.icolb.data()};
  h.ready = true;
  return BBTC_OK;
}

bbtc_status count_hybrid_impl(bbtc_plan* pl, hipStream_t s, uint64_t* d_per_task, uint64_t* d_total,
                              int32_t nthreads, int64_t cutoff, bbtc_hybrid_stats* out) {
  const auto t0 = std::chrono::steady_clock::now();
  bbtc_status st = hybrid_prepare(pl, s);
  if (st != BBTC_OK) return st;
  const auto& h = pl->hy;
  const int64_t nt = (int64_t)pl->h_tasks.size();
  if (cutoff < 0) cutoff = nt / 2;
  cutoff = std::min<int64_t>(cutoff, nt);
  if (nthreads <= 0)
    nthreads = (int32_t)std::max(1u, std::min(kHybridMaxThreads, std::thread::hardware_concurrency() - 1));
  HIP_TRY(launch_reset(d_per_task, nt, d_total, pl->cursor.ptr, s), "reset");
  const int grid_max = pl->blocks_per_cu * pl->ncu;
  int64_t launches = 0;
  // one persistent launch over the items of tasks [a, b) (plan order)
  auto gpu_range = [&](int64_t a, int64_t b) -> bbtc_status {
    const int64_t i0 = h.istart[a], i1 = h.istart[b];
    if (i1 <= i0) return BBTC_OK;
    CountParams cp;
    std::memset(&cp, 0, sizeof(cp));
    cp.one = plan_ctx(pl, d_per_task, d_total);
    cp.one.items = pl->items.ptr;
    cp.items = pl->items.ptr + i0;
    cp.nitems = (uint32_t)(i1 - i0);
    cp.cursor = pl->cursor.ptr;
    one_queue(cp);
    HIP_TRY(launch_reset(nullptr, 0, nullptr, pl->cursor.ptr, s), "cursor");
    HIP_TRY(launch_count_persistent(cp, (int)std::min<int64_t>(grid_max, cp.nitems), false, s), "count");
    ++launches;
    return BBTC_OK;
  };
  std::mutex mu;
  int64_t front = cutoff, back = nt;  // GPU claims [front, ...), host threads back-1, back-2, ...
  std::vector<uint64_t> cpu_per((size_t)nt, 0);
  std::vector<double> busy((size_t)nthreads, 0.0);
  std::vector<int64_t> done((size_t)nthreads, 0);
  int32_t started = 0;  // host threads that have made their first claim
  std::condition_variable all_started;
  auto worker = [&](int w) {
    const auto b0 = std::chrono::steady_clock::now();
    for (bool first = true;; first = false) {
      int64_t t;
      {
        std::lock_guard<std::mutex> lock(mu);
        if (first && ++started == nthreads) all_started.notify_one();
        if (back <= front || back <= cutoff) break;
        t = --back;
      }
      const bbtc_task& tk = pl->h_tasks[t];
      if (tk.kind != BBTC_TASK_WORK) continue;
      cpu_per[t] = cpu_count_task(h.t, tk.i, tk.j, tk.k);
      done[w]++;
    }
    busy[w] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - b0).count();
  };
  // the tasks below the cut-off go to the GPU at once; the host threads start
  // from the back meanwhile
  if ((st = gpu_range(0, cutoff)) != BBTC_OK) return st;
  std::vector<std::thread> th;
  try {
    for (int w = 0; w < nthreads; ++w) th.emplace_back(worker, w);
  } catch (const std::exception&) {  // no thread could be started: stop the ones that were
    {
      std::lock_guard<std::mutex> lock(mu);
      front = back;
    }
    for (auto& x : th) x.join();
    (void)hipStreamSynchronize(s);
    return fail(BBTC_ENOMEM, "could not start the host threads");
  }
  hipError_t herr = hipSuccess;
  for (bool first = true;; first = false) {
    herr = hipStreamSynchronize(s);
    if (herr != hipSuccess) break;
    int64_t a, b;
    {
      std::unique_lock<std::mutex> lock(mu);
      // the GPU competes for the tasks past the cut-off only once every host
      // thread has made its first claim (a thread that starts late would
      // otherwise find the list taken on small plans)
      if (first) all_started.wait(lock, [&] { return started == nthreads; });
      if (front >= back) break;
      a = front;
      b = front + std::max<int64_t>(1, (back - front) / 2);
      front = b;
    }
    if ((st = gpu_range(a, b)) != BBTC_OK) break;
  }
  if (herr == hipSuccess && st == BBTC_OK) herr = hipStreamSynchronize(s);
  {  // no new claims; the host threads finish their current task
    std::lock_guard<std::mutex> lock(mu);
    front = std::max(front, back);
  }
  for (auto& x : th) x.join();
  if (herr != hipSuccess) return hip_fail(herr, "hybrid count");
  if (st != BBTC_OK) return st;
  // the host threads' tasks are the tail [back, nt): their counts into the
  // per-task output, their sum onto the total
  uint64_t cpu_sum = 0;
  for (int64_t t = back; t < nt; ++t) cpu_sum += cpu_per[t];
  if (back < nt) {
    HIP_TRY(hipMemcpyAsync(d_per_task + back, cpu_per.data() + back, sizeof(uint64_t) * (size_t)(nt - back),
                           hipMemcpyHostToDevice, s),
            "H2D");
    HIP_TRY(launch_add_u64(d_total, cpu_sum, s), "add host counts");
  }
  HIP_TRY(hipStreamSynchronize(s), "sync");
  if (out) {
    std::memset(out, 0, sizeof(*out));
    for (int64_t t = 0; t < nt; ++t)
      if (pl->h_tasks[t].kind == BBTC_TASK_WORK) (t < back ? out->gpu_tasks : out->cpu_tasks)++;
    out->gpu_launches = launches;
    out->cpu_threads = nthreads;
    out->cutoff = cutoff;
    out->split = back;
    for (double b : busy) out->cpu_ms = std::max(out->cpu_ms, b);
    out->cpu_triangles = cpu_sum;
    out->total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return BBTC_OK;
}

// ---- shared launches without allocation (bbtc_count_multi_static)
// The launch state lives in `scratch`, a fixed device array of this file:
// PlanCtx[kStaticPlans] | uint32 plan_off[kStaticPlans] | uint32
// cursor[kMaxQueues].  Host code uses the device address obtained once per
// device by hipGetSymbolAddress, never the array's name; the contexts are
// written into it by a kernel that takes them as arguments (no host staging,
// no copy engine), so a call is only kernel launches.
constexpr int kStaticPlans = BBTC_STATIC_MAX_PLANS;
constexpr size_t kStaticCtxBytes = sizeof(PlanCtx) * kStaticPlans;
constexpr size_t kStaticOffBytes = sizeof(uint32_t) * kStaticPlans;
static_assert(kStaticCtxBytes % 16 == 0, "cursor alignment");
static_assert(kStaticCtxBytes + kStaticOffBytes + sizeof(uint32_t) * kMaxQueues <= BBTC_STATIC_BYTES,
              "static launch state exceeds its array");

static __device__ __align__(256) char scratch[BBTC_STATIC_BYTES];

constexpr int kMaxDevices = 64;
struct StaticState {
  std::mutex mu;
  char* ptr[kMaxDevices] = {};  // device address of `scratch` on each device
};
StaticState g_static;

// The device address of this device's `scratch`, looked up on the first call
// made with the device current.
bbtc_status static_scratch(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(BBTC_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_static.mu);
  if (!g_static.ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (!p) return fail(BBTC_EDEVICE, "no device address for the static launch state");
    g_static.ptr[dev] = (char*)p;
  }
  *out = g_static.ptr[dev];
  return BBTC_OK;
}

constexpr int kCtxBatch = 8;  // contexts per fill launch (kernel arguments stay well under 4 KB)
struct CtxBatch {
  PlanCtx ctx[kCtxBatch];
  uint32_t off[kCtxBatch];
  int32_t first, count;
};

// Writes contexts [first, first+count) and their item offsets.
__global__ __launch_bounds__(kThreads) void k_put_ctx(PlanCtx* __restrict__ ctxs, uint32_t* __restrict__ offs,
                                                      CtxBatch b) {
  constexpr int kWords = (int)(sizeof(PlanCtx) / 4);
  static_assert(sizeof(PlanCtx) % 4 == 0, "word copy");
  for (int t = threadIdx.x; t < b.count * kWords; t += kThreads) {
    const int q = t / kWords, w = t % kWords;
    reinterpret_cast<uint32_t*>(ctxs + b.first + q)[w] = reinterpret_cast<const uint32_t*>(&b.ctx[q])[w];
  }
  if (threadIdx.x < (unsigned)b.count) offs[b.first + threadIdx.x] = b.off[threadIdx.x];
}

bbtc_status count_multi_static_impl(bbtc_plan* const* plans, int32_t nplans, hipStream_t s,
                                    uint64_t* const* d_per_task, uint64_t* d_totals) {
  char* base = nullptr;
  bbtc_status st = static_scratch(&base);
  if (st != BBTC_OK) return st;
  PlanCtx* d_ctx = (PlanCtx*)base;
  uint32_t* d_off = (uint32_t*)(base + kStaticCtxBytes);
  uint32_t* d_cursor = (uint32_t*)(base + kStaticCtxBytes + kStaticOffBytes);
  // heavier plans first (sum of task estimates), as bbtc_count_multi
  int32_t order[kStaticPlans];
  for (int32_t q = 0; q < nplans; ++q) {
    int32_t r = q;
    while (r > 0 && plans[order[r - 1]]->est_sum < plans[q]->est_sum) {
      order[r] = order[r - 1];
      --r;
    }
    order[r] = q;
  }
  uint64_t nitems = 0;
  CtxBatch b;
  for (int32_t r0 = 0; r0 < nplans; r0 += kCtxBatch) {
    std::memset(&b, 0, sizeof(b));
    b.first = r0;
    b.count = std::min(kCtxBatch, nplans - r0);
    for (int32_t t = 0; t < b.count; ++t) {
      const int32_t q = order[r0 + t];
      b.ctx[t] = plan_ctx(plans[q], d_per_task[q], d_totals + q);
      b.off[t] = (uint32_t)nitems;
      nitems += plans[q]->nitems;
    }
    if (nitems > 0xFFFFFFFFull) return fail(BBTC_EINVAL, "too many work items for one shared launch");
    hipLaunchKernelGGL(k_put_ctx, dim3(1), dim3(kThreads), 0, s, d_ctx, d_off, b);
    HIP_TRY(hipGetLastError(), "fill launch state");
  }
  HIP_TRY(launch_reset_multi(d_ctx, nplans, d_cursor, s), "reset");
  if (nitems) {
    CountParams cp;
    std::memset(&cp, 0, sizeof(cp));
    cp.many = d_ctx;
    cp.plan_off = d_off;
    cp.nplans = nplans;
    cp.items = nullptr;
    cp.nitems = (uint32_t)nitems;
    cp.cursor = d_cursor;
    one_queue(cp);
    const int grid = (int)std::min<int64_t>((int64_t)plans[0]->blocks_per_cu * plans[0]->ncu, (int64_t)nitems);
    HIP_TRY(launch_count_persistent(cp, grid, true, s), "count");
  }
  return BBTC_OK;
}

}  // namespace

extern "C" {

void bbtc_options_default(bbtc_options* opt) {
  if (opt) fill_defaults(opt);
}

bbtc_status bbtc_partition(const bbtc_csr* g, const bbtc_options* opt, void* stream, bbtc_plan** plan) {
  g_err.clear();
  if (!g || !plan) return fail(BBTC_EINVAL, "null argument");
  try {
    bbtc_plan* pl = *plan;
    bool fresh = false;
    if (!pl) {
      pl = new bbtc_plan();
      fresh = true;
    }
    bbtc_status st = partition_impl(g, opt, (hipStream_t)stream, pl);
    if (st != BBTC_OK) {
      if (fresh) delete pl;
      else pl->ready = false;
      return st;
    }
    *plan = pl;
    return BBTC_OK;
  } catch (const std::bad_alloc&) {
    return fail(BBTC_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(BBTC_EDEVICE, "unexpected exception");
  }
}

bbtc_status bbtc_count(bbtc_plan* pl, void* stream, uint64_t* d_per_task, uint64_t* d_total) {
  g_err.clear();
  if (!pl || !pl->ready) return fail(BBTC_ESTATE, "plan is not ready");
  if (!d_total || (!d_per_task && !pl->h_tasks.empty())) return fail(BBTC_EINVAL, "null output");
  hipStream_t s = (hipStream_t)stream;
  if (pl->streamed) return count_streamed(pl, s, d_per_task, d_total);
  const int64_t nt = (int64_t)pl->h_tasks.size();
  const bool graphed = pl->opt.mode == BBTC_MODE_PERSISTENT && pl->opt.graph == 0 && pl->nitems > 0;
  if (!graphed) HIP_TRY(launch_reset(d_per_task, nt, d_total, pl->cursor.ptr, s), "reset");
  CountParams cp;
  cp.one = plan_ctx(pl, d_per_task, d_total);
  cp.many = nullptr;
  cp.items = pl->items.ptr;
  cp.nitems = (uint32_t)pl->nitems;
  cp.cursor = pl->cursor.ptr;
  one_queue(cp);
  if (pl->opt.mode == BBTC_MODE_PERSISTENT) {
    if (cp.nitems == 0) return BBTC_OK;
    cp.items = pl->xitems.ptr;
    cp.nq = pl->nq;
    for (int x = 0; x < kMaxQueues; ++x) {
      cp.qbeg[x] = pl->qbeg[x];
      cp.qlen[x] = pl->qlen[x];
    }
    int grid = pl->opt.grid > 0 ? pl->opt.grid : pl->blocks_per_cu * pl->ncu;
    grid = (int)std::min<int64_t>(grid, (int64_t)cp.nitems);
    const bool have_graph = pl->gexec && pl->g_per == d_per_task && pl->g_tot == d_total;
    const bool repeat = pl->d_per == d_per_task && pl->d_tot == d_total;
    if (pl->opt.graph == -1 || (!have_graph && !repeat)) {
      // first count of this plan into these outputs: launching beats capturing
      if (graphed) HIP_TRY(launch_reset(d_per_task, nt, d_total, pl->cursor.ptr, s), "reset");
      HIP_TRY(launch_count_persistent(cp, grid, false, s), "count");
      pl->d_per = d_per_task;
      pl->d_tot = d_total;
      return BBTC_OK;
    }
    if (!have_graph) {
      // capture {reset kernel, persistent count} on a plan-owned stream
      pl->drop_graph();
      hipStream_t cs = pl->side[0];
      HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
      hipError_t e1 = launch_reset(d_per_task, nt, d_total, pl->cursor.ptr, cs);
      hipError_t e2 = e1 == hipSuccess ? launch_count_persistent(cp, grid, false, cs) : e1;
      hipGraph_t gr = nullptr;
      hipError_t e3 = hipStreamEndCapture(cs, &gr);
      if (e2 != hipSuccess || e3 != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return hip_fail(e2 != hipSuccess ? e2 : e3, "capture count");
      }
      pl->graph = gr;
      HIP_TRY(hipGraphInstantiate(&pl->gexec, pl->graph, nullptr, nullptr, 0), "instantiate graph");
      pl->g_per = d_per_task;
      pl->g_tot = d_total;
    }
    HIP_TRY(hipGraphLaunch(pl->gexec, s), "graph launch");
    return BBTC_OK;
  }
  // plain: one launch per task, round-robin over four side streams
  HIP_TRY(hipEventRecord(pl->ev_fork, s), "event");
  for (int q = 0; q < 4; ++q) HIP_TRY(hipStreamWaitEvent(pl->side[q], pl->ev_fork, 0), "wait");
  for (size_t w = 0; w < pl->h_work.size(); ++w) {
    const int32_t t = pl->h_work[w];
    HIP_TRY(launch_count_items(cp, (uint32_t)pl->h_hub_first[t], (uint32_t)pl->h_hub_count[t], pl->side[w % 4]),
            "count task");
  }
  for (int q = 0; q < 4; ++q) {
    HIP_TRY(hipEventRecord(pl->ev_join[q], pl->side[q]), "event");
    HIP_TRY(hipStreamWaitEvent(s, pl->ev_join[q], 0), "wait");
  }
  return BBTC_OK;
}

bbtc_status bbtc_count_multi(bbtc_plan* const* plans, int32_t nplans, void* stream, uint64_t* const* d_per_task,
                             uint64_t* d_totals) {
  g_err.clear();
  if (nplans < 0 || (nplans > 0 && (!plans || !d_per_task || !d_totals))) return fail(BBTC_EINVAL, "null argument");
  if (nplans == 0) return BBTC_OK;
  for (int32_t q = 0; q < nplans; ++q) {
    if (!plans[q] || !plans[q]->ready) return fail(BBTC_ESTATE, "plan is not ready");
    if (plans[q]->streamed) return fail(BBTC_ESTATE, "a streamed (over-budget) plan cannot join a shared launch");
    if (!d_per_task[q]) return fail(BBTC_EINVAL, "null output");
  }
  try {
    return count_multi_impl(plans, nplans, (hipStream_t)stream, d_per_task, d_totals);
  } catch (const std::bad_alloc&) {
    return fail(BBTC_ENOMEM, "host allocation failed");
  }
}

bbtc_status bbtc_count_multi_static(bbtc_plan* const* plans, int32_t nplans, void* stream,
                                    uint64_t* const* d_per_task, uint64_t* d_totals) {
  g_err.clear();
  if (nplans < 0 || (nplans > 0 && (!plans || !d_per_task || !d_totals))) return fail(BBTC_EINVAL, "null argument");
  if (nplans > BBTC_STATIC_MAX_PLANS)
    return fail(BBTC_EINVAL, "more plans than the static launch state holds (BBTC_STATIC_MAX_PLANS)");
  if (nplans == 0) return BBTC_OK;
  for (int32_t q = 0; q < nplans; ++q) {
    if (!plans[q] || !plans[q]->ready) return fail(BBTC_ESTATE, "plan is not ready");
    if (plans[q]->streamed) return fail(BBTC_ESTATE, "a streamed (over-budget) plan cannot join a shared launch");
    if (!d_per_task[q]) return fail(BBTC_EINVAL, "null output");
  }
  return count_multi_static_impl(plans, nplans, (hipStream_t)stream, d_per_task, d_totals);
}

bbtc_status bbtc_count_hybrid(bbtc_plan* pl, void* stream, uint64_t* d_per_task, uint64_t* d_total,
                              int32_t cpu_threads, int64_t cutoff, bbtc_hybrid_stats* stats) {
  g_err.clear();
  if (!pl || !pl->ready) return fail(BBTC_ESTATE, "plan is not ready");
  if (pl->streamed) return fail(BBTC_ESTATE, "a streamed (over-budget) plan is counted by bbtc_count only");
  if (!d_total || (!d_per_task && !pl->h_tasks.empty())) return fail(BBTC_EINVAL, "null output");
  if (cpu_threads < 0 || cpu_threads > 1024) return fail(BBTC_EINVAL, "cpu_threads must be in [0, 1024]");
  if (cutoff < -1 || cutoff > (int64_t)pl->h_tasks.size()) return fail(BBTC_EINVAL, "cutoff must be in [-1, |T|]");
  try {
    return count_hybrid_impl(pl, (hipStream_t)stream, d_per_task, d_total, cpu_threads, cutoff, stats);
  } catch (const std::bad_alloc&) {
    return fail(BBTC_ENOMEM, "host allocation failed");
  } catch (const std::system_error&) {
    return fail(BBTC_EDEVICE, "could not start host threads");
  }
}

bbtc_status bbtc_autotune(const bbtc_csr* g, const bbtc_options* base, int32_t reps, void* stream, bbtc_options* out,
                          double* best_ms) {
  g_err.clear();
  if (!g || !out) return fail(BBTC_EINVAL, "null argument");
  if (reps < 1 || reps > 100) return fail(BBTC_EINVAL, "reps must be in [1, 100]");
  hipStream_t s = (hipStream_t)stream;
  bbtc_options cur;
  if (base) cur = *base; else fill_defaults(&cur);
  cur.mode = BBTC_MODE_PERSISTENT;
  bbtc_plan* pl = nullptr;
  uint64_t* d_out = nullptr;
  size_t d_cap = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bbtc_status st = BBTC_OK;
  double best = 1e300;
  bbtc_options best_opt = cur;
  // time one candidate; returns the median count time in ms (or a status < 0)
  auto measure = [&](const bbtc_options& o, double* ms) -> bbtc_status {
    bbtc_status r = bbtc_partition(g, &o, stream, &pl);
    if (r != BBTC_OK) return r;
    const size_t need = pl->h_tasks.size() + 1;
    if (need > d_cap) {
      if (d_out) (void)hipFree(d_out);
      d_out = nullptr;
      HIP_TRY(hipMalloc((void**)&d_out, need * sizeof(uint64_t)), "alloc");
      d_cap = need;
    }
    uint64_t* tot = d_out + (need - 1);
    r = bbtc_count(pl, stream, d_out, tot);
    if (r != BBTC_OK) return r;
    std::vector<float> t;
    for (int q = 0; q < reps; ++q) {
      HIP_TRY(hipEventRecord(e0, s), "event");
      r = bbtc_count(pl, stream, d_out, tot);
      if (r != BBTC_OK) return r;
      HIP_TRY(hipEventRecord(e1, s), "event");
      HIP_TRY(hipEventSynchronize(e1), "event sync");
      float v = 0;
      HIP_TRY(hipEventElapsedTime(&v, e0, e1), "event time");
      t.push_back(v);
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return BBTC_OK;
  };
  try {
    HIP_TRY(hipEventCreate(&e0), "event");
    HIP_TRY(hipEventCreate(&e1), "event");
    // p0: requested, or from the average degree (needs n and nnz only)
    int32_t p0 = cur.p;
    if (p0 <= 0) {
      const double avg = g->n > 0 ? (double)g->nnz / (double)g->n : 1.0;
      p0 = std::max(1, (int32_t)std::lround(avg));
    }
    const int64_t pmax = std::min<int64_t>(g->n, kMaxP);
    std::vector<int32_t> ps;
    for (int32_t c : {p0 / 4, p0 / 2, p0, 2 * p0}) {
      int32_t q = (int32_t)std::max<int64_t>(1, std::min<int64_t>(c, pmax));
      if (std::find(ps.begin(), ps.end(), q) == ps.end()) ps.push_back(q);
    }
    for (int32_t q : ps) {
      bbtc_options o = cur;
      o.p = q;
      double ms = 0;
      st = measure(o, &ms);
      if (st != BBTC_OK) break;
      if (ms < best) { best = ms; best_opt = o; }
    }
    // past the ends of the candidates: halve (double) p while the count gets faster
    for (int dir = 0; dir < 2 && st == BBTC_OK; ++dir) {
      const int32_t edge = dir == 0 ? ps.front() : ps.back();
      if (best_opt.p != edge) continue;
      for (int32_t q = dir == 0 ? edge / 2 : 2 * edge; q >= 1 && q <= pmax; q = dir == 0 ? q / 2 : 2 * q) {
        bbtc_options o = cur;
        o.p = q;
        double ms = 0;
        st = measure(o, &ms);
        if (st != BBTC_OK || ms >= best) break;
        best = ms;
        best_opt = o;
      }
    }
    // the two thresholds move off their current value only for a gain above
    // the timing noise, so that repeated tunings of one graph agree
    for (int32_t wm : {16, 32, 64, 128, 256, 512}) {  // 512: the whole wavefront stage
      if (st != BBTC_OK) break;
      bbtc_options o = best_opt;
      o.wave_min = wm;
      double ms = 0;
      st = measure(o, &ms);
      if (st == BBTC_OK && ms < best * kTuneMargin) { best = ms; best_opt = o; }
    }
    for (int32_t hm : {-1, 1, 32, 256}) {
      if (st != BBTC_OK) break;
      bbtc_options o = best_opt;
      o.hash_min = hm;
      double ms = 0;
      st = measure(o, &ms);
      if (st == BBTC_OK && ms < best * kTuneMargin) { best = ms; best_opt = o; }
    }
  } catch (const std::bad_alloc&) {
    st = fail(BBTC_ENOMEM, "host allocation failed");
  }
  std::string msg = g_err;
  if (pl) bbtc_plan_destroy(pl);
  if (d_out) (void)hipFree(d_out);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != BBTC_OK) return fail(st, msg);
  *out = best_opt;
  if (best_ms) *best_ms = best;
  return BBTC_OK;
}

bbtc_status bbtc_check_tables(const bbtc_tables* t) {
  g_err.clear();
  if (!t || !t->cuts || !t->orow || !t->botp || !t->acp) return fail(BBTC_EINVAL, "null argument");
  if (t->n < 1 || t->n > 2147483647LL || t->p < 1 || t->p > kMaxP || t->m < 0) return fail(BBTC_EINVAL, "bad sizes");
  TableView v{t->n, t->m, t->p, t->rT, t->cuts, t->orow, t->ocol, t->botp, t->bot, t->acp, t->acol, t->aoff, t->icolb};
  try {
    const std::string msg = check_tables(v);
    if (!msg.empty()) return fail(BBTC_EINVAL, msg);
  } catch (const std::bad_alloc&) {
    return fail(BBTC_ENOMEM, "host allocation failed");
  }
  return BBTC_OK;
}

bbtc_status bbtc_plan_verify(const bbtc_plan* pl, void* stream) {
  g_err.clear();
  if (!pl || !pl->ready) return fail(BBTC_ESTATE, "plan is not ready");
  hipStream_t s = (hipStream_t)stream;
  try {
    const int64_t n = pl->n, m = pl->m, p = pl->p, nb = p * (p + 1) / 2;
    std::vector<uint32_t> orow(n + 1), bot, aoff;
    std::vector<int32_t> ocol(m + 1), icolb(m + 1), acol;
    std::vector<uint64_t> botp(p + 1), acp(nb + 1);
    HIP_TRY(hipMemcpyAsync(orow.data(), pl->orow.ptr, 4 * (n + 1), hipMemcpyDeviceToHost, s), "D2H");
    HIP_TRY(hipMemcpyAsync(botp.data(), pl->botp, 8 * (p + 1), hipMemcpyDeviceToHost, s), "D2H");
    HIP_TRY(hipMemcpyAsync(acp.data(), pl->acp.ptr, 8 * (nb + 1), hipMemcpyDeviceToHost, s), "D2H");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    bot.resize(botp[p] + 1);
    acol.resize(acp[nb] + 1);
    aoff.resize(acp[nb] + 1);
    if (pl->streamed) {
      std::memcpy(ocol.data(), pl->h_ocol, 4 * m);
      std::memcpy(icolb.data(), pl->h_icolb, 4 * m);
      std::memcpy(bot.data(), pl->h_bot, 4 * botp[p]);
      std::memcpy(acol.data(), pl->h_acol, 4 * acp[nb]);
      std::memcpy(aoff.data(), pl->h_aoff, 4 * (acp[nb] + 1));
    } else {
      HIP_TRY(hipMemcpyAsync(ocol.data(), pl->ocol.ptr, 4 * m, hipMemcpyDeviceToHost, s), "D2H");
      HIP_TRY(hipMemcpyAsync(icolb.data(), pl->icolb.ptr, 4 * m, hipMemcpyDeviceToHost, s), "D2H");
      HIP_TRY(hipMemcpyAsync(bot.data(), pl->bot.ptr, 4 * botp[p], hipMemcpyDeviceToHost, s), "D2H");
      HIP_TRY(hipMemcpyAsync(acol.data(), pl->acol.ptr, 4 * acp[nb], hipMemcpyDeviceToHost, s), "D2H");
      HIP_TRY(hipMemcpyAsync(aoff.data(), pl->aoff.ptr, 4 * (acp[nb] + 1), hipMemcpyDeviceToHost, s), "D2H");
    }
    // work items, in the layout the count launches read
    const bool queued = pl->opt.mode == BBTC_MODE_PERSISTENT && !pl->streamed;
    std::vector<DevItem> items(pl->nitems + 1);
    HIP_TRY(hipMemcpyAsync(items.data(), queued ? pl->xitems.ptr : pl->items.ptr, sizeof(DevItem) * pl->nitems,
                           hipMemcpyDeviceToHost, s),
            "D2H");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    TableView v{n, m, (int32_t)p, (int32_t)pl->rT, pl->h_cuts.data(), orow.data(), ocol.data(), botp.data(),
                bot.data(), acp.data(), acol.data(), aoff.data(), icolb.data()};
    std::string msg = check_tables(v);
    if (!msg.empty()) return fail(BBTC_EDEVICE, "plan tables: " + msg);
    // dense slices: a (row, block) pair of the region has a bitmap exactly
    // when its slice holds at least |V_k|/16 entries, and the bitmap holds
    // the slice's vertices and nothing else (padding included)
    if (!pl->streamed && pl->dense_k0 < p) {
      const int32_t k0 = pl->dense_k0;
      const int64_t u0 = pl->h_cuts[k0], nk = p - k0, npairs = (n - u0) * nk;
      std::vector<uint32_t> dslot((size_t)npairs), dbits((size_t)pl->dense_words + 1);
      HIP_TRY(hipMemcpyAsync(dslot.data(), pl->dslot.ptr, 4 * npairs, hipMemcpyDeviceToHost, s), "D2H");
      HIP_TRY(hipMemcpyAsync(dbits.data(), pl->dbits.ptr, 4 * pl->dense_words, hipMemcpyDeviceToHost, s), "D2H");
      HIP_TRY(hipStreamSynchronize(s), "sync");
      int64_t seen = 0;
      std::vector<uint32_t> want;
      for (int64_t u = u0; u < n; ++u)
        for (int32_t k = k0; k < p; ++k) {
          const int64_t ck = pl->h_cuts[k], ck1 = pl->h_cuts[k + 1];
          const int32_t* r0 = ocol.data() + orow[u];
          const int32_t* r1 = ocol.data() + orow[u + 1];
          const int32_t* a0 = std::lower_bound(r0, r1, (int32_t)ck);
          const int32_t* a1 = std::lower_bound(a0, r1, (int32_t)ck1);
          const uint64_t len = (uint64_t)(a1 - a0), vk = (uint64_t)(ck1 - ck);
          const uint32_t slot = dslot[(u - u0) * nk + (k - k0)];
          const bool dense = len > 0 && 16 * len >= vk;
          const std::string at = "dense slice of row " + std::to_string(u) + ", block " + std::to_string(k);
          if (dense != (slot != 0)) return fail(BBTC_EDEVICE, at + (dense ? " missing" : " not dense"));
          if (!slot) continue;
          const uint64_t words = ((vk + 31) / 32 + 7) & ~7ull;
          if (slot - 1 + words > (uint64_t)pl->dense_words) return fail(BBTC_EDEVICE, at + " past the bitmaps");
          want.assign(words, 0u);
          for (const int32_t* e = a0; e < a1; ++e) want[(uint32_t)(*e - ck) >> 5] |= 1u << ((uint32_t)(*e - ck) & 31);
          if (!std::equal(want.begin(), want.end(), dbits.begin() + (slot - 1)))
            return fail(BBTC_EDEVICE, at + ": bitmap differs from the slice");
          ++seen;
        }
      if (seen != pl->dense_slices) return fail(BBTC_EDEVICE, "dense slice count differs");
    }
    // every item within its task's active columns or hub in-slice; the
    // column items of a task cover its columns exactly once, hub columns
    // (in-slices longer than the split) excluded
    const int64_t nt = (int64_t)pl->h_tasks.size();
    std::vector<std::vector<std::pair<int64_t, int64_t>>> cover((size_t)nt);
    for (size_t q = 0; q < pl->nitems; ++q) {
      const DevItem& it = items[q];
      const std::string at = "work item " + std::to_string(q);
      if (it.task < 0 || it.task >= nt) return fail(BBTC_EDEVICE, at + ": bad task");
      const bbtc_task& tk = pl->h_tasks[it.task];
      if (tk.kind != BBTC_TASK_WORK) return fail(BBTC_EDEVICE, at + " of an empty task");
      const int64_t cid = col_block_id(tk.i, tk.j);
      if (it.lo >= it.hi) return fail(BBTC_EDEVICE, at + " is empty");
      if (it.v < 0) {
        if ((int64_t)it.hi > (int64_t)(acp[cid + 1] - acp[cid])) return fail(BBTC_EDEVICE, at + " past the active columns");
        cover[it.task].push_back({(int64_t)it.lo, (int64_t)it.hi});
      } else {
        const uint64_t x = (uint64_t)it.v;
        if (x < acp[cid] || x >= acp[cid + 1]) return fail(BBTC_EDEVICE, at + ": hub column outside block (i,j)");
        const uint32_t len = aoff[x + 1] - aoff[x];
        if (len <= pl->split || it.hi > len) return fail(BBTC_EDEVICE, at + ": not a hub or past its in-slice");
      }
    }
    for (int64_t q = 0; q < nt; ++q) {
      auto& c = cover[q];
      std::sort(c.begin(), c.end());
      int64_t next = 0;
      for (const auto& r : c) {
        if (r.first != next) return fail(BBTC_EDEVICE, "work items of task " + std::to_string(q) + " leave a gap");
        next = r.second;
      }
      const bbtc_task& tk = pl->h_tasks[q];
      if (tk.kind == BBTC_TASK_WORK) {
        const int64_t cid = col_block_id(tk.i, tk.j);
        if (next != (int64_t)(acp[cid + 1] - acp[cid]))
          return fail(BBTC_EDEVICE, "work items of task " + std::to_string(q) + " miss columns");
      }
    }
  } catch (const std::bad_alloc&) {
    return fail(BBTC_ENOMEM, "host allocation failed");
  }
  return BBTC_OK;
}

bbtc_status bbtc_plan_tasks(const bbtc_plan* pl, const bbtc_task** tasks, int64_t* ntasks) {
  if (!pl || !pl->ready) return fail(BBTC_ESTATE, "plan is not ready");
  if (!tasks || !ntasks) return fail(BBTC_EINVAL, "null argument");
  *tasks = pl->h_tasks.data();
  *ntasks = (int64_t)pl->h_tasks.size();
  return BBTC_OK;
}

bbtc_status bbtc_plan_cuts(const bbtc_plan* pl, const int32_t** cuts, int32_t* p) {
  if (!pl || !pl->ready) return fail(BBTC_ESTATE, "plan is not ready");
  if (!cuts || !p) return fail(BBTC_EINVAL, "null argument");
  *cuts = pl->h_cuts.data();
  *p = pl->p;
  return BBTC_OK;
}

bbtc_status bbtc_plan_block_nnz(const bbtc_plan* pl, const int64_t** nnz, int64_t* nblocks) {
  if (!pl || !pl->ready) return fail(BBTC_ESTATE, "plan is not ready");
  if (!nnz || !nblocks) return fail(BBTC_EINVAL, "null argument");
  *nnz = pl->h_nnz.data();
  *nblocks = (int64_t)pl->h_nnz.size();
  return BBTC_OK;
}

bbtc_status bbtc_plan_stats(const bbtc_plan* pl, bbtc_stats* out) {
  if (!pl || !pl->ready) return fail(BBTC_ESTATE, "plan is not ready");
  if (!out) return fail(BBTC_EINVAL, "null argument");
  *out = pl->stats;
  out->streamed = pl->streamed ? 1 : 0;
  out->stripe_slots = (int64_t)pl->slots.size();
  out->stripe_bytes = (int64_t)pl->slot_bytes;
  out->stripe_uploads = pl->copies;
  out->resident_bytes = pl->streamed ? pl->resident_bytes : pl->stats.footprint;
  return BBTC_OK;
}

bbtc_status bbtc_plan_copy_perm(const bbtc_plan* pl, int32_t* dst, void* stream) {
  if (!pl || !pl->ready) return fail(BBTC_ESTATE, "plan is not ready");
  if (!dst) return fail(BBTC_EINVAL, "null argument");
  HIP_TRY(hipMemcpyAsync(dst, pl->perm.ptr, sizeof(int32_t) * pl->n, hipMemcpyDefault, (hipStream_t)stream), "copy");
  return BBTC_OK;
}

bbtc_status bbtc_plan_copy_oriented(const bbtc_plan* pl, uint32_t* orow, int32_t* ocol, void* stream) {
  if (!pl || !pl->ready) return fail(BBTC_ESTATE, "plan is not ready");
  if (!orow || (pl->m > 0 && !ocol)) return fail(BBTC_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  const uint32_t* src_row = pl->streamed ? pl->h_orow : pl->orow.ptr;
  const int32_t* src_col = pl->streamed ? pl->h_ocol : pl->ocol.ptr;
  HIP_TRY(hipMemcpyAsync(orow, src_row, sizeof(uint32_t) * (pl->n + 1), hipMemcpyDefault, s), "copy");
  if (pl->m > 0) HIP_TRY(hipMemcpyAsync(ocol, src_col, sizeof(int32_t) * pl->m, hipMemcpyDefault, s), "copy");
  return BBTC_OK;
}

void bbtc_plan_destroy(bbtc_plan* pl) { delete pl; }

const char* bbtc_last_error(void) { return g_err.c_str(); }

}  // extern "C"
