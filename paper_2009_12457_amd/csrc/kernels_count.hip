// Per-task triangle counting kernels (arXiv 2009.12457, Sec. 4.3).
//
// A task {i,j,k} counts, for every u in V_i and v in N(G_ij,u), the common
// elements of N(G_ik,u) and N(G_jk,v).  Only rows u of the active-row list of
// block (i,j) are visited (others have N(G_ij,u) empty); rows with N(G_ik,u)
// empty are skipped.
//
// Two row mappings (the split is a tuning knob; both are exact):
//   * light rows (d(G_ij,u) < wave_min): one lane per row, a two-pointer
//     count of sorted lists (the list intersection of Alg. 1);
//   * heavy rows: one 64-lane wavefront per row.  N(G_ik,u) is staged in LDS
//     once, the lanes flatten the probe space {(v,w): v in N(G_ij,u),
//     w in N(G_jk,v)} with a wavefront prefix sum, and each probe w is tested
//     against the staged row:
//       - Intersect form: binary search of a sorted LDS copy;
//       - HMap form: a dense bitmap over the columns of V_k (the paper's dense
//         hash map of the block's column range) when |V_k| fits in LDS, else
//         an open-addressing LDS hash of N(G_ik,u).
//     Rows longer than the LDS buffer are staged in disjoint pieces; a probe
//     matches at most one piece, so the count stays exact.
#include "bbtc_internal.h"
#include "dev_common.h"

namespace bbtc {

namespace {

constexpr int kABuf = 2048;                   // LDS words per wavefront
constexpr uint32_t kBitmapBits = kABuf * 32;  // bitmap capacity in columns
constexpr int kHashBits = 11;                 // 2^11 = kABuf hash slots
static_assert((1 << kHashBits) == kABuf, "hash table fills the wave buffer");

struct CountLds {
  uint32_t abuf[4][kABuf];  // per wave: sorted copy / bitmap / hash; all-zero between rows
  uint32_t sc0[4][kWave];   // per wave: start of N(G_jk,v) for the batch's lanes
  uint32_t sex[4][kWave];   // per wave: exclusive prefix of the batch's lengths
  uint32_t q[kThreads][4];  // heavy-row queue: sb0, sb1, sa0, sa1
  uint32_t qn;
  uint32_t item;
  unsigned long long red[4];
};

struct TaskCtx {
  int32_t ci, cj, ck, ck1;
  int32_t dj, dk, dkj;      // j-i, k-i, k-j
  uint32_t stri, strj;      // bot row strides of parts i and j
  const uint32_t* boti;
  const uint32_t* botj;
  const int32_t* ar;        // active rows of block (i,j)
};

__device__ __forceinline__ TaskCtx make_ctx(const GraphView& g, const DevTask& t) {
  TaskCtx c;
  c.ci = g.cuts[t.i];
  c.cj = g.cuts[t.j];
  c.ck = g.cuts[t.k];
  c.ck1 = g.cuts[t.k + 1];
  c.dj = t.j - t.i;
  c.dk = t.k - t.i;
  c.dkj = t.k - t.j;
  c.stri = (uint32_t)(g.p - t.i + 1);
  c.strj = (uint32_t)(g.p - t.j + 1);
  c.boti = g.bot + g.botp[t.i];
  c.botj = g.bot + g.botp[t.j];
  c.ar = g.arow + g.arp[block_id(g.p, t.i, t.j)];
  return c;
}

// |N(G_ik,u) cap N(G_jk,v)| summed over v in N(G_ij,u), one lane.
__device__ __forceinline__ uint64_t light_row(const int32_t* __restrict__ col, const TaskCtx& c, uint32_t sb0,
                                              uint32_t sb1, uint32_t sa0, uint32_t sa1) {
  uint64_t cnt = 0;
  for (uint32_t e = sb0; e < sb1; ++e) {
    const int32_t v = col[e];
    const uint32_t* vr = c.botj + (uint64_t)(v - c.cj) * c.strj;
    uint32_t b = vr[c.dkj];
    const uint32_t be = vr[c.dkj + 1];
    if (b >= be) continue;
    uint32_t a = sa0;
    int32_t x = col[a], y = col[b];
    while (true) {
      if (x == y) {
        ++cnt;
        if (++a >= sa1 || ++b >= be) break;
        x = col[a];
        y = col[b];
      } else if (x < y) {
        if (++a >= sa1) break;
        x = col[a];
      } else {
        if (++b >= be) break;
        y = col[b];
      }
    }
  }
  return cnt;
}

__device__ __forceinline__ uint32_t hash_slot(uint32_t w) { return (w * 0x9E3779B1u) >> (32 - kHashBits); }

// One wavefront counts one heavy row.  Wave-uniform arguments.
__device__ uint64_t heavy_row(const int32_t* __restrict__ col, const TaskCtx& c, uint32_t sb0, uint32_t sb1,
                              uint32_t sa0, uint32_t sa1, bool use_hash, uint32_t mcol, uint32_t* abuf,
                              uint32_t* sc0, uint32_t* sex) {
  const int l = lane_id();
  uint64_t cnt = 0;
  // 0: sorted copy + binary search, 1: bitmap over V_k, 2: hash of the row
  int mode = 0;
  uint32_t piece = kABuf;
  if (use_hash) {
    if ((uint32_t)(c.ck1 - c.ck) <= kBitmapBits) {
      mode = 1;
      piece = sa1 - sa0;
    } else {
      mode = 2;
      piece = kABuf / 2;
    }
  }
  for (uint32_t a_lo = sa0; a_lo < sa1; a_lo += piece) {
    const uint32_t an = min(piece, sa1 - a_lo);
    if (mode == 0) {
      for (uint32_t t = l; t < an; t += kWave) abuf[t] = (uint32_t)col[a_lo + t];
    } else if (mode == 1) {
      for (uint32_t t = l; t < an; t += kWave) {
        const uint32_t x = (uint32_t)(col[a_lo + t] - c.ck);
        atomicOr(&abuf[x >> 5], 1u << (x & 31));
      }
    } else {
      for (uint32_t t = l; t < an; t += kWave) {
        const uint32_t key = (uint32_t)col[a_lo + t] + 1u;  // 0 marks an empty slot
        uint32_t s = hash_slot(key - 1u);
        for (int guard = 0; guard < kABuf && atomicCAS(&abuf[s], 0u, key) != 0u; ++guard) s = (s + 1) & (kABuf - 1);
      }
    }
    wave_sync();
    const int32_t amin = col[a_lo], amax = col[a_lo + an - 1];
    for (uint32_t eb = sb0; eb < sb1; eb += kWave) {
      const uint32_t e = eb + l;
      uint32_t len = 0, c0 = 0;
      if (e < sb1) {
        const int32_t v = col[e];
        const uint32_t* vr = c.botj + (uint64_t)(v - c.cj) * c.strj;
        c0 = vr[c.dkj];
        len = vr[c.dkj + 1] - c0;
      }
      const uint32_t inc = wave_incl_scan_u32(len);
      const uint32_t tot = __shfl(inc, kWave - 1, kWave);
      sc0[l] = c0;
      sex[l] = inc - len;
      wave_sync();
      for (uint32_t qb = 0; qb < tot; qb += kWave) {
        const uint32_t q = qb + l;
        if (q < tot) {
          int lo = 0, hi = kWave - 1;  // owner: the largest lane o with sex[o] <= q
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sex[mid] <= q) lo = mid; else hi = mid - 1;
          }
          const uint32_t src = sc0[lo] + (q - sex[lo]);
          const int32_t w = col[src < mcol ? src : mcol - 1];
          if (w >= amin && w <= amax) {
            if (mode == 0) {
              uint32_t x = 0, y = an;
              while (x < y) {
                const uint32_t mid = (x + y) >> 1;
                if (abuf[mid] < (uint32_t)w) x = mid + 1; else y = mid;
              }
              cnt += (x < an && abuf[x] == (uint32_t)w) ? 1u : 0u;
            } else if (mode == 1) {
              const uint32_t x = (uint32_t)(w - c.ck);
              cnt += (abuf[x >> 5] >> (x & 31)) & 1u;
            } else {
              const uint32_t key = (uint32_t)w + 1u;
              uint32_t s = hash_slot((uint32_t)w);
              for (int guard = 0; guard < kABuf; ++guard) {
                const uint32_t k = abuf[s];
                if (k == key) { ++cnt; break; }
                if (k == 0u) break;
                s = (s + 1) & (kABuf - 1);
              }
            }
          }
        }
      }
      wave_sync();
    }
    // restore the all-zero buffer
    if (mode == 0) {
      for (uint32_t t = l; t < an; t += kWave) abuf[t] = 0;
    } else if (mode == 1) {
      for (uint32_t t = l; t < an; t += kWave) abuf[(uint32_t)(col[a_lo + t] - c.ck) >> 5] = 0;
    } else {
      for (uint32_t t = l; t < kABuf; t += kWave) abuf[t] = 0;
    }
    wave_sync();
  }
  return cnt;
}

// Rows [lo, hi) of the task's active-row list, by the whole workgroup.
__device__ uint64_t process_rows(const PlanCtx& cp, const TaskCtx& c, uint32_t lo, uint32_t hi, CountLds& s) {
  const int t = threadIdx.x, w = t / kWave;
  const int32_t* __restrict__ col = cp.g.ocol;
  uint64_t cnt = 0;
  for (uint32_t base = lo; base < hi; base += kThreads) {
    const uint32_t x = base + t;
    if (x < hi) {
      const int32_t u = c.ar[x];
      const uint32_t* ur = c.boti + (uint64_t)(u - c.ci) * c.stri;
      const uint32_t sb0 = ur[c.dj], sb1 = ur[c.dj + 1], sa0 = ur[c.dk], sa1 = ur[c.dk + 1];
      if (sa1 > sa0 && sb1 > sb0) {
        if (sb1 - sb0 >= (uint32_t)cp.wave_min) {
          const uint32_t qi = atomicAdd(&s.qn, 1u);
          s.q[qi][0] = sb0;
          s.q[qi][1] = sb1;
          s.q[qi][2] = sa0;
          s.q[qi][3] = sa1;
        } else {
          cnt += light_row(col, c, sb0, sb1, sa0, sa1);
        }
      }
    }
    __syncthreads();
    const uint32_t nq = s.qn;
    for (uint32_t h = w; h < nq; h += 4) {
      const uint32_t sb0 = s.q[h][0], sb1 = s.q[h][1], sa0 = s.q[h][2], sa1 = s.q[h][3];
      const bool use_hash = cp.hash_min >= 0 && (sa1 - sa0) >= (uint32_t)cp.hash_min;
      cnt += heavy_row(col, c, sb0, sb1, sa0, sa1, use_hash, cp.g.m, s.abuf[w], s.sc0[w], s.sex[w]);
    }
    __syncthreads();
    if (t == 0) s.qn = 0;
    __syncthreads();
  }
  return cnt;
}

__device__ __forceinline__ void init_lds(CountLds& s) {
  uint32_t* a = &s.abuf[0][0];
  for (int t = threadIdx.x; t < 4 * kABuf; t += kThreads) a[t] = 0;
  if (threadIdx.x == 0) s.qn = 0;
  __syncthreads();
}

__device__ __forceinline__ void flush(const PlanCtx& cp, int32_t out, uint64_t cnt, CountLds& s) {
  cnt = block256_sum_u64(cnt, s.red);
  if (threadIdx.x == 0 && cnt) {
    atomicAdd((unsigned long long*)&cp.per_task[out], (unsigned long long)cnt);
    atomicAdd((unsigned long long*)cp.total, (unsigned long long)cnt);
  }
}

// One launch per task (the unbatched form): workgroup b takes rows
// [b*256, b*256+256) of the task's active rows.
__global__ __launch_bounds__(kThreads) void k_count_task(CountParams cp, int32_t task, uint32_t nrows) {
  __shared__ CountLds s;
  init_lds(s);
  const PlanCtx& pc = cp.one;
  const DevTask t = pc.tasks[task];
  const TaskCtx c = make_ctx(pc.g, t);
  const uint32_t lo = blockIdx.x * kThreads;
  const uint32_t hi = min(nrows, lo + kThreads);
  const uint64_t cnt = process_rows(pc, c, lo, hi, s);
  flush(pc, t.out, cnt, s);
}

// Persistent work-stealing form: every workgroup claims work items from a
// global cursor until none are left.  MULTI: items of several plans.
template <bool MULTI>
__global__ __launch_bounds__(kThreads) void k_count_persistent(CountParams cp) {
  __shared__ CountLds s;
  init_lds(s);
  while (true) {
    if (threadIdx.x == 0) s.item = atomicAdd(cp.cursor, 1u);
    __syncthreads();
    const uint32_t it = s.item;
    __syncthreads();
    if (it >= cp.nitems) break;
    const DevItem item = cp.items[it];
    const PlanCtx pc = MULTI ? cp.many[item.plan] : cp.one;
    const DevTask t = pc.tasks[item.task];
    const TaskCtx c = make_ctx(pc.g, t);
    const uint64_t cnt = process_rows(pc, c, item.lo, item.hi, s);
    flush(pc, t.out, cnt, s);
  }
}

__global__ __launch_bounds__(kThreads) void k_reset(uint64_t* per_task, int64_t ntasks, uint64_t* total,
                                                    uint32_t* cursor) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntasks; t += (int64_t)gridDim.x * blockDim.x)
    per_task[t] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *total = 0;
    if (cursor) *cursor = 0;
  }
}

}  // namespace

hipError_t launch_reset(uint64_t* per_task, int64_t ntasks, uint64_t* total, uint32_t* cursor, hipStream_t s) {
  int64_t g = (ntasks + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_reset, dim3((unsigned)g), dim3(kThreads), 0, s, per_task, ntasks, total, cursor);
  return hipGetLastError();
}

hipError_t launch_count_task(const CountParams& cp, int32_t task, uint32_t nrows, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  const unsigned g = (nrows + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_count_task, dim3(g), dim3(kThreads), 0, s, cp, task, nrows);
  return hipGetLastError();
}

hipError_t launch_count_persistent(const CountParams& cp, int grid, bool multi, hipStream_t s) {
  if (multi)
    hipLaunchKernelGGL(k_count_persistent<true>, dim3(grid), dim3(kThreads), 0, s, cp);
  else
    hipLaunchKernelGGL(k_count_persistent<false>, dim3(grid), dim3(kThreads), 0, s, cp);
  return hipGetLastError();
}

int count_persistent_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_count_persistent<false>, kThreads, 0) != hipSuccess ||
      nb < 1)
    nb = 1;
  return nb;
}

}  // namespace bbtc
