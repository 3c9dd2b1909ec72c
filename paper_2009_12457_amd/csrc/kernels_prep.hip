// Preprocessing kernels: input validation, degree ordering, orientation, the
// symmetric rectilinear cut and the block row index (arXiv 2009.12457,
// Sec. 2 and 4.1).  Everything runs on the device; the host only sizes
// buffers between steps.
#include <algorithm>

#include "bbtc_internal.h"
#include "dev_common.h"

namespace bbtc {

namespace {

inline unsigned grid_for(uint64_t work_items, unsigned per_block, unsigned cap = 1u << 20) {
  uint64_t g = (work_items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// Wave-per-row grid: enough waves to fill the chip several times over.
constexpr unsigned kRowGrid = 8192;  // workgroups (4 waves each)

// ------------------------------------------------------------ validation
// Checks a symmetric CSR: rows within [0, nnz], entries in [0, n), strictly
// increasing, no self-loop, and (optionally) every (x,y) mirrored by (y,x).
// Every index is clamped before use, so malformed input cannot read out of
// bounds.  Error bits: 1 range, 2 order, 4 self-loop, 8 rowptr, 16 asymmetric.
//
// Row kernels here come in two forms: one lane per row for rows of at most
// kLaneRow entries (longer rows are appended to a list), and one wavefront
// per listed row.
constexpr int64_t kLaneRow = 64;     // longest row handled by one lane
constexpr int64_t kWaveRow = 4096;   // longest row handled by one wavefront
constexpr int64_t kRowChunk = 2048;  // entries of a huge row per wavefront work unit

// Lists: rows of (kLaneRow, kWaveRow] entries go to `list` (one wavefront
// each), longer rows to `hlist`, which is short (the hubs): its rows are cut
// into chunks of kRowChunk entries, and a wavefront finds its chunks by
// walking that list.
// hpref[q] = chunks of hlist rows before position q (q = 0..hcnt), written by
// k_hprefix; work unit u belongs to the row q with hpref[q] <= u < hpref[q+1].
template <typename RP>
__global__ __launch_bounds__(kThreads) void k_hprefix(const RP* __restrict__ rowptr, const uint32_t* hlist,
                                                      const uint32_t* nhlist, uint32_t* hpref) {
  __shared__ uint32_t lds[4];
  const uint32_t cnt = *nhlist;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < cnt; base += kThreads) {
    const uint32_t q = base + threadIdx.x;
    uint32_t nch = 0;
    if (q < cnt) {
      const int64_t r = hlist[q];
      nch = (uint32_t)((((int64_t)rowptr[r + 1] - (int64_t)rowptr[r]) + kRowChunk - 1) / kRowChunk);
    }
    uint32_t tot;
    const uint32_t ex = block256_excl_scan<uint32_t>(nch, lds, &tot);
    if (q < cnt) hpref[q] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) hpref[cnt] = carry;
}

template <typename RP>
__device__ __forceinline__ void unit_of(const RP* __restrict__ rowptr, const uint32_t* hlist, const uint32_t* hpref,
                                        uint32_t cnt, uint32_t u, uint32_t* li, int64_t* x, int64_t* b, int64_t* e) {
  uint32_t lo = 0, hi = cnt - 1;  // the largest q with hpref[q] <= u
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (hpref[mid] <= u) lo = mid; else hi = mid - 1;
  }
  const int64_t r = hlist[lo];
  const int64_t rb = (int64_t)rowptr[r], re = (int64_t)rowptr[r + 1];
  *li = lo;
  *x = r;
  *b = rb + (int64_t)(u - hpref[lo]) * kRowChunk;
  *e = min(re, *b + kRowChunk);
}

template <typename RP>
__device__ __forceinline__ uint32_t check_entry(const RP* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                                int64_t n, int64_t nnz, int symmetric, int64_t x, int64_t b, int64_t q) {
  uint32_t e = 0;
  const int32_t y = colidx[q];
  if (y < 0 || y >= n) return 1;
  if (y == x) e |= 4;
  if (q > b && colidx[q - 1] >= y) e |= 2;
  if (symmetric) {
    int64_t lo = (int64_t)rowptr[y], hi = (int64_t)rowptr[y + 1];
    if (lo < 0 || hi < lo || hi > nnz) return e | 8;
    const int64_t end = hi;
    while (lo < hi) {  // lower_bound of x in row y
      int64_t mid = (lo + hi) >> 1;
      if (colidx[mid] < x) lo = mid + 1; else hi = mid;
    }
    if (lo >= end || colidx[lo] != x) e |= 16;
  }
  return e;
}

template <typename RP>
__global__ __launch_bounds__(kThreads) void k_validate_lane(const RP* __restrict__ rowptr,
                                                            const int32_t* __restrict__ colidx, int64_t n, int64_t nnz,
                                                            int symmetric, uint32_t* err, uint32_t* list,
                                                            uint32_t* nlist, uint32_t* hlist, uint32_t* nhlist) {
  uint32_t e = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if ((int64_t)rowptr[0] != 0 || (int64_t)rowptr[n] != nnz) e |= 8;
  }
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = (int64_t)rowptr[x], en = (int64_t)rowptr[x + 1];
    if (b < 0 || en < b || en > nnz) {
      e |= 8;
      continue;
    }
    if (en - b > kWaveRow) {
      hlist[atomicAdd(nhlist, 1u)] = (uint32_t)x;
      continue;
    }
    if (en - b > kLaneRow) {
      list[atomicAdd(nlist, 1u)] = (uint32_t)x;
      continue;
    }
    for (int64_t q = b; q < en; ++q) e |= check_entry(rowptr, colidx, n, nnz, symmetric, x, b, q);
  }
  if (e) atomicOr(err, e);
}

template <typename RP>
__global__ __launch_bounds__(kThreads) void k_validate_wave(const RP* __restrict__ rowptr,
                                                            const int32_t* __restrict__ colidx, int64_t n, int64_t nnz,
                                                            int symmetric, uint32_t* err, const uint32_t* list,
                                                            const uint32_t* nlist, const uint32_t* hlist,
                                                            const uint32_t* nhlist, const uint32_t* hpref) {
  const int l = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  uint32_t e = 0;
  const int64_t cnt = *nlist;
  for (int64_t r = wave; r < cnt; r += nwaves) {
    const int64_t x = list[r];
    const int64_t b = (int64_t)rowptr[x], en = (int64_t)rowptr[x + 1];
    for (int64_t q = b + l; q < en; q += kWave) e |= check_entry(rowptr, colidx, n, nnz, symmetric, x, b, q);
  }
  const uint32_t hcnt = *nhlist;
  const uint32_t units = hcnt ? hpref[hcnt] : 0u;
  for (uint32_t u = (uint32_t)wave; u < units; u += (uint32_t)nwaves) {
    uint32_t li;
    int64_t x, b, en;
    unit_of(rowptr, hlist, hpref, hcnt, u, &li, &x, &b, &en);
    const int64_t rb = (int64_t)rowptr[x];
    for (int64_t q = b + l; q < en; q += kWave) e |= check_entry(rowptr, colidx, n, nnz, symmetric, x, rb, q);
  }
  if (e) atomicOr(err, e);
}

template <typename RP>
__global__ __launch_bounds__(kThreads) void k_degkey(const RP* __restrict__ rowptr, int64_t n, int idbits,
                                                     uint64_t* __restrict__ keys) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    uint64_t d = (uint64_t)((int64_t)rowptr[x + 1] - (int64_t)rowptr[x]);
    keys[x] = (d << idbits) | (uint64_t)x;
  }
}

// ------------------------------------------------------------ prefix scan
__device__ __forceinline__ uint32_t tile_load(const uint32_t* in, uint64_t i, uint64_t count) {
  return i < count ? in[i] : 0u;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ in, uint64_t count,
                                                          uint32_t* __restrict__ partial) {
  __shared__ uint32_t lds[4];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) s += tile_load(in, base + (uint64_t)r * kThreads + threadIdx.x, count);
  uint32_t tot;
  block256_excl_scan<uint32_t>(s, lds, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the tile sums in place, grand total to *total.
__global__ __launch_bounds__(kThreads) void k_scan_spine(uint32_t* __restrict__ partial, uint64_t nparts,
                                                         uint32_t* __restrict__ total) {
  __shared__ uint32_t lds[4];
  uint32_t carry = 0;
  for (uint64_t base = 0; base < nparts; base += kThreads) {
    uint64_t i = base + threadIdx.x;
    uint32_t v = i < nparts ? partial[i] : 0u;
    uint32_t tot;
    uint32_t ex = block256_excl_scan<uint32_t>(v, lds, &tot);
    if (i < nparts) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

// Blocked arrangement: thread t owns items [t*kScanItems, (t+1)*kScanItems).
__global__ __launch_bounds__(kThreads) void k_scan_down(const uint32_t* in, uint32_t* out, uint64_t count,
                                                        const uint32_t* __restrict__ partial) {
  __shared__ uint32_t lds[4];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    v[r] = tile_load(in, base + r, count);
    s += v[r];
  }
  uint32_t tot;
  uint32_t run = partial[blockIdx.x] + block256_excl_scan<uint32_t>(s, lds, &tot);
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    if (base + r < count) out[base + r] = run;
    run += v[r];
  }
}

// ------------------------------------------------------------ radix sort
// Stable LSD radix sort of 64-bit keys, 8 bits per pass: per-tile digit
// histograms, one global exclusive scan over (digit, tile), then a stable
// scatter in which every key's rank among equal digits follows input order.
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint64_t* __restrict__ keys, uint64_t count,
                                                         int shift, uint32_t* __restrict__ hist, uint32_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kRadixTile;
  for (int r = 0; r < kRadixItems; ++r) {
    uint64_t i = base + (uint64_t)r * kThreads + threadIdx.x;
    if (i < count) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                            uint64_t* __restrict__ kout, uint64_t count, int shift,
                                                            const uint32_t* __restrict__ hist, uint32_t ntiles) {
  __shared__ uint32_t next[256];     // next output slot per digit for this tile
  __shared__ uint32_t wbase[4][256]; // per-wave counts, then per-wave bases
  const int t = threadIdx.x, w = t / kWave;
  next[t] = hist[(uint64_t)t * ntiles + blockIdx.x];
  const uint64_t base = (uint64_t)blockIdx.x * kRadixTile;
  for (int r = 0; r < kRadixItems; ++r) {
    const uint64_t i = base + (uint64_t)r * kThreads + t;
    const bool valid = i < count;
    const uint64_t key = valid ? kin[i] : 0ull;
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
#pragma unroll
    for (int q = 0; q < 4; ++q) wbase[q][t] = 0;
    __syncthreads();
    uint64_t same = ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t b = ballot(on);
      same &= on ? b : ~b;
    }
    const uint32_t below = lanes_below(same);
    if (valid && below == 0) wbase[w][d] = (uint32_t)__popcll(same);
    __syncthreads();
    {  // thread t owns digit t
      uint32_t c0 = wbase[0][t], c1 = wbase[1][t], c2 = wbase[2][t], c3 = wbase[3][t];
      uint32_t b0 = next[t];
      wbase[0][t] = b0;
      wbase[1][t] = b0 + c0;
      wbase[2][t] = b0 + c0 + c1;
      wbase[3][t] = b0 + c0 + c1 + c2;
      next[t] = b0 + c0 + c1 + c2 + c3;
    }
    __syncthreads();
    const uint32_t dst = wbase[w][d] + below;
    if (valid && dst < count) kout[dst] = key;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_perm(const uint64_t* __restrict__ keys, int64_t n, uint64_t mask,
                                                   int32_t* __restrict__ order, int32_t* __restrict__ perm) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = (int64_t)(keys[r] & mask);
    if (x < n) {
      order[r] = (int32_t)x;
      perm[x] = (int32_t)r;
    }
  }
}

// ------------------------------------------------------------ orientation
// For original vertex x of rank r: neighbours y with rank(y) > r form the
// out-row N(G,r), the others the in-row of r.
// With `check` set, the degree pass also validates the input (every check
// but symmetry): rowptr bounds per row (a bad row is skipped, its entries
// never read), column range (a bad entry is not used as an index), self-
// loops and strictly increasing rows, ORed into err as the validation
// kernels do.
template <typename RP>
__device__ __forceinline__ uint32_t entry_flags(const int32_t* __restrict__ colidx, int64_t n, int64_t x,
                                                int64_t rb, int64_t q, int32_t y) {
  if (y < 0 || y >= n) return 1;
  uint32_t e = 0;
  if (y == x) e |= 4;
  if (q > rb && colidx[q - 1] >= y) e |= 2;
  return e;
}

// Rows of at most kLaneRow entries are handled 64 consecutive rows per
// wavefront with their entries spread over the lanes ("flattened"): a
// wavefront prefix sum of the row lengths gives each lane its entry, the
// owner row follows by binary search over the prefix, and per-row counts and
// positions come from ballots over the runs of equal owners.
struct FlatRows {
  uint32_t off[kWave];  // exclusive prefix of the group's lane-row lengths
  int64_t beg[kWave];   // first entry of each row in colidx
  int32_t rank[kWave];  // rank of each row (perm)
  uint32_t c0[kWave];   // per row: running count / next out-row slot
  uint32_t c1[kWave];   // per row: next in-row slot
};

__device__ __forceinline__ uint32_t owner_lane(const uint32_t* off, uint32_t f) {
  uint32_t lo = 0;
#pragma unroll
  for (uint32_t step = kWave / 2; step > 0; step >>= 1)
    if (off[lo + step] <= f) lo += step;
  return lo;
}

// Lanes of the run (equal owner) that lane l belongs to, within one chunk of
// 64 flattened entries: `heads` marks the first lane of every run.
__device__ __forceinline__ uint64_t run_mask(uint64_t heads, int l) {
  const uint64_t below = (l == 63) ? ~0ull : ((1ull << (l + 1)) - 1);  // lanes 0..l
  const uint64_t h = heads & below;
  const int first = 63 - __clzll(h);  // the run's head (lane 0 is always a head)
  const uint64_t after = heads & ~below;
  const int next = after ? __ffsll((unsigned long long)after) - 1 : 64;
  const uint64_t upto = (next == 64) ? ~0ull : ((1ull << next) - 1);
  return upto & ~((1ull << first) - 1);
}

// Row kernels work on a range of the input rows: local row x is original
// vertex rr.x0 + x (its rank perm[rr.x0 + x]), the row pointers passed in
// start at that row and hold absolute positions, which index the column
// pointer passed in (shifted when only the range's entries are resident).
// Entries are checked against rr.ntot vertices and the row pointers against
// [rr.nnz_lo, rr.nnz_hi].  With od == nullptr the degree pass only lists the
// long and huge rows (for a later fill of the same range).
template <typename RP>
__global__ __launch_bounds__(kThreads) void k_degs_lane(const RP* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colidx, int64_t n, RowRange rr,
                                                        const int32_t* __restrict__ perm, uint32_t* __restrict__ od,
                                                        uint32_t* __restrict__ idg, uint32_t* list, uint32_t* nlist,
                                                        uint32_t* hlist, uint32_t* nhlist, uint32_t* err, int check,
                                                        int32_t* __restrict__ rc) {
  __shared__ FlatRows fr[kThreads / kWave];
  const int l = lane_id();
  FlatRows& F = fr[threadIdx.x / kWave];
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const bool count = od != nullptr;
  uint32_t bad = 0;
  if (check && blockIdx.x == 0 && threadIdx.x == 0) {
    if ((int64_t)rowptr[0] != rr.nnz_lo || (int64_t)rowptr[n] != rr.nnz_hi) bad |= 8;
  }
  for (int64_t x0 = wave * kWave; x0 < n; x0 += nwaves * kWave) {  // uniform per wavefront
    const int64_t x = x0 + l;
    int32_t r = -1;
    int64_t b = 0, e = 0;
    bool mine = false;  // a lane row: counted by this group
    if (x < n) {
      r = perm[rr.x0 + x];
      b = (int64_t)rowptr[x];
      e = (int64_t)rowptr[x + 1];
      if (r >= 0 && r < rr.ntot) {
        if (check && (b < rr.nnz_lo || e < b || e > rr.nnz_hi)) {
          bad |= 8;
          if (count) od[r] = idg[r] = 0;
        } else if (e - b > kWaveRow) {
          if (count) od[r] = idg[r] = 0;
          hlist[atomicAdd(nhlist, 1u)] = (uint32_t)x;
        } else if (e - b > kLaneRow) {
          list[atomicAdd(nlist, 1u)] = (uint32_t)x;
        } else {
          mine = count;
        }
      }
    }
    const uint32_t len = mine ? (uint32_t)(e - b) : 0u;
    const uint32_t inc = wave_incl_scan_u32(len);
    const uint32_t tot = last_lane(inc);
    F.off[l] = inc - len;
    F.beg[l] = b;
    F.rank[l] = r;
    F.c0[l] = 0;
    wave_sync();
    for (uint32_t fb = 0; fb < tot; fb += kWave) {
      const uint32_t f = fb + l;
      const bool act = f < tot;
      uint32_t o = 0;
      bool up = false;
      if (act) {
        o = owner_lane(F.off, f);
        const int64_t rb = F.beg[o], q = rb + (f - F.off[o]);
        const int32_t y = colidx[q];
        uint32_t fl = 0;
        if (check) fl = entry_flags<RP>(colidx, rr.ntot, rr.x0 + x0 + o, rb, q, y);
        bad |= fl;
        if (!(fl & 1)) {
          const int32_t ry = perm[y];
          if (rc) rc[q] = ry;
          up = ry > F.rank[o];
        }
      }
      const uint64_t heads = ballot(act && (l == 0 || f == F.off[o]));
      const uint64_t ups = ballot(up);
      if (act && ((heads >> l) & 1ull)) atomicAdd(&F.c0[o], (uint32_t)__popcll(ups & run_mask(heads, l)));
    }
    wave_sync();
    if (mine) {
      od[r] = F.c0[l];
      idg[r] = len - F.c0[l];
    }
    wave_sync();
  }
  if (bad) atomicOr(err, bad);
}

constexpr int kUnroll = 4;  // 64-entry chunks of a row in flight per wavefront step

// This lane's count of entries q in [b, e) (row x of rank r, starting at rb)
// with a higher-ranked neighbour; with `check`, the entry checks are ORed
// into *bad.  Loads of kUnroll chunks are issued before any is used.
template <typename RP>
__device__ __forceinline__ uint32_t count_up(const int32_t* __restrict__ colidx, int64_t n,
                                             const int32_t* __restrict__ perm, int64_t x, int32_t r, int64_t rb,
                                             int64_t b, int64_t e, int check, uint32_t* bad,
                                             int32_t* __restrict__ rcout, const int32_t* __restrict__ rcin) {
  const int l = lane_id();
  uint32_t c = 0;
  for (int64_t base = b; base < e; base += kUnroll * kWave) {
    int32_t y[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const int64_t q = base + k * kWave + l;
      y[k] = q < e ? (rcin ? rcin[q] : colidx[q]) : -1;
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const int64_t q = base + k * kWave + l;
      if (q < e) {
        const uint32_t f = check ? entry_flags<RP>(colidx, n, x, rb, q, y[k]) : 0u;
        *bad |= f;
        if (!(f & 1)) {
          const int32_t ry = rcin ? y[k] : perm[y[k]];
          if (rcout) rcout[q] = ry;
          if (ry > r) ++c;
        }
      }
    }
  }
  return c;
}

// Listed rows: one wavefront per row; huge rows: chunks counted by different
// wavefronts and added to od/idg, which k_degs_lane zeroed for them.
template <typename RP>
__global__ __launch_bounds__(kThreads) void k_degs_wave(const RP* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colidx, RowRange rr,
                                                        const int32_t* __restrict__ perm, uint32_t* __restrict__ od,
                                                        uint32_t* __restrict__ idg, const uint32_t* list,
                                                        const uint32_t* nlist, const uint32_t* hlist,
                                                        const uint32_t* nhlist, const uint32_t* hpref, uint32_t* err,
                                                        int check, int32_t* __restrict__ rc) {
  const int l = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  uint32_t bad = 0;
  const int64_t cnt = *nlist;
  for (int64_t i = wave; i < cnt; i += nwaves) {
    const int64_t x = list[i];
    const int32_t r = perm[rr.x0 + x];
    const int64_t b = (int64_t)rowptr[x], e = (int64_t)rowptr[x + 1];
    const uint32_t c =
        (uint32_t)wave_sum_u64(count_up<RP>(colidx, rr.ntot, perm, rr.x0 + x, r, b, b, e, check, &bad, rc, nullptr));
    if (l == 0) {
      od[r] = c;
      idg[r] = (uint32_t)(e - b) - c;
    }
  }
  const uint32_t hcnt = *nhlist;
  const uint32_t units = hcnt ? hpref[hcnt] : 0u;
  for (uint32_t u = (uint32_t)wave; u < units; u += (uint32_t)nwaves) {
    uint32_t li;
    int64_t x, b, e;
    unit_of(rowptr, hlist, hpref, hcnt, u, &li, &x, &b, &e);
    const int32_t r = perm[rr.x0 + x];
    const int64_t rb = (int64_t)rowptr[x];
    const uint32_t c =
        (uint32_t)wave_sum_u64(count_up<RP>(colidx, rr.ntot, perm, rr.x0 + x, r, rb, b, e, check, &bad, rc, nullptr));
    if (l == 0) {
      atomicAdd(&od[r], c);
      atomicAdd(&idg[r], (uint32_t)(e - b) - c);
    }
  }
  if (bad) atomicOr(err, bad);
}

// Scatters rank ids into the out- and in-rows (order within a row follows the
// input row; rows are sorted afterwards).  Writes are bounded by the row
// extents computed from the same predicate; a null ocol or icol skips that
// side.
template <typename RP>
__global__ __launch_bounds__(kThreads) void k_fill_lane(const RP* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colidx, int64_t n, RowRange rr,
                                                        const int32_t* __restrict__ perm,
                                                        const uint32_t* __restrict__ orow,
                                                        const uint32_t* __restrict__ irow, int32_t* __restrict__ ocol,
                                                        int32_t* __restrict__ icol, const int32_t* __restrict__ rc) {
  __shared__ FlatRows fr[kThreads / kWave];
  __shared__ uint32_t lim[kThreads / kWave][2][kWave];  // per row: end of its out- and in-row
  const int l = lane_id(), w = threadIdx.x / kWave;
  FlatRows& F = fr[w];
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t x0 = wave * kWave; x0 < n; x0 += nwaves * kWave) {  // uniform per wavefront
    const int64_t x = x0 + l;
    int32_t r = -1;
    int64_t b = 0, e = 0;
    bool mine = false;
    if (x < n) {
      r = perm[rr.x0 + x];
      b = (int64_t)rowptr[x];
      e = (int64_t)rowptr[x + 1];
      // listed rows: k_fill_wave; rows of ranks outside [rlo, rhi): not this pass
      mine = r >= rr.rlo && r < rr.rhi && e - b >= 0 && e - b <= kLaneRow;
    }
    const uint32_t len = mine ? (uint32_t)(e - b) : 0u;
    const uint32_t inc = wave_incl_scan_u32(len);
    const uint32_t tot = last_lane(inc);
    F.off[l] = inc - len;
    F.beg[l] = b;
    F.rank[l] = r;
    F.c0[l] = mine ? orow[r] : 0u;
    F.c1[l] = mine ? irow[r] : 0u;
    lim[w][0][l] = mine ? orow[r + 1] : 0u;
    lim[w][1][l] = mine ? irow[r + 1] : 0u;
    wave_sync();
    for (uint32_t fb = 0; fb < tot; fb += kWave) {
      const uint32_t f = fb + l;
      const bool act = f < tot;
      uint32_t o = 0;
      int32_t ry = 0;
      bool up = false;
      if (act) {
        o = owner_lane(F.off, f);
        const int64_t q = F.beg[o] + (f - F.off[o]);
        ry = rc ? rc[q] : perm[colidx[q]];
        up = ry > F.rank[o];
      }
      const uint64_t heads = ballot(act && (l == 0 || f == F.off[o]));
      const uint64_t ups = ballot(act && up), downs = ballot(act && !up);
      if (act) {
        const uint64_t run = run_mask(heads, l);
        const uint64_t before = run & ((1ull << l) - 1);  // lanes of my run below me
        if (up) {
          const uint32_t d = F.c0[o] + (uint32_t)__popcll(ups & before);
          if (ocol && d < lim[w][0][o]) ocol[d] = ry;
        } else {
          const uint32_t d = F.c1[o] + (uint32_t)__popcll(downs & before);
          if (icol && d < lim[w][1][o]) icol[d] = ry;
        }
      }
      wave_sync();  // every lane has read the counters before the heads advance them
      if (act && ((heads >> l) & 1ull)) {
        const uint64_t run = run_mask(heads, l);
        F.c0[o] += (uint32_t)__popcll(ups & run);
        F.c1[o] += (uint32_t)__popcll(downs & run);
      }
      wave_sync();
    }
    wave_sync();
  }
}

// Entries [b, e) of a row of rank r, by one wavefront: higher-ranked
// neighbours go to ocol from po on, the others to icol from pi on, in input
// order (ballot compaction); kUnroll chunks are gathered before any is
// written.  Writes stop at po_end / pi_end.
__device__ __forceinline__ void scatter_run(const int32_t* __restrict__ colidx, const int32_t* __restrict__ perm,
                                            int32_t r, int64_t b, int64_t e, uint32_t po, uint32_t pi,
                                            uint32_t po_end, uint32_t pi_end, int32_t* __restrict__ ocol,
                                            int32_t* __restrict__ icol, const int32_t* __restrict__ rc) {
  const int l = lane_id();
  for (int64_t base = b; base < e; base += kUnroll * kWave) {
    int32_t ry[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const int64_t q = base + k * kWave + l;
      ry[k] = q < e ? (rc ? rc[q] : colidx[q]) : -1;
    }
    if (!rc) {
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) ry[k] = ry[k] >= 0 ? perm[ry[k]] : -1;
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const int64_t q = base + k * kWave + l;
      const bool up = ry[k] > r;
      const bool down = q < e && !up;
      const uint64_t mu = ballot(up), md = ballot(down);
      const uint32_t du = po + lanes_below(mu), dd = pi + lanes_below(md);
      if (ocol && up && du < po_end) ocol[du] = ry[k];
      if (icol && down && dd < pi_end) icol[dd] = ry[k];
      po += (uint32_t)__popcll(mu);
      pi += (uint32_t)__popcll(md);
    }
  }
}

// Zeroes a[0..*count) and b[0..*count) (the huge rows' fill cursors).
__global__ __launch_bounds__(kThreads) void k_zero2(uint32_t* __restrict__ a, uint32_t* __restrict__ b,
                                                    const uint32_t* __restrict__ count) {
  const uint32_t c = *count;
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < c; x += gridDim.x * blockDim.x) a[x] = b[x] = 0;
}

// Listed rows: one wavefront per row (ballot compaction keeps input order).
// Huge rows: chunks reserve their slots with atomics on per-row cursors
// (cur_o/cur_i, zeroed, indexed by position in hlist), so the order inside
// such a row depends on timing; every row is sorted afterwards, which makes
// the result exact and deterministic.
template <typename RP>
__global__ __launch_bounds__(kThreads) void k_fill_wave(const RP* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colidx, RowRange rr,
                                                        const int32_t* __restrict__ perm,
                                                        const uint32_t* __restrict__ orow,
                                                        const uint32_t* __restrict__ irow, int32_t* __restrict__ ocol,
                                                        int32_t* __restrict__ icol, const uint32_t* list,
                                                        const uint32_t* nlist, const uint32_t* hlist,
                                                        const uint32_t* nhlist, const uint32_t* hpref, uint32_t* cur_o,
                                                        uint32_t* cur_i, const int32_t* __restrict__ rc) {
  const int l = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t cnt = *nlist;
  for (int64_t i = wave; i < cnt; i += nwaves) {
    const int64_t x = list[i];
    const int32_t r = perm[rr.x0 + x];
    if (r < rr.rlo || r >= rr.rhi) continue;
    const int64_t b = (int64_t)rowptr[x], e = (int64_t)rowptr[x + 1];
    scatter_run(colidx, perm, r, b, e, orow[r], irow[r], orow[r + 1], irow[r + 1], ocol, icol, rc);
  }
  const uint32_t hcnt = *nhlist;
  const uint32_t units = hcnt ? hpref[hcnt] : 0u;
  for (uint32_t u = (uint32_t)wave; u < units; u += (uint32_t)nwaves) {
    uint32_t li;
    int64_t x, b, e;
    unit_of(rowptr, hlist, hpref, hcnt, u, &li, &x, &b, &e);
    const int32_t r = perm[rr.x0 + x];
    if (r < rr.rlo || r >= rr.rhi) continue;
    const uint32_t ob = orow[r], ib = irow[r];
    const uint32_t po_end = orow[r + 1], pi_end = irow[r + 1];
    uint32_t nb = 0;
    const uint32_t nu =
        (uint32_t)wave_sum_u64(count_up<RP>(colidx, 0, perm, rr.x0 + x, r, b, b, e, 0, &nb, nullptr, rc));
    uint32_t po = 0, pi = 0;
    if (l == 0) {
      po = ob + atomicAdd(&cur_o[li], nu);
      pi = ib + atomicAdd(&cur_i[li], (uint32_t)(e - b) - nu);
    }
    po = __shfl(po, 0, kWave);
    pi = __shfl(pi, 0, kWave);
    scatter_run(colidx, perm, r, b, e, po, pi, po_end, pi_end, ocol, icol, rc);
  }
}

// ------------------------------------------------------------ row sort
// Bitonic sort of buf[0..N), N a power of two, by `nthr` cooperating threads
// numbered tid; SYNC orders LDS between stages.
template <typename SYNC>
__device__ __forceinline__ void bitonic_lds(int32_t* buf, uint32_t N, uint32_t tid, uint32_t nthr, SYNC sync) {
  for (uint32_t k = 2; k <= N; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t q = tid; q < (N >> 1); q += nthr) {
        const uint32_t i = ((q & ~(j - 1)) << 1) | (q & (j - 1));
        const uint32_t ixj = i | j;
        const int32_t a = buf[i], c = buf[ixj];
        const bool up = (i & k) == 0;
        if ((a > c) == up) {
          buf[i] = c;
          buf[ixj] = a;
        }
      }
      sync();
    }
  }
}

constexpr uint32_t kSegWave = 1024;    // longest row sorted by one wavefront
constexpr uint32_t kSegBlock = 16384;  // longest row sorted by one workgroup

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t x) {
  uint32_t n = 2;
  while (n < x) n <<= 1;
  return n;
}

constexpr uint32_t kSegLane = 16;  // longest row sorted by one lane, in registers

// Bitonic network over v[0..kSegLane) held in registers (indices are
// compile-time constants once the loops are unrolled).
__device__ __forceinline__ void bitonic_regs(int32_t (&v)[kSegLane]) {
#pragma unroll
  for (uint32_t k = 2; k <= kSegLane; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (uint32_t i = 0; i < kSegLane; ++i) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const int32_t a = v[i], c = v[ixj];
          const bool up = (i & k) == 0;
          const bool sw = up ? (a > c) : (a < c);
          v[i] = sw ? c : a;
          v[ixj] = sw ? a : c;
        }
      }
    }
  }
}

// Rows in groups of 64 consecutive rows per wavefront: a row of at most
// kSegLane entries is sorted by its own lane in registers; longer rows are
// queued: up to kSegWave entries for k_segsort_mid, up to kSegBlock for
// k_segsort_long, beyond that for k_segsort_huge.  q[2], q[0] and q[1]
// count them; every list has room for every row.
__global__ __launch_bounds__(kThreads) void k_segsort(const uint32_t* __restrict__ rp, int32_t* __restrict__ col,
                                                      int64_t nrows, uint32_t* __restrict__ midrows,
                                                      uint32_t* __restrict__ longrows,
                                                      uint32_t* __restrict__ hugerows, uint32_t* __restrict__ q) {
  const int l = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t g = wave * kWave; g < nrows; g += nwaves * kWave) {
    const int64_t r = g + l;
    if (r >= nrows) continue;
    const uint32_t s = rp[r], len = rp[r + 1] - s;
    if (len <= 1) continue;
    if (len <= kSegLane) {
      int32_t v[kSegLane];
#pragma unroll
      for (uint32_t t = 0; t < kSegLane; ++t) v[t] = t < len ? col[s + t] : 0x7FFFFFFF;
      bitonic_regs(v);
#pragma unroll
      for (uint32_t t = 0; t < kSegLane; ++t)
        if (t < len) col[s + t] = v[t];
    } else if (len <= kSegWave) {
      midrows[atomicAdd(&q[2], 1u)] = (uint32_t)r;
    } else if (len <= kSegBlock) {
      longrows[atomicAdd(&q[0], 1u)] = (uint32_t)r;
    } else {
      hugerows[atomicAdd(&q[1], 1u)] = (uint32_t)r;
    }
  }
}

// Bitonic sort of 64*E values held by one wavefront, E consecutive values
// per lane (value i in register i mod E of lane i / E): exchanges at
// distances below E stay in registers, longer ones pair lane l with lane
// l ^ (distance / E) through a lane shuffle; no LDS.
template <int E>
__device__ __forceinline__ void bitonic_wave(int32_t (&v)[E], uint32_t l) {
#pragma unroll
  for (uint32_t k = 2; k <= 64u * E; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j < (uint32_t)E) {
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
          const uint32_t o = r ^ j;
          if (o > r) {
            const bool up = ((l * E + r) & k) == 0;
            const int32_t a = v[r], b = v[o];
            v[r] = up ? min(a, b) : max(a, b);
            v[o] = up ? max(a, b) : min(a, b);
          }
        }
      } else {
        const int lj = (int)(j / E);
        const bool low = (l & (uint32_t)lj) == 0;
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)E; ++r) {
          const int32_t y = __shfl_xor(v[r], lj, kWave);
          const bool up = ((l * E + r) & k) == 0;
          v[r] = (low == up) ? min(v[r], y) : max(v[r], y);
        }
      }
    }
  }
}

// col[s, s+len) sorted by one wavefront in registers, len <= 64*E.
template <int E>
__device__ __forceinline__ void sort_row_wave(int32_t* __restrict__ col, uint32_t s, uint32_t len, uint32_t l) {
  int32_t v[E];
#pragma unroll
  for (uint32_t r = 0; r < (uint32_t)E; ++r) {
    const uint32_t t = l * E + r;
    v[r] = t < len ? col[s + t] : 0x7FFFFFFF;
  }
  bitonic_wave<E>(v, l);
#pragma unroll
  for (uint32_t r = 0; r < (uint32_t)E; ++r) {
    const uint32_t t = l * E + r;
    if (t < len) col[s + t] = v[r];
  }
}

// Bitonic sort of one value per lane within each group of W aligned lanes
// (W a power of two up to 64), every group ascending: the network of
// bitonic_wave<1> stopped at width W, its last merge ascending everywhere.
template <uint32_t W>
__device__ __forceinline__ void bitonic_groups(int32_t& v, uint32_t l) {
#pragma unroll
  for (uint32_t k = 2; k <= W; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      const int32_t y = __shfl_xor(v, (int)j, kWave);
      const bool up = k == W || (l & k) == 0;
      const bool low = (l & j) == 0;
      v = (low == up) ? min(v, y) : max(v, y);
    }
  }
}

// col[s, s+len) sorted by one wavefront at the power of two that holds it.
__device__ __forceinline__ void sort_mid_row(int32_t* __restrict__ col, uint32_t s, uint32_t len, uint32_t l) {
  if (len > kSegWave) return;
  if (len <= 64u) sort_row_wave<1>(col, s, len, l);
  else if (len <= 128u) sort_row_wave<2>(col, s, len, l);
  else if (len <= 256u) sort_row_wave<4>(col, s, len, l);
  else if (len <= 512u) sort_row_wave<8>(col, s, len, l);
  else sort_row_wave<16>(col, s, len, l);
}

// Wavefront per pair of queued rows of up to kSegWave entries, sorted in the
// lanes' registers (bitonic_wave) at the power of two that holds each; two
// rows of at most 32 entries are sorted together, one per half-wavefront.
__global__ __launch_bounds__(kThreads) void k_segsort_mid(const uint32_t* __restrict__ rp, int32_t* __restrict__ col,
                                                          const uint32_t* __restrict__ midrows,
                                                          const uint32_t* __restrict__ q) {
  static_assert(kSegWave == 16 * kWave, "rows of up to 16 entries per lane");
  const uint32_t l = (uint32_t)lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t step = 2 * (((int64_t)gridDim.x * blockDim.x) / kWave);
  const int64_t cnt = q[2];
  // the pair after next is looked up and the next pair's bounds are loaded
  // while this pair is sorted, so that a pair costs one round trip to memory
  // instead of three
  int64_t i = 2 * wave;
  uint32_t sa = 0, la = 0, sb = 0, lb = 0, na = 0, nb = 0;
  if (i < cnt) {
    const uint32_t r = midrows[i];
    sa = rp[r];
    la = rp[r + 1] - sa;
  }
  if (i + 1 < cnt) {
    const uint32_t r = midrows[i + 1];
    sb = rp[r];
    lb = rp[r + 1] - sb;
  }
  if (i + step < cnt) na = midrows[i + step];
  if (i + step + 1 < cnt) nb = midrows[i + step + 1];
  for (; i < cnt; i += step) {
    const uint32_t csa = sa, cla = la, csb = sb, clb = i + 1 < cnt ? lb : 0u;
    if (i + step < cnt) {
      sa = rp[na];
      la = rp[na + 1] - sa;
      if (i + step + 1 < cnt) {
        sb = rp[nb];
        lb = rp[nb + 1] - sb;
      }
      if (i + 2 * step < cnt) na = midrows[i + 2 * step];
      if (i + 2 * step + 1 < cnt) nb = midrows[i + 2 * step + 1];
    }
    if (cla <= 32u && clb <= 32u) {
      const uint32_t hl = l & 31u;
      const uint32_t s = l < 32u ? csa : csb, len = l < 32u ? cla : clb;
      int32_t v = hl < len ? col[s + hl] : 0x7FFFFFFF;
      bitonic_groups<32>(v, l);
      if (hl < len) col[s + hl] = v;
    } else {
      sort_mid_row(col, csa, cla, l);
      if (clb) sort_mid_row(col, csb, clb, l);
    }
  }
}

// Workgroup per queued long row (up to kSegBlock entries).
__global__ __launch_bounds__(kThreads) void k_segsort_long(const uint32_t* __restrict__ rp, int32_t* __restrict__ col,
                                                           const uint32_t* __restrict__ longrows,
                                                           const uint32_t* __restrict__ q) {
  __shared__ int32_t buf[kSegBlock];
  const uint32_t cnt = q[0];
  for (uint32_t qi = blockIdx.x; qi < cnt; qi += gridDim.x) {
    const uint32_t r = longrows[qi];
    const uint32_t s = rp[r], len = rp[r + 1] - s;
    if (len > kSegBlock) continue;
    const uint32_t N = pow2_at_least(len);
    for (uint32_t t = threadIdx.x; t < N; t += kThreads) buf[t] = t < len ? col[s + t] : 0x7FFFFFFF;
    __syncthreads();
    bitonic_lds(buf, N, threadIdx.x, kThreads, [] __device__() { __syncthreads(); });
    for (uint32_t t = threadIdx.x; t < len; t += kThreads) col[s + t] = buf[t];
    __syncthreads();
  }
}

// Workgroup per queued huge row: LSD radix sort of the row, 8 bits per pass,
// ping-ponging with scratch[rp[r] .. rp[r+1]) (rows own disjoint scratch, so
// rows sort concurrently).  Each pass histograms the row, scans the 256 bins
// and scatters tile by tile in input order, which keeps every pass stable.
__global__ __launch_bounds__(kThreads) void k_segsort_huge(const uint32_t* __restrict__ rp, int32_t* __restrict__ col,
                                                           int32_t* __restrict__ scratch,
                                                           const uint32_t* __restrict__ hugerows,
                                                           const uint32_t* __restrict__ q, int bits) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wcnt[4][256];
  __shared__ uint32_t lds[4];
  const int t = threadIdx.x, w = t / kWave;
  const uint32_t cnt = q[1];
  for (uint32_t qi = blockIdx.x; qi < cnt; qi += gridDim.x) {
    const uint32_t r = hugerows[qi];
    const uint32_t s = rp[r], len = rp[r + 1] - s;
    uint32_t* src = (uint32_t*)col + s;
    uint32_t* dst = (uint32_t*)scratch + s;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 8, ++passes) {
      hist[t] = 0;
      __syncthreads();
      for (uint32_t e = t; e < len; e += kThreads) atomicAdd(&hist[(src[e] >> shift) & 255u], 1u);
      __syncthreads();
      uint32_t tot;
      const uint32_t base = block256_excl_scan<uint32_t>(hist[t], lds, &tot);
      __syncthreads();
      hist[t] = base;  // next output slot per digit
      __syncthreads();
      for (uint32_t tb = 0; tb < len; tb += kThreads) {
        const uint32_t e = tb + t;
        const bool valid = e < len;
        const uint32_t key = valid ? src[e] : 0u;
        const uint32_t d = (key >> shift) & 255u;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) wcnt[qq][t] = 0;
        __syncthreads();
        uint64_t same = ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
          const bool on = (d >> bit) & 1u;
          const uint64_t bm = ballot(on);
          same &= on ? bm : ~bm;
        }
        const uint32_t below = lanes_below(same);
        if (valid && below == 0) wcnt[w][d] = (uint32_t)__popcll(same);
        __syncthreads();
        {
          const uint32_t c0 = wcnt[0][t], c1 = wcnt[1][t], c2 = wcnt[2][t], c3 = wcnt[3][t];
          const uint32_t b0 = hist[t];
          wcnt[0][t] = b0;
          wcnt[1][t] = b0 + c0;
          wcnt[2][t] = b0 + c0 + c1;
          wcnt[3][t] = b0 + c0 + c1 + c2;
          hist[t] = b0 + c0 + c1 + c2 + c3;
        }
        __syncthreads();
        const uint32_t pos = wcnt[w][d] + below;
        if (valid && pos < len) dst[pos] = key;
        __syncthreads();
      }
      uint32_t* tmp = src;
      src = dst;
      dst = tmp;
    }
    if (passes & 1) {  // result is in scratch: copy back
      for (uint32_t e = t; e < len; e += kThreads) ((uint32_t*)col)[s + e] = ((uint32_t*)scratch)[s + e];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ cut vector
// c_0 = 0, c_p = n; balanced: c_i = the smallest x > c_{i-1} with
// orow[x] >= ceil(i*m/p); uniform: c_i = floor(i*n/p).  Either is clamped
// into [c_{i-1}+1, n-(p-i)] so that no part is empty.
// The balanced searches are independent (the smallest x > c_{i-1} with
// orow[x] >= t_i is max(c_{i-1}+1, smallest x >= 1 with orow[x] >= t_i), as
// orow is non-decreasing), so they run in parallel; one thread then applies
// the clamps in order.
__global__ __launch_bounds__(kThreads) void k_cuts(const uint32_t* __restrict__ orow, int64_t n, int32_t p, int mode,
                                                   int32_t* __restrict__ cuts) {
  __shared__ int32_t c[kMaxP + 1];
  const uint64_t m = orow[n];
  for (int32_t i = threadIdx.x + 1; i < p; i += kThreads) {
    int64_t x;
    if (mode == BBTC_CUT_UNIFORM) {
      x = (int64_t)i * n / p;
    } else {
      const uint64_t target = ((uint64_t)i * m + (uint64_t)p - 1) / (uint64_t)p;
      int64_t lo = 1, hi = n;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((uint64_t)orow[mid] < target) lo = mid + 1; else hi = mid;
      }
      x = lo;
    }
    c[i] = (int32_t)x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t prev = 0;
    cuts[0] = 0;
    for (int32_t i = 1; i < p; ++i) {
      int64_t x = c[i];
      if (x < prev + 1) x = prev + 1;
      if (x > n - (p - i)) x = n - (p - i);
      cuts[i] = (int32_t)x;
      prev = x;
    }
    cuts[p] = (int32_t)n;
  }
}

// ------------------------------------------------------------ 16-bit out-rows
// Each column index relative to the first vertex of its part: for parts of
// at most 65536 vertices the counting kernels gather these two-byte entries
// instead of the four-byte ones.  Eight entries (two 16-byte loads, one
// 16-byte store) per thread; the part by binary search in the cut vector,
// staged in LDS.
__global__ __launch_bounds__(kThreads) void k_ocol16(const int32_t* __restrict__ ocol, uint64_t m,
                                                     const int32_t* __restrict__ cuts, int32_t p,
                                                     uint16_t* __restrict__ ocol16) {
  __shared__ int32_t sc[kMaxP + 1];
  for (int a = threadIdx.x; a <= p; a += kThreads) sc[a] = cuts[a];
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * kThreads * 8;
  for (uint64_t e0 = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) * 8; e0 < m; e0 += stride) {
    int32_t x[8];
    if (e0 + 8 <= m) {  // e0 is a multiple of 8: the loads are 32-byte aligned
      const int4 a0 = *reinterpret_cast<const int4*>(ocol + e0);
      const int4 a1 = *reinterpret_cast<const int4*>(ocol + e0 + 4);
      x[0] = a0.x; x[1] = a0.y; x[2] = a0.z; x[3] = a0.w;
      x[4] = a1.x; x[5] = a1.y; x[6] = a1.z; x[7] = a1.w;
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) x[t] = e0 + t < m ? ocol[e0 + t] : -1;
    }
    uint32_t h[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      h[t] = 0;
      if (x[t] >= 0) {
        const int32_t w = x[t];
        int lo = 0, hi = p;  // largest a with cuts[a] <= w
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (sc[mid] <= w) lo = mid; else hi = mid;
        }
        h[t] = (uint32_t)(w - sc[lo]) & 0xFFFFu;
      }
    }
    uint4 v;
    v.x = h[0] | (h[1] << 16);
    v.y = h[2] | (h[3] << 16);
    v.z = h[4] | (h[5] << 16);
    v.w = h[6] | (h[7] << 16);
    *reinterpret_cast<uint4*>(ocol16 + e0) = v;
  }
}

// ------------------------------------------------------------ in-rows by part
// The counting kernels need an in-row only grouped by the part of each entry
// (parts in increasing order), not sorted.  Listed rows (the long and huge
// ones left by k_segsort) are grouped by one counting pass per row: histogram
// of part ids in LDS, scan, scatter into scratch[rp[r] .. rp[r+1]) (rows own
// disjoint ranges), copy back.  The order inside a part is left to timing.
__device__ __forceinline__ int32_t part_of(const int32_t* scut, int32_t p, int32_t v) {
  int32_t lo = 0, hi = p - 1;  // largest a with scut[a] <= v
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (scut[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Exclusive scan of one value per thread over an NT-thread workgroup; `lds`
// needs NT/64 slots.  Contains barriers: call from uniform control flow.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan_n(uint32_t v, uint32_t* lds, uint32_t* total) {
  const int l = lane_id(), w = threadIdx.x / kWave;
  const uint32_t inc = wave_incl_scan_u32(v);
  if (l == kWave - 1) lds[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < NT / kWave; ++q) {
    const uint32_t x = lds[q];
    if (q < w) off += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

constexpr int kGroupUnroll = 4;  // entries per thread in flight in k_group_parts

// Rows whose combined list index (the huge rows, then the long ones after
// the *before huge rows) is below `taken` were grouped by the chunked
// kernels and are skipped.
template <int NT>
__global__ __launch_bounds__(NT) void k_group_parts(const uint32_t* __restrict__ rp, int32_t* __restrict__ col,
                                                    int32_t* __restrict__ scratch, const uint32_t* __restrict__ rows,
                                                    const uint32_t* __restrict__ nrows,
                                                    const int32_t* __restrict__ cuts, int32_t p,
                                                    const uint32_t* __restrict__ before, uint32_t taken) {
  __shared__ int32_t scut[kMaxP + 1];
  __shared__ uint32_t bins[kMaxP];
  __shared__ uint32_t lds[NT / kWave];
  const int t = threadIdx.x;
  for (int a = t; a <= p; a += NT) scut[a] = cuts[a];
  const uint32_t cnt = *nrows;
  const uint32_t b0 = before ? *before : 0u;
  const uint32_t first = taken > b0 ? taken - b0 : 0u;
  const int per = (p + NT - 1) / NT;  // bins per thread in the scan
  __syncthreads();
  for (uint32_t qi = first + blockIdx.x; qi < cnt; qi += gridDim.x) {
    const uint32_t r = rows[qi];
    const uint32_t s = rp[r], len = rp[r + 1] - s;
    for (int a = t; a < p; a += NT) bins[a] = 0;
    __syncthreads();
    for (uint32_t e0 = t; e0 < len; e0 += kGroupUnroll * NT) {
      int32_t v[kGroupUnroll];
#pragma unroll
      for (int k = 0; k < kGroupUnroll; ++k) v[k] = e0 + k * NT < len ? col[s + e0 + k * NT] : -1;
#pragma unroll
      for (int k = 0; k < kGroupUnroll; ++k)
        if (v[k] >= 0) atomicAdd(&bins[part_of(scut, p, v[k])], 1u);
    }
    __syncthreads();
    uint32_t sum = 0;
    for (int k = 0; k < per; ++k) {
      const int a = t * per + k;
      if (a < p) sum += bins[a];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan_n<NT>(sum, lds, &tot);
    for (int k = 0; k < per; ++k) {  // bins become the next free slot of each part
      const int a = t * per + k;
      if (a < p) {
        const uint32_t b = bins[a];
        bins[a] = off;
        off += b;
      }
    }
    __syncthreads();
    for (uint32_t e0 = t; e0 < len; e0 += kGroupUnroll * NT) {
      int32_t v[kGroupUnroll];
#pragma unroll
      for (int k = 0; k < kGroupUnroll; ++k) v[k] = e0 + k * NT < len ? col[s + e0 + k * NT] : -1;
#pragma unroll
      for (int k = 0; k < kGroupUnroll; ++k) {
        if (v[k] >= 0) {
          const uint32_t pos = atomicAdd(&bins[part_of(scut, p, v[k])], 1u);
          if (pos < len) scratch[s + pos] = v[k];
        }
      }
    }
    __syncthreads();
    for (uint32_t e = t; e < len; e += NT) col[s + e] = scratch[s + e];
    __syncthreads();
  }
}

// Chunked grouping of the long and huge in-rows: a hub's in-row (hundreds of
// thousands of entries) is cut into chunks of kGroupChunk entries spread
// over the whole chip instead of one workgroup per row.  The first `cap`
// rows of the combined list (huge rows, then long rows) take this path:
//   k_gchunk_list   the chunks (row index, chunk number), one thread per row,
//                   and clears those rows' counters and maps each row to its
//                   list index;
//   k_gchunk_count  per chunk, the entries of each part (LDS counts, then one
//                   global add per part into cnt[row * p + part]);
//   k_gchunk_scan   per row, cnt becomes the exclusive prefix over the parts
//                   (the start of each part within the row);
//   k_gchunk_scatter per chunk, recounted; each part's range is reserved by
//                   one global atomic on cnt and the entries are scattered
//                   into scratch (order within a part is free);
//   k_gchunk_copy   the rows back from scratch.
// Afterwards cnt[row * p + a] is the end of part a's run in the row (the
// block-major in side reads the slices from there instead of searching).
constexpr uint32_t kGroupChunk = kGroupChunkEntries;

__device__ __forceinline__ uint32_t glist_row(const uint32_t* longrows, const uint32_t* hugerows, uint32_t nhuge,
                                              uint32_t li) {
  return li < nhuge ? hugerows[li] : longrows[li - nhuge];
}

__global__ __launch_bounds__(kThreads) void k_gchunk_list(const uint32_t* __restrict__ rp,
                                                          const uint32_t* __restrict__ longrows,
                                                          const uint32_t* __restrict__ hugerows,
                                                          const uint32_t* __restrict__ q, uint32_t cap, int32_t p,
                                                          uint2* __restrict__ chunks, uint32_t* __restrict__ nchunks,
                                                          uint32_t* __restrict__ cnt, uint32_t* __restrict__ rowmap) {
  const uint32_t nhuge = q[1], nrows = min(q[0] + nhuge, cap);
  for (uint64_t x = blockIdx.x * kThreads + threadIdx.x; x < (uint64_t)nrows * p; x += gridDim.x * kThreads) cnt[x] = 0;
  for (uint32_t li = blockIdx.x * kThreads + threadIdx.x; li < nrows; li += gridDim.x * kThreads) {
    const uint32_t r = glist_row(longrows, hugerows, nhuge, li);
    rowmap[r] = li;
    const uint32_t len = rp[r + 1] - rp[r];
    const uint32_t nc = (len + kGroupChunk - 1) / kGroupChunk;
    const uint32_t at = atomicAdd(nchunks, nc);
    for (uint32_t c = 0; c < nc; ++c) chunks[at + c] = make_uint2(li, c);
  }
}

// Counts the parts of chunk (li, c) into bins (LDS, zero on entry); returns
// the row's start and length and the chunk's range.
__device__ __forceinline__ void gchunk_bins(const uint32_t* rp, const int32_t* col, const uint32_t* longrows,
                                            const uint32_t* hugerows, uint32_t nhuge, uint2 ch, const int32_t* scut,
                                            int32_t p, uint32_t* bins, uint32_t& s, uint32_t& len, uint32_t& e0,
                                            uint32_t& e1) {
  const uint32_t r = glist_row(longrows, hugerows, nhuge, ch.x);
  s = rp[r];
  len = rp[r + 1] - s;
  e0 = ch.y * kGroupChunk;
  e1 = min(len, e0 + kGroupChunk);
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += kThreads) atomicAdd(&bins[part_of(scut, p, col[s + e])], 1u);
}

__global__ __launch_bounds__(kThreads) void k_gchunk_count(const uint32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col,
                                                           const uint32_t* __restrict__ longrows,
                                                           const uint32_t* __restrict__ hugerows,
                                                           const uint32_t* __restrict__ q,
                                                           const uint2* __restrict__ chunks,
                                                           const uint32_t* __restrict__ nchunks,
                                                           const int32_t* __restrict__ cuts, int32_t p,
                                                           uint32_t* __restrict__ cnt) {
  extern __shared__ uint32_t lds_gc[];
  int32_t* scut = (int32_t*)lds_gc;  // p + 1
  uint32_t* bins = lds_gc + p + 1;   // p
  for (int a = threadIdx.x; a <= p; a += kThreads) scut[a] = cuts[a];
  const uint32_t nhuge = q[1], nc = *nchunks;
  for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
    for (int a = threadIdx.x; a < p; a += kThreads) bins[a] = 0;
    __syncthreads();
    const uint2 ch = chunks[c];
    uint32_t s, len, e0, e1;
    gchunk_bins(rp, col, longrows, hugerows, nhuge, ch, scut, p, bins, s, len, e0, e1);
    __syncthreads();
    for (int a = threadIdx.x; a < p; a += kThreads)
      if (bins[a]) atomicAdd(&cnt[(uint64_t)ch.x * p + a], bins[a]);
    __syncthreads();
  }
}

// One wavefront per row: cnt[row * p .. +p) becomes its exclusive prefix.
__global__ __launch_bounds__(kThreads) void k_gchunk_scan(const uint32_t* __restrict__ q, uint32_t cap, int32_t p,
                                                          uint32_t* __restrict__ cnt) {
  const uint32_t nrows = min(q[0] + q[1], cap);
  const uint32_t l = (uint32_t)lane_id();
  const uint32_t wave = (blockIdx.x * kThreads + threadIdx.x) / kWave, nwaves = gridDim.x * (kThreads / kWave);
  for (uint32_t li = wave; li < nrows; li += nwaves) {
    uint32_t* c = cnt + (uint64_t)li * p;
    uint32_t carry = 0;
    for (int32_t a0 = 0; a0 < p; a0 += kWave) {
      const int32_t a = a0 + (int32_t)l;
      const uint32_t v = a < p ? c[a] : 0u;
      const uint32_t inc = wave_incl_scan_u32(v);
      if (a < p) c[a] = carry + inc - v;
      carry += last_lane(inc);
    }
  }
}

// The chunk's entries are first placed part by part in an LDS buffer, then
// written out in that order, so that every part's run goes to consecutive
// positions of the row (coalesced) rather than entry by entry.
__global__ __launch_bounds__(kThreads) void k_gchunk_scatter(const uint32_t* __restrict__ rp,
                                                             const int32_t* __restrict__ col,
                                                             const uint32_t* __restrict__ longrows,
                                                             const uint32_t* __restrict__ hugerows,
                                                             const uint32_t* __restrict__ q,
                                                             const uint2* __restrict__ chunks,
                                                             const uint32_t* __restrict__ nchunks,
                                                             const int32_t* __restrict__ cuts, int32_t p,
                                                             uint32_t* __restrict__ cnt,
                                                             int32_t* __restrict__ scratch) {
  extern __shared__ uint32_t lds_gc[];
  int32_t* scut = (int32_t*)lds_gc;  // p + 1
  uint32_t* bins = lds_gc + p + 1;   // p: counts, then the next free slot of each part in buf
  uint32_t* lstart = bins + p;       // p: first slot of each part in buf
  uint32_t* gbase = lstart + p;      // p: position of the part's run in the row
  int32_t* buf = (int32_t*)(gbase + p);  // kGroupChunk
  __shared__ uint32_t red[kThreads / kWave];
  for (int a = threadIdx.x; a <= p; a += kThreads) scut[a] = cuts[a];
  const uint32_t nhuge = q[1], nc = *nchunks;
  const int per = (p + kThreads - 1) / kThreads;  // parts per thread in the scan
  for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
    for (int a = threadIdx.x; a < p; a += kThreads) bins[a] = 0;
    __syncthreads();
    const uint2 ch = chunks[c];
    uint32_t s, len, e0, e1;
    gchunk_bins(rp, col, longrows, hugerows, nhuge, ch, scut, p, bins, s, len, e0, e1);
    __syncthreads();
    uint32_t sum = 0;
    for (int k = 0; k < per; ++k) {
      const int a = threadIdx.x * per + k;
      if (a < p) sum += bins[a];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan_n<kThreads>(sum, red, &tot);
    for (int k = 0; k < per; ++k) {
      const int a = threadIdx.x * per + k;
      if (a < p) {
        const uint32_t n = bins[a];
        lstart[a] = off;
        gbase[a] = n ? atomicAdd(&cnt[(uint64_t)ch.x * p + a], n) : 0u;  // this chunk's run of part a
        bins[a] = off;
        off += n;
      }
    }
    __syncthreads();
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
      const int32_t v = col[s + e];
      buf[atomicAdd(&bins[part_of(scut, p, v)], 1u)] = v;
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < e1 - e0; t += kThreads) {
      const int32_t v = buf[t];
      const int32_t a = part_of(scut, p, v);
      const uint32_t pos = gbase[a] + (t - lstart[a]);
      if (pos < len) scratch[s + pos] = v;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_gchunk_copy(const uint32_t* __restrict__ rp, int32_t* __restrict__ col,
                                                          const uint32_t* __restrict__ longrows,
                                                          const uint32_t* __restrict__ hugerows,
                                                          const uint32_t* __restrict__ q,
                                                          const uint2* __restrict__ chunks,
                                                          const uint32_t* __restrict__ nchunks,
                                                          const int32_t* __restrict__ scratch) {
  const uint32_t nhuge = q[1], nc = *nchunks;
  for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const uint2 ch = chunks[c];
    const uint32_t r = glist_row(longrows, hugerows, nhuge, ch.x);
    const uint32_t s = rp[r], len = rp[r + 1] - s;
    const uint32_t e1 = min(len, (ch.y + 1) * kGroupChunk);
    for (uint32_t e = ch.y * kGroupChunk + threadIdx.x; e < e1; e += kThreads) col[s + e] = scratch[s + e];
  }
}

// ------------------------------------------------------------ block row index
// Workgroup per chunk of kPrepRows consecutive rows of one part; thread per
// row.  chunk0[a] is the first chunk of part a.
__device__ __forceinline__ int chunk_part(const int32_t* chunk0, int32_t p, int32_t c) {
  int lo = 0, hi = p;  // largest a with chunk0[a] <= c
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (chunk0[mid] <= c) lo = mid; else hi = mid;
  }
  return lo;
}

// First position in sorted col[ptr..re) whose value is >= key.
__device__ __forceinline__ uint32_t seek(const int32_t* __restrict__ col, uint32_t ptr, uint32_t re, int32_t key) {
  if (re - ptr > 16) {
    uint32_t lo = ptr, hi = re;
    while (lo < hi) {
      uint32_t mid = (lo + hi) >> 1;
      if (col[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
  }
  while (ptr < re && col[ptr] < key) ++ptr;
  return ptr;
}

// Out side: the row of u in part a gets its block boundaries for b = a..p
// (written for stored rows, u >= rT, only); per block the entries, the
// non-empty rows and the longest slice are counted for every row.  A row of
// at most kBotLane entries is walked by its own thread; longer rows are
// queued and taken by whole wavefronts (part_bounds_wave below; the row is
// sorted, so the boundary of block b is its first entry of a block >= b).
// Workgroups take chunks of kPrepRows rows in turn (grid-stride) and add
// their block counters to the global ones when their part changes and at the
// end.  LDS (dynamic, sized by p): per-block entry and row counters, the cut
// vector, one boundary row per wavefront and the long-row queue.
constexpr uint32_t kBotLane = 32;

// One wavefront: the slice boundaries of a row col[rb, re) whose entries lie
// in parts [first, last) in non-decreasing part order.  pos[x - first] is the
// first position holding a part >= x, for x in [first, last] (pos[0] = rb,
// pos[last - first] = re).  Rows of up to kWalkRow entries are walked 64
// entries at a time (kWalkUnroll steps loaded at once): the entry where the
// part changes is the boundary of every part in between.  Longer rows (a hub's in-row has hundreds of
// thousands of entries) are searched instead, one part per lane: the entries
// below c_x form a prefix of the row.  Ends with the wavefront's writes
// visible to it.
constexpr uint32_t kWalkRow = 2048;
constexpr uint32_t kWalkUnroll = 4;  // 64-entry steps of a walk loaded at once

__device__ __forceinline__ void part_bounds_wave(const int32_t* __restrict__ col, uint32_t rb, uint32_t re,
                                                 int32_t first, int32_t last, const int32_t* scut, int32_t p,
                                                 uint32_t* pos) {
  const int l = lane_id();
  if (re - rb <= kWalkRow) {
    int32_t carry = first;  // part of the entry before the current 64
    for (uint32_t q0 = rb; q0 < re; q0 += kWalkUnroll * kWave) {
      int32_t val[kWalkUnroll];  // kWalkUnroll loads in flight at once
#pragma unroll
      for (uint32_t h = 0; h < kWalkUnroll; ++h) {
        const uint32_t e = q0 + h * kWave + (uint32_t)l;
        val[h] = e < re ? col[e] : 0;
      }
#pragma unroll
      for (uint32_t h = 0; h < kWalkUnroll; ++h) {
        const uint32_t e = q0 + h * kWave + (uint32_t)l;
        const int32_t pe = e < re ? part_of(scut, p, val[h]) : last;
        int32_t prv = __shfl_up(pe, 1, kWave);
        if (l == 0) prv = carry;
        for (int32_t x = prv + 1; x <= pe; ++x) pos[x - first] = e;  // e = re for the first lane past the row
        carry = __shfl(pe, kWave - 1, kWave);
      }
    }
    for (int32_t x = carry + 1 + l; x <= last; x += kWave) pos[x - first] = re;  // rows ending on a multiple of 64
  } else {
    for (int32_t x = first + 1 + l; x < last; x += kWave) {
      const int32_t key = scut[x];
      uint32_t lo = rb, hi = re;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (col[mid] < key) lo = mid + 1; else hi = mid;
      }
      pos[x - first] = lo;
    }
    if (l == 0) pos[last - first] = re;
  }
  if (l == 0) pos[0] = rb;
  wave_sync();
}

__host__ __device__ constexpr size_t bot_lds_words(int32_t p) {
  return 2 * (size_t)p + 2 * (size_t)(p + 1) + 4 * (size_t)(p + 2) + kThreads + 4;
}

__global__ __launch_bounds__(kThreads) void k_bot(BlockBuild bb, int nchunks) {
  extern __shared__ uint32_t lds_bot[];
  const int32_t p = bb.p;
  uint32_t* s_nnz = lds_bot;                      // p
  uint32_t* s_nzr = s_nnz + p;                    // p
  int32_t* s_cut = (int32_t*)(s_nzr + p);         // p + 1
  uint32_t* s_pos = (uint32_t*)(s_cut + p + 1);   // 4 x (p + 2)
  uint32_t* s_q = s_pos + 4 * (p + 2);            // kThreads
  uint32_t* s_misc = s_q + kThreads;              // dmax, dfull, queue length
  int32_t* s_c0 = (int32_t*)(s_misc + 4);         // p + 1: first chunk of each part
  for (int b = threadIdx.x; b < p; b += kThreads) s_nnz[b] = s_nzr[b] = 0;
  for (int b = threadIdx.x; b <= p; b += kThreads) {
    s_cut[b] = bb.cuts[b];
    s_c0[b] = bb.chunk0[b];
  }
  if (threadIdx.x < 3) s_misc[threadIdx.x] = 0;
  __syncthreads();
  // the block counters of part `held` go out when the part changes (a
  // workgroup's chunks come in decreasing part order) and at the end: one
  // global add per workgroup and block instead of one per chunk
  int held = -1;
  auto flush = [&]() {
    const int64_t bid0 = block_id(p, held, held);
    for (int b = threadIdx.x; b < p - held; b += kThreads) {
      if (s_nnz[b]) {
        atomicAdd(&bb.bnnz[bid0 + b], (unsigned long long)s_nnz[b]);
        atomicAdd(&bb.bnzr[bid0 + b], (unsigned long long)s_nzr[b]);
      }
      s_nnz[b] = s_nzr[b] = 0;
    }
  };
  const int w = threadIdx.x / kWave, l = lane_id();
  uint32_t* pos = s_pos + w * (p + 2);  // pos[b - a]: boundary of block b, b = a..p
  for (int ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {
    // last chunk first: the last parts hold the hubs, whose long rows take
    // longest, so they start at once instead of trailing the launch
    const int chunk = nchunks - 1 - ci + bb.chunk_base;
    const int a = chunk_part(s_c0, p, chunk);
    if (a != held) {
      if (held >= 0) flush();
      held = a;
      __syncthreads();
    }
    const int lc = chunk - s_c0[a];
    const int64_t ca = s_cut[a];
    const int64_t sa = ca > bb.rT ? ca : (int64_t)bb.rT;  // first stored row of part a
    // column-major per part: entry b-a of row u at column (b-a), row u - sa
    const uint64_t ns = (uint64_t)(s_cut[a + 1] - sa);  // stored rows of part a
    const int64_t u = ca + (int64_t)lc * kPrepRows + threadIdx.x;
    const bool live = u < s_cut[a + 1];
    const uint32_t rb = live ? bb.orow[u] : 0u, re = live ? bb.orow[u + 1] : 0u;
    const bool walk = live && re - rb <= kBotLane;  // this thread's row; longer ones are queued
    if (live && !walk) s_q[atomicAdd(&s_misc[2], 1u)] = (uint32_t)threadIdx.x;
    {
      const uint32_t dfull = wave_max_u32(re - rb);
      if (l == 0 && dfull) atomicMax(&s_misc[1], dfull);
    }
    // every lane runs the block loop (walk or not) so that the per-block sums
    // over the wavefront's rows are formed by lane reductions: one LDS atomic
    // per wavefront and block instead of one per row
    uint32_t* out = walk && u >= sa ? bb.bot + bb.botp[a] + (uint64_t)(u - sa) : nullptr;
    if (out) out[0] = rb;
    const uint32_t rw = walk ? re : rb;  // the end of the walk (none for a queued row)
    uint32_t ptr = rb, prev = rb, dmax = 0;
    for (int b = a + 1; b <= p; ++b) {
      if (b == p) {
        ptr = rw;
      } else {
        const int32_t key = s_cut[b];
        while (ptr < rw && bb.ocol[ptr] < key) ++ptr;
      }
      if (out) out[(uint64_t)(b - a) * ns] = ptr;
      const uint32_t len = walk ? ptr - prev : 0u;
      const uint32_t rows = (uint32_t)__popcll(ballot(len != 0));
      if (rows) {
        const uint32_t sum = last_lane(wave_incl_scan_u32(len));
        if (l == 0) {
          atomicAdd(&s_nnz[b - 1 - a], sum);
          atomicAdd(&s_nzr[b - 1 - a], rows);
        }
      }
      dmax = len > dmax ? len : dmax;
      prev = ptr;
    }
    dmax = wave_max_u32(dmax);
    if (l == 0 && dmax) atomicMax(&s_misc[0], dmax);
    __syncthreads();
    // long rows, one wavefront each
    const uint32_t nq = s_misc[2];
    for (uint32_t h = w; h < nq; h += kThreads / kWave) {
      const int64_t v = ca + (int64_t)lc * kPrepRows + s_q[h];
      const uint32_t rb = bb.orow[v], re = bb.orow[v + 1];
      part_bounds_wave(bb.ocol, rb, re, a, p, s_cut, p, pos);  // entries lie in blocks a..p-1
      uint32_t* out = v >= sa ? bb.bot + bb.botp[a] + (uint64_t)(v - sa) : nullptr;
      uint32_t dmax = 0;
      for (int32_t b = a + l; b <= p; b += kWave) {
        const uint32_t pb = pos[b - a];
        if (out) out[(uint64_t)(b - a) * ns] = pb;
        if (b < p) {
          const uint32_t len = pos[b + 1 - a] - pb;
          if (len) {
            atomicAdd(&s_nnz[b - a], len);
            atomicAdd(&s_nzr[b - a], 1u);
            dmax = len > dmax ? len : dmax;
          }
        }
      }
      dmax = wave_max_u32(dmax);
      if (l == 0 && dmax) atomicMax(&s_misc[0], dmax);
      wave_sync();  // pos is rewritten by the next row
    }
    __syncthreads();
    if (threadIdx.x == 0) s_misc[2] = 0;  // the queue of the next chunk
    __syncthreads();
  }
  __syncthreads();
  if (held >= 0) flush();
  if (threadIdx.x == 0) {
    if (s_misc[0]) atomicMax(bb.dmax_block, s_misc[0]);
    if (s_misc[1]) atomicMax(bb.dmax_block + 1, s_misc[1]);
  }
}

// ------------------------------------------------------------ in side
// The ends of the part runs of in-row v (relative to its start) when the
// chunked grouping took the row, else null.
__device__ __forceinline__ const uint32_t* grouped_ends(const BlockBuild& bb, int64_t v) {
  if (bb.rowmap == nullptr) return nullptr;
  const uint32_t li = bb.rowmap[v];
  const uint32_t nhuge = bb.gq[1], nrows = min(bb.gq[0] + nhuge, bb.gcap);
  if (li >= nrows) return nullptr;
  const uint32_t r = li < nhuge ? bb.ghuge[li] : bb.glong[li - nhuge];
  return r == (uint32_t)v ? bb.gcnt + (uint64_t)li * (uint32_t)bb.p : nullptr;
}

// The in-side of the count is block-major: for block (a,b), in column-major
// block order, its active columns (v in V_b with an in-neighbour in V_a,
// ascending) in acol, and for active column x the in-slice of v from V_a at
// icolb[aoff[x] .. aoff[x+1]) (the block G_ab in compressed-column form with
// only its non-empty columns indexed).  Built from the in-rows (grouped by
// part): k_acount counts, per block and chunk of columns, the active columns
// and their entries; after two scans k_acol writes acol, aoff and the source
// position of each slice (asrc), and lists the hub columns (slices longer
// than `split`); k_icolb copies the slices.

// The in-slice [lo, hi) of in-row v from part a, given lo (the slice of part
// a starts where the one of part a-1 ended).
__device__ __forceinline__ uint32_t in_slice_end(const BlockBuild& bb, uint32_t lo, uint32_t re, int a, int na) {
  return (a + 1 == na) ? re : seek(bb.icol, lo, re, bb.cuts[a + 1]);
}

// Workgroups take chunks of 256 columns in turn (grid-stride), thread per
// column; in-rows longer than kBotLane are queued and taken by whole
// wavefronts (part_bounds_wave).  Per chunk the counts go to ccnt/ecnt; the
// active-column totals per block are summed in LDS and added to bnzc when the
// workgroup's part changes and at the end.  LDS (dynamic): per-block column,
// entry and total counters, the cut vector, a boundary row per wavefront, the
// queue.
__host__ __device__ constexpr size_t acount_lds_words(int32_t p) {
  return 3 * (size_t)p + 2 * (size_t)(p + 1) + 4 * (size_t)(p + 2) + kThreads + 4;
}

__global__ __launch_bounds__(kThreads) void k_acount(BlockBuild bb, int nchunks) {
  extern __shared__ uint32_t lds_ac[];
  const int32_t p = bb.p;
  uint32_t* s_nzc = lds_ac;                       // p: active columns of the chunk per block
  uint32_t* s_ent = s_nzc + p;                    // p: their entries
  uint32_t* s_tot = s_ent + p;                    // p: active columns of the held part per block
  int32_t* s_cut = (int32_t*)(s_tot + p);         // p + 1
  uint32_t* s_pos = (uint32_t*)(s_cut + p + 1);   // 4 x (p + 2)
  uint32_t* s_q = s_pos + 4 * (p + 2);            // kThreads
  uint32_t* s_misc = s_q + kThreads;              // queue length
  int32_t* s_c0 = (int32_t*)(s_misc + 4);         // p + 1: first chunk of each part
  for (int a = threadIdx.x; a < p; a += kThreads) s_nzc[a] = s_ent[a] = s_tot[a] = 0;
  for (int a = threadIdx.x; a <= p; a += kThreads) {
    s_cut[a] = bb.cuts[a];
    s_c0[a] = bb.chunk0[a];
  }
  if (threadIdx.x == 0) s_misc[0] = 0;
  __syncthreads();
  int held = -1;
  auto flush = [&]() {
    const int64_t cid0 = (int64_t)held * (held + 1) / 2;
    for (int a = threadIdx.x; a <= held; a += kThreads) {
      if (s_tot[a]) atomicAdd(&bb.bnzc[cid0 + a], (unsigned long long)s_tot[a]);
      s_tot[a] = 0;
    }
  };
  const int w = threadIdx.x / kWave, l = lane_id();
  uint32_t* pos = s_pos + w * (p + 2);
  for (int ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {
    // last chunk first: the last parts hold the hubs, whose long rows take
    // longest, so they start at once instead of trailing the launch
    const int chunk = nchunks - 1 - ci + bb.chunk_base;
    const int b = chunk_part(s_c0, p, chunk);
    if (b != held) {
      if (held >= 0) flush();
      held = b;
      __syncthreads();
    }
    const int lc = chunk - s_c0[b];
    const int nch = s_c0[b + 1] - s_c0[b];
    const int na = b + 1;  // blocks (0,b)..(b,b)
    const int64_t cb = s_cut[b];
    const int64_t v = cb + (int64_t)lc * kPrepRows + threadIdx.x;
    const bool live = v < s_cut[b + 1];
    uint32_t lo = live ? bb.irow[v] : 0u;
    const uint32_t re = live ? bb.irow[v + 1] : 0u;
    const bool walk = live && re - lo <= kBotLane;  // this thread's row; longer ones are queued
    if (live && !walk) s_q[atomicAdd(&s_misc[0], 1u)] = (uint32_t)threadIdx.x;
    // the wavefront walks its rows' parts together (until every row is done)
    // so that the per-block sums are formed by lane reductions: one LDS
    // atomic per wavefront and block instead of one per column
    const uint32_t rw = walk ? re : lo;
    for (int a = 0; a < na && ballot(lo < rw) != 0; ++a) {
      uint32_t hi = rw;
      if (a + 1 < na) {
        const int32_t key = s_cut[a + 1];
        hi = lo;
        while (hi < rw && bb.icol[hi] < key) ++hi;
      }
      const uint32_t len = hi - lo;
      const uint32_t cols = (uint32_t)__popcll(ballot(len != 0));
      if (cols) {
        const uint32_t sum = last_lane(wave_incl_scan_u32(len));
        if (l == 0) {
          atomicAdd(&s_nzc[a], cols);
          atomicAdd(&s_ent[a], sum);
        }
      }
      lo = hi;
    }
    __syncthreads();
    const uint32_t nq = s_misc[0];
    for (uint32_t h = w; h < nq; h += kThreads / kWave) {
      const int64_t x = cb + (int64_t)lc * kPrepRows + s_q[h];
      const uint32_t xb = bb.irow[x], xe = bb.irow[x + 1];
      const uint32_t* ends = xe - xb > kSegWave ? grouped_ends(bb, x) : nullptr;
      if (ends != nullptr) {  // a row grouped in chunks: its runs are known
        for (int32_t a = l; a < na; a += kWave) pos[a + 1] = xb + ends[a];
        if (l == 0) pos[0] = xb;
        wave_sync();
      } else {
        part_bounds_wave(bb.icol, xb, xe, 0, na, s_cut, p, pos);  // in-neighbours in parts 0..b
      }
      for (int32_t a = l; a < na; a += kWave) {
        const uint32_t len = pos[a + 1] - pos[a];
        if (len) {
          atomicAdd(&s_nzc[a], 1u);
          atomicAdd(&s_ent[a], len);
        }
      }
      wave_sync();  // pos is rewritten by the next row
    }
    __syncthreads();
    for (int a = threadIdx.x; a < na; a += kThreads) {
      const uint64_t q = bb.ccbase[b] + (uint64_t)a * nch + lc;
      bb.ccnt[q] = s_nzc[a];
      bb.ecnt[q] = s_ent[a];
      s_tot[a] += s_nzc[a];
      s_nzc[a] = s_ent[a] = 0;
    }
    if (threadIdx.x == 0) s_misc[0] = 0;
    __syncthreads();
  }
  if (held >= 0) flush();
}

// Writes, for every block (a,b), its active columns in increasing order at
// the offsets of the scanned chunk counters (ccoff: columns, ecoff: entries);
// positions are absolute in the plan's acol/aoff/icolb arrays (the arrays
// passed in are shifted accordingly when only some columns are resident).
__global__ __launch_bounds__(kThreads) void k_acol(BlockBuild bb) {
  __shared__ uint32_t lds[4];
  const int32_t p = bb.p;
  const int chunk = (int)blockIdx.x + bb.chunk_base;
  const int b = chunk_part(bb.chunk0, p, chunk);
  const int lc = chunk - bb.chunk0[b];
  const int nch = bb.chunk0[b + 1] - bb.chunk0[b];
  const int na = b + 1;
  const int64_t cb = bb.cuts[b];
  const int64_t v = cb + (int64_t)lc * kPrepRows + threadIdx.x;
  const bool valid = v < bb.cuts[b + 1];
  const uint32_t re = valid ? bb.irow[v + 1] : 0u;
  uint32_t lo = valid ? bb.irow[v] : 0u;
  const uint32_t rb = lo;
  const uint32_t* ends = valid && re - lo > kSegWave ? grouped_ends(bb, v) : nullptr;
  for (int a = 0; a < na; ++a) {
    const uint32_t hi = !(valid && lo < re) ? lo : ends != nullptr ? rb + ends[a] : in_slice_end(bb, lo, re, a, na);
    const uint32_t f = hi > lo ? 1u : 0u, len = hi - lo;
    uint32_t tot;
    const uint32_t off = block256_excl_scan<uint32_t>(f, lds, &tot);
    const uint32_t eoff = block256_excl_scan<uint32_t>(len, lds, &tot);
    if (f) {
      const uint64_t q = bb.ccbase[b] + (uint64_t)a * nch + lc;
      const uint64_t x = (uint64_t)bb.ccoff[q] + off;
      bb.acol[x] = (int32_t)v;
      bb.aoff[x] = bb.ebase + bb.ecoff[q] + eoff;
      bb.asrc[x] = lo;
      if (len > bb.split) {
        const uint32_t r = atomicAdd(bb.nheavy, 1u);
        if (r < bb.heavy_cap) bb.heavy[r] = HeavyCol{(uint32_t)col_block_id(a, b), (uint32_t)(bb.xbase + x), len};
      }
    }
    lo = hi;
  }
}

// Copies the in-slices of active columns [0, *ncolsp) (relative to the
// arrays passed in) into icolb: 64 columns per wavefront, their entries
// flattened over the lanes; slices longer than `split` are left to
// k_icolb_heavy.
__global__ __launch_bounds__(kThreads) void k_icolb(const uint32_t* __restrict__ aoff,
                                                    const uint32_t* __restrict__ asrc,
                                                    const int32_t* __restrict__ icol, int32_t* __restrict__ icolb,
                                                    const uint32_t* __restrict__ ncolsp, uint32_t split) {
  const uint64_t ncols = *ncolsp;
  __shared__ uint32_t off[kThreads / kWave][kWave + 1];
  __shared__ uint32_t src[kThreads / kWave][kWave];
  __shared__ uint32_t dst[kThreads / kWave][kWave];
  const int l = lane_id(), w = threadIdx.x / kWave;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t x0 = wave * kWave; x0 < (int64_t)ncols; x0 += nwaves * kWave) {  // uniform per wavefront
    const int64_t x = x0 + l;
    uint32_t len = 0, d0 = 0;
    if (x < (int64_t)ncols) {
      d0 = aoff[x];
      len = aoff[x + 1] - d0;
      if (len > split) len = 0;
    }
    const uint32_t inc = wave_incl_scan_u32(len);
    const uint32_t tot = last_lane(inc);
    off[w][l] = inc - len;
    src[w][l] = len ? asrc[x] : 0u;
    dst[w][l] = d0;
    wave_sync();
    for (uint32_t fb = 0; fb < tot; fb += kWave) {
      const uint32_t f = fb + l;
      if (f < tot) {
        const uint32_t o = owner_lane(off[w], f);
        const uint32_t t = f - off[w][o];
        icolb[dst[w][o] + t] = icol[src[w][o] + t];
      }
    }
    wave_sync();
  }
}

// One workgroup per hub column (slice longer than `split`), records
// [h0, min(*h1p, cap)): x is its absolute active-column index; xbase is the
// index of the first column of the arrays passed in.
__global__ __launch_bounds__(kThreads) void k_icolb_heavy(const HeavyCol* __restrict__ heavy, uint32_t h0,
                                                          const uint32_t* __restrict__ h1p, uint32_t cap,
                                                          uint64_t xbase, const uint32_t* __restrict__ aoff,
                                                          const uint32_t* __restrict__ asrc,
                                                          const int32_t* __restrict__ icol,
                                                          int32_t* __restrict__ icolb) {
  const uint32_t h1 = min(*h1p, cap);
  for (uint32_t h = h0 + blockIdx.x; h < h1; h += gridDim.x) {
    const uint64_t x = heavy[h].x - xbase;
    const uint32_t d = aoff[x], len = aoff[x + 1] - d, sp = asrc[x];
    for (uint32_t t = threadIdx.x; t < len; t += kThreads) icolb[d + t] = icol[sp + t];
  }
}

// W = sum over ranks r of in-degree(r) * out-degree(r): the number of
// oriented two-paths x -> r -> y, i.e. the probe volume of a per-vertex
// list count over the degree-ordered graph (the work measure of Sec. 4.4);
// and, for each of four degree thresholds, the number of ranks whose
// undirected degree is at most it, which is where stored block boundaries
// start for that threshold (degrees rise with rank).  Integer, so the order
// of the atomic additions does not matter.
__global__ __launch_bounds__(kThreads) void k_degree_stats(const uint32_t* __restrict__ od,
                                                           const uint32_t* __restrict__ idg, int64_t n, DegThresholds th,
                                                           unsigned long long* __restrict__ wedges,
                                                           uint32_t* __restrict__ nshort) {
  __shared__ unsigned long long red[4];
  unsigned long long acc = 0, cnt[4] = {0, 0, 0, 0};
  for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < n; r += (int64_t)gridDim.x * kThreads) {
    const uint32_t o = od[r], i = idg[r];
    acc += (unsigned long long)o * (unsigned long long)i;
    const int64_t d = (int64_t)o + (int64_t)i;
#pragma unroll
    for (int t = 0; t < 4; ++t) cnt[t] += d <= th.t[t] ? 1ull : 0ull;
  }
  acc = block256_sum_u64(acc, red);
#pragma unroll
  for (int t = 0; t < 4; ++t) cnt[t] = block256_sum_u64(cnt[t], red);
  if (threadIdx.x == 0) {
    if (acc) atomicAdd(wedges, acc);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (cnt[t]) atomicAdd(nshort + t, (uint32_t)cnt[t]);
  }
}

}  // namespace

// ------------------------------------------------------------ launchers
hipError_t launch_degree_stats(const uint32_t* od, const uint32_t* idg, int64_t n, const DegThresholds& th,
                               unsigned long long* wedges, uint32_t* nshort, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_degree_stats, dim3(grid_for((uint64_t)n, kThreads, 2048)), dim3(kThreads), 0, s, od, idg, n,
                     th, wedges, nshort);
  return hipGetLastError();
}

hipError_t launch_validate(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, int64_t nnz,
                           int symmetric, uint32_t* err, uint32_t* list, uint32_t* nlist, uint32_t* hlist,
                           uint32_t* nhlist, uint32_t* hpref, hipStream_t s) {
  const unsigned g = grid_for((uint64_t)n, kThreads, 65536);
  if (rp64) {
    hipLaunchKernelGGL(k_validate_lane<int64_t>, dim3(g), dim3(kThreads), 0, s, (const int64_t*)rowptr, colidx, n, nnz,
                       symmetric, err, list, nlist, hlist, nhlist);
    hipLaunchKernelGGL(k_hprefix<int64_t>, dim3(1), dim3(kThreads), 0, s, (const int64_t*)rowptr, (const uint32_t*)hlist,
                       (const uint32_t*)nhlist, hpref);
    hipLaunchKernelGGL(k_validate_wave<int64_t>, dim3(kRowGrid), dim3(kThreads), 0, s, (const int64_t*)rowptr, colidx,
                       n, nnz, symmetric, err, (const uint32_t*)list, (const uint32_t*)nlist, (const uint32_t*)hlist,
                       (const uint32_t*)nhlist, (const uint32_t*)hpref);
  } else {
    hipLaunchKernelGGL(k_validate_lane<int32_t>, dim3(g), dim3(kThreads), 0, s, (const int32_t*)rowptr, colidx, n, nnz,
                       symmetric, err, list, nlist, hlist, nhlist);
    hipLaunchKernelGGL(k_hprefix<int32_t>, dim3(1), dim3(kThreads), 0, s, (const int32_t*)rowptr, (const uint32_t*)hlist,
                       (const uint32_t*)nhlist, hpref);
    hipLaunchKernelGGL(k_validate_wave<int32_t>, dim3(kRowGrid), dim3(kThreads), 0, s, (const int32_t*)rowptr, colidx,
                       n, nnz, symmetric, err, (const uint32_t*)list, (const uint32_t*)nlist, (const uint32_t*)hlist,
                       (const uint32_t*)nhlist, (const uint32_t*)hpref);
  }
  return hipGetLastError();
}

hipError_t launch_degkey(const void* rowptr, int rp64, int64_t n, int idbits, uint64_t* keys, hipStream_t s) {
  if (n == 0) return hipSuccess;
  unsigned g = grid_for((uint64_t)n, kThreads, 65536);
  if (rp64)
    hipLaunchKernelGGL(k_degkey<int64_t>, dim3(g), dim3(kThreads), 0, s, (const int64_t*)rowptr, n, idbits, keys);
  else
    hipLaunchKernelGGL(k_degkey<int32_t>, dim3(g), dim3(kThreads), 0, s, (const int32_t*)rowptr, n, idbits, keys);
  return hipGetLastError();
}

size_t scan_partial_entries(uint64_t count) { return (size_t)((count + kScanTile - 1) / kScanTile) + 1; }

size_t radix_hist_entries(uint64_t count) {
  uint64_t ntiles = (count + kRadixTile - 1) / kRadixTile;
  return (size_t)(256 * ntiles + 1);
}

hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint64_t count, uint32_t* partial, hipStream_t s) {
  uint64_t nparts = (count + kScanTile - 1) / kScanTile;
  if (nparts == 0) {
    return hipMemsetAsync(out, 0, sizeof(uint32_t), s);
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nparts), dim3(kThreads), 0, s, in, count, partial);
  hipLaunchKernelGGL(k_scan_spine, dim3(1), dim3(kThreads), 0, s, partial, nparts, out + count);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nparts), dim3(kThreads), 0, s, in, out, count,
                     (const uint32_t*)partial);
  return hipGetLastError();
}

hipError_t radix_sort_u64(uint64_t* a, uint64_t* b, uint64_t count, int lo, int hi, uint32_t* hist,
                          uint32_t* partial, uint64_t** result, hipStream_t s) {
  uint64_t* src = a;
  uint64_t* dst = b;
  if (count > 1) {
    const uint64_t ntiles = (count + kRadixTile - 1) / kRadixTile;
    for (int shift = lo; shift < hi; shift += 8) {
      hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(kThreads), 0, s, src, count, shift, hist,
                         (uint32_t)ntiles);
      hipError_t e = scan_u32(hist, hist, 256 * ntiles, partial, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(kThreads), 0, s, src, dst, count, shift,
                         hist, (uint32_t)ntiles);
      std::swap(src, dst);
    }
  }
  *result = src;
  return hipGetLastError();
}

hipError_t launch_perm(const uint64_t* keys, int64_t n, int idbits, int32_t* order, int32_t* perm, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t mask = (idbits >= 64) ? ~0ull : ((1ull << idbits) - 1);
  hipLaunchKernelGGL(k_perm, dim3(grid_for((uint64_t)n, kThreads, 65536)), dim3(kThreads), 0, s, keys, n, mask, order,
                     perm);
  return hipGetLastError();
}

hipError_t launch_degs(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, const RowRange& rr,
                       const int32_t* perm, uint32_t* od, uint32_t* idg, uint32_t* list, uint32_t* nlist,
                       uint32_t* hlist, uint32_t* nhlist, uint32_t* hpref, uint32_t* err, int check, int32_t* rc,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned g = grid_for((uint64_t)n, kThreads, 65536);
  if (rp64) {
    hipLaunchKernelGGL(k_degs_lane<int64_t>, dim3(g), dim3(kThreads), 0, s, (const int64_t*)rowptr, colidx, n, rr,
                       perm, od, idg, list, nlist, hlist, nhlist, err, check, rc);
    hipLaunchKernelGGL(k_hprefix<int64_t>, dim3(1), dim3(kThreads), 0, s, (const int64_t*)rowptr, (const uint32_t*)hlist,
                       (const uint32_t*)nhlist, hpref);
    if (od)
      hipLaunchKernelGGL(k_degs_wave<int64_t>, dim3(kRowGrid), dim3(kThreads), 0, s, (const int64_t*)rowptr, colidx,
                         rr, perm, od, idg, (const uint32_t*)list, (const uint32_t*)nlist, (const uint32_t*)hlist,
                         (const uint32_t*)nhlist, (const uint32_t*)hpref, err, check, rc);
  } else {
    hipLaunchKernelGGL(k_degs_lane<int32_t>, dim3(g), dim3(kThreads), 0, s, (const int32_t*)rowptr, colidx, n, rr,
                       perm, od, idg, list, nlist, hlist, nhlist, err, check, rc);
    hipLaunchKernelGGL(k_hprefix<int32_t>, dim3(1), dim3(kThreads), 0, s, (const int32_t*)rowptr, (const uint32_t*)hlist,
                       (const uint32_t*)nhlist, hpref);
    if (od)
      hipLaunchKernelGGL(k_degs_wave<int32_t>, dim3(kRowGrid), dim3(kThreads), 0, s, (const int32_t*)rowptr, colidx,
                         rr, perm, od, idg, (const uint32_t*)list, (const uint32_t*)nlist, (const uint32_t*)hlist,
                         (const uint32_t*)nhlist, (const uint32_t*)hpref, err, check, rc);
  }
  return hipGetLastError();
}

hipError_t launch_fill(const void* rowptr, int rp64, const int32_t* colidx, int64_t n, const RowRange& rr,
                       const int32_t* perm,
                       const uint32_t* orow, const uint32_t* irow, int32_t* ocol, int32_t* icol, const uint32_t* list,
                       const uint32_t* nlist, const uint32_t* hlist, const uint32_t* nhlist, const uint32_t* hpref,
                       uint32_t* cur_o, uint32_t* cur_i, const int32_t* rc, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned g = grid_for((uint64_t)n, kThreads, 65536);
  hipLaunchKernelGGL(k_zero2, dim3(64), dim3(kThreads), 0, s, cur_o, cur_i, nhlist);
  if (rp64) {
    hipLaunchKernelGGL(k_fill_lane<int64_t>, dim3(g), dim3(kThreads), 0, s, (const int64_t*)rowptr, colidx, n, rr,
                       perm, orow, irow, ocol, icol, rc);
    hipLaunchKernelGGL(k_fill_wave<int64_t>, dim3(kRowGrid), dim3(kThreads), 0, s, (const int64_t*)rowptr, colidx, rr,
                       perm, orow, irow, ocol, icol, list, nlist, hlist, nhlist, hpref, cur_o, cur_i, rc);
  } else {
    hipLaunchKernelGGL(k_fill_lane<int32_t>, dim3(g), dim3(kThreads), 0, s, (const int32_t*)rowptr, colidx, n, rr,
                       perm, orow, irow, ocol, icol, rc);
    hipLaunchKernelGGL(k_fill_wave<int32_t>, dim3(kRowGrid), dim3(kThreads), 0, s, (const int32_t*)rowptr, colidx, rr,
                       perm, orow, irow, ocol, icol, list, nlist, hlist, nhlist, hpref, cur_o, cur_i, rc);
  }
  return hipGetLastError();
}

hipError_t launch_segsort(const uint32_t* rp, int32_t* col, int64_t nrows, int bits, uint32_t* midrows,
                          uint32_t* longrows, uint32_t* hugerows, uint32_t* q, int32_t* scratch, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_segsort, dim3(grid_for((uint64_t)nrows, kThreads, kRowGrid)), dim3(kThreads), 0, s, rp, col,
                     nrows, midrows, longrows, hugerows, q);
  hipLaunchKernelGGL(k_segsort_mid, dim3(kRowGrid), dim3(kThreads), 0, s, rp, col, (const uint32_t*)midrows,
                     (const uint32_t*)q);
  hipLaunchKernelGGL(k_segsort_long, dim3(1024), dim3(kThreads), 0, s, rp, col, (const uint32_t*)longrows,
                     (const uint32_t*)q);
  hipLaunchKernelGGL(k_segsort_huge, dim3(256), dim3(kThreads), 0, s, rp, col, scratch, (const uint32_t*)hugerows,
                     (const uint32_t*)q, bits);
  return hipGetLastError();
}

hipError_t launch_cuts(const uint32_t* orow, int64_t n, int32_t p, int mode, int32_t* cuts, hipStream_t s) {
  hipLaunchKernelGGL(k_cuts, dim3(1), dim3(kThreads), 0, s, orow, n, p, mode, cuts);
  return hipGetLastError();
}

hipError_t launch_inrows_sort(const uint32_t* rp, int32_t* col, int64_t nrows, uint32_t* midrows, uint32_t* longrows,
                              uint32_t* hugerows, uint32_t* q, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_segsort, dim3(grid_for((uint64_t)nrows, kThreads, kRowGrid)), dim3(kThreads), 0, s, rp, col,
                     nrows, midrows, longrows, hugerows, q);
  hipLaunchKernelGGL(k_segsort_mid, dim3(kRowGrid), dim3(kThreads), 0, s, rp, col, (const uint32_t*)midrows,
                     (const uint32_t*)q);
  return hipGetLastError();
}

hipError_t launch_inrows_group(const uint32_t* rp, int32_t* col, const uint32_t* longrows, const uint32_t* hugerows,
                               const uint32_t* q, int32_t* scratch, const int32_t* cuts, int32_t p,
                               const GroupChunks& gc, hipStream_t s) {
  if (gc.cap > 0) {
    const size_t lds = sizeof(uint32_t) * (2 * (size_t)p + 1);
    const unsigned g = gc.max_chunks < 2048u ? (gc.max_chunks > 0 ? gc.max_chunks : 1u) : 2048u;
    const unsigned gl = gc.cap / kThreads + 1 < 256u ? gc.cap / kThreads + 1 : 256u;
    hipLaunchKernelGGL(k_gchunk_list, dim3(gl), dim3(kThreads), 0, s, rp, longrows, hugerows, q, gc.cap, p,
                       gc.chunks, gc.nchunks, gc.cnt, gc.rowmap);
    hipLaunchKernelGGL(k_gchunk_count, dim3(g), dim3(kThreads), lds, s, rp, (const int32_t*)col, longrows, hugerows, q,
                       (const uint2*)gc.chunks, (const uint32_t*)gc.nchunks, cuts, p, gc.cnt);
    hipLaunchKernelGGL(k_gchunk_scan, dim3(gl), dim3(kThreads), 0, s, q, gc.cap, p, gc.cnt);
    const size_t lds_s = sizeof(uint32_t) * (4 * (size_t)p + 1 + kGroupChunk);
    hipLaunchKernelGGL(k_gchunk_scatter, dim3(g), dim3(kThreads), lds_s, s, rp, (const int32_t*)col, longrows,
                       hugerows, q, (const uint2*)gc.chunks, (const uint32_t*)gc.nchunks, cuts, p, gc.cnt, scratch);
    hipLaunchKernelGGL(k_gchunk_copy, dim3(g), dim3(kThreads), 0, s, rp, col, longrows, hugerows, q,
                       (const uint2*)gc.chunks, (const uint32_t*)gc.nchunks, (const int32_t*)scratch);
    if (gc.all_taken) return hipGetLastError();
  }
  hipLaunchKernelGGL(k_group_parts<kThreads>, dim3(1024), dim3(kThreads), 0, s, rp, col, scratch, longrows, q, cuts, p,
                     q + 1, gc.cap);
  hipLaunchKernelGGL(k_group_parts<1024>, dim3(256), dim3(1024), 0, s, rp, col, scratch, hugerows, q + 1, cuts, p,
                     (const uint32_t*)nullptr, gc.cap);
  return hipGetLastError();
}

hipError_t launch_bot(const BlockBuild& bb, int nchunks, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bot, dim3(nchunks < 2048 ? nchunks : 2048), dim3(kThreads), sizeof(uint32_t) * bot_lds_words(bb.p),
                     s, bb, nchunks);
  return hipGetLastError();
}

hipError_t launch_acount(const BlockBuild& bb, int nchunks, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_acount, dim3(nchunks < 2048 ? nchunks : 2048), dim3(kThreads),
                     sizeof(uint32_t) * acount_lds_words(bb.p), s, bb, nchunks);
  return hipGetLastError();
}

hipError_t launch_acol(const BlockBuild& bb, int nchunks, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_acol, dim3(nchunks), dim3(kThreads), 0, s, bb);
  return hipGetLastError();
}

hipError_t launch_icolb(const uint32_t* aoff, const uint32_t* asrc, const int32_t* icol, int32_t* icolb,
                        const uint32_t* ncolsp, uint64_t ncols_max, uint32_t split, const HeavyCol* heavy, uint32_t h0,
                        const uint32_t* h1p, uint32_t cap, uint64_t xbase, hipStream_t s) {
  if (ncols_max > 0)
    hipLaunchKernelGGL(k_icolb, dim3(grid_for(ncols_max, kThreads, kRowGrid)), dim3(kThreads), 0, s, aoff, asrc, icol,
                       icolb, ncolsp, split);
  if (cap > h0)
    hipLaunchKernelGGL(k_icolb_heavy, dim3(1024), dim3(kThreads), 0, s, heavy, h0, h1p, cap, xbase, aoff, asrc, icol,
                       icolb);
  return hipGetLastError();
}

__global__ void k_set_at(uint32_t* __restrict__ arr, const uint32_t* __restrict__ idx, uint32_t value) {
  if (threadIdx.x == 0) arr[*idx] = value;
}

hipError_t launch_ocol16(const int32_t* ocol, uint64_t m, const int32_t* cuts, int32_t p, uint16_t* ocol16,
                         hipStream_t s) {
  if (m == 0) return hipSuccess;
  const uint64_t groups = (m + 8ull * kThreads - 1) / (8ull * kThreads);
  hipLaunchKernelGGL(k_ocol16, dim3((unsigned)std::min<uint64_t>(groups, 65536)), dim3(kThreads), 0, s, ocol, m, cuts,
                     p, ocol16);
  return hipGetLastError();
}

// Dense slices as bitmaps over the (row u, block k) pairs, u in [c_k0, n),
// k in [k0, p), 64 pairs per wavefront, a lane each: the slice N(G_ik,u)
// comes from the stored boundaries (or two searches of a row without them).
// A slice of at least |V_k|/16 entries (where a bitmap of V_k is no larger
// than the 16-bit list) is then built by the whole wavefront, bit by bit in
// its LDS words, and written out whole.
__global__ __launch_bounds__(kThreads) void k_dense_build(const uint32_t* __restrict__ orow,
                                                          const int32_t* __restrict__ ocol,
                                                          const uint16_t* __restrict__ ocol16,
                                                          const uint32_t* __restrict__ bot,
                                                          const uint64_t* __restrict__ botp,
                                                          const int32_t* __restrict__ cuts, int32_t p, int32_t rT,
                                                          int32_t k0, int64_t n, uint32_t* __restrict__ dslot,
                                                          uint32_t* __restrict__ dbits, uint32_t* __restrict__ nwords,
                                                          uint64_t cap) {
  __shared__ uint32_t bm[kThreads / kWave][kDenseRows / 32];
  __shared__ int32_t scut[kMaxP + 1];
  for (int a = threadIdx.x; a <= p; a += kThreads) scut[a] = cuts[a];
  __syncthreads();
  const int w = threadIdx.x / kWave, l = lane_id();
  uint32_t* b = bm[w];
  const int64_t u0 = scut[k0], nk = p - k0;
  const int64_t npairs = (n - u0) * nk;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t x0 = wave * kWave; x0 < npairs; x0 += nwaves * kWave) {  // uniform per wavefront
    const int64_t x = x0 + l;
    uint32_t a0 = 0, a1 = 0, vk = 0;
    if (x < npairs) {
      const int64_t u = u0 + x / nk;
      const int32_t k = k0 + (int32_t)(x % nk);
      const int32_t a = part_of(scut, p, (int32_t)u);
      vk = (uint32_t)(scut[k + 1] - scut[k]);
      if (k >= a) {
        if (u >= rT) {
          const int64_t sa = scut[a] > rT ? scut[a] : rT;
          const uint64_t ns = (uint64_t)(scut[a + 1] - sa);
          const uint32_t* col0 = bot + botp[a] + (uint64_t)(k - a) * ns + (uint64_t)(u - sa);
          a0 = col0[0];
          a1 = col0[ns];
        } else {
          const uint32_t re = orow[u + 1];
          uint32_t lo = orow[u], hi = re;
          while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (ocol[mid] < scut[k]) lo = mid + 1; else hi = mid;
          }
          a0 = lo;
          hi = re;
          while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (ocol[mid] < scut[k + 1]) lo = mid + 1; else hi = mid;
          }
          a1 = lo;
        }
      }
    }
    const bool dense = a1 > a0 && vk <= (uint32_t)kDenseRows && 16ull * (a1 - a0) >= vk;
    uint32_t slot = 0;
    for (uint64_t mask = ballot(dense); mask != 0; mask &= mask - 1) {  // the dense pairs in turn
      const int src = __ffsll((long long)mask) - 1;
      const uint32_t s0 = __shfl(a0, src, kWave), s1 = __shfl(a1, src, kWave), sv = __shfl(vk, src, kWave);
      const uint32_t words = ((sv + 31) / 32 + 7) & ~7u;
      uint32_t off = 0;
      if (l == 0) off = atomicAdd(nwords, words);
      off = __shfl(off, 0, kWave);
      if ((uint64_t)off + words > cap) continue;  // the bound holds; never taken
      for (uint32_t t = l; t < words; t += kWave) b[t] = 0;
      wave_sync();
      for (uint32_t e = s0 + l; e < s1; e += kWave) {
        const uint32_t v = ocol16[e];
        atomicOr(&b[v >> 5], 1u << (v & 31));
      }
      wave_sync();
      for (uint32_t t = l; t < words; t += kWave) dbits[off + t] = b[t];
      wave_sync();
      if (l == src) slot = off + 1;
      if (l == 0) atomicAdd(nwords + 1, 1u);
    }
    if (x < npairs) dslot[x] = slot;
  }
}

hipError_t launch_dense_build(const uint32_t* orow, const int32_t* ocol, const uint16_t* ocol16, const uint32_t* bot,
                              const uint64_t* botp, const int32_t* cuts, int32_t p, int32_t rT, int32_t k0, int64_t n,
                              int64_t npairs, uint32_t* dslot, uint32_t* dbits, uint32_t* nwords, uint64_t cap,
                              hipStream_t s) {
  if (k0 >= p || npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_build, dim3((unsigned)std::min<int64_t>(1024, npairs / kThreads + 1)), dim3(kThreads), 0,
                     s, orow, ocol, ocol16, bot, botp, cuts, p, rT, k0,
                     n, dslot, dbits, nwords, cap);
  return hipGetLastError();
}

hipError_t launch_set_at(uint32_t* arr, const uint32_t* idx, uint32_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_at, dim3(1), dim3(64), 0, s, arr, idx, value);
  return hipGetLastError();
}

namespace {

// One thread per emitted item.
__global__ __launch_bounds__(kThreads) void k_emit_items(const ItemRun* __restrict__ runs, int32_t nruns,
                                                         const TaskItems* __restrict__ ti,
                                                         const uint32_t* __restrict__ hstart,
                                                         const HeavyCol* __restrict__ hrec,
                                                         const uint32_t* __restrict__ hcum, uint32_t chunk,
                                                         DevItem* __restrict__ out, uint32_t nitems) {
  const uint32_t pos = blockIdx.x * kThreads + threadIdx.x;
  if (pos >= nitems) return;
  int32_t a = 0, b = nruns - 1;  // the last run starting at or before pos
  while (a < b) {
    const int32_t mid = (a + b + 1) >> 1;
    if (runs[mid].dst <= pos) a = mid; else b = mid - 1;
  }
  const ItemRun ru = runs[a];
  const uint32_t r = ru.r0 + (pos - ru.dst);
  const TaskItems t = ti[ru.task];
  DevItem it;
  it.task = ru.task;
  if (r < t.nhub) {
    uint32_t x = hstart[t.cid], y = hstart[t.cid + 1] - 1;  // the record whose chunks hold r
    while (x < y) {
      const uint32_t mid = (x + y + 1) >> 1;
      if (hcum[mid] <= r) x = mid; else y = mid - 1;
    }
    const HeavyCol hc = hrec[x];
    it.lo = (r - hcum[x]) * chunk;
    it.hi = min(hc.cnt, it.lo + chunk);
    it.v = (int32_t)hc.x;
  } else {
    it.lo = (r - t.nhub) * t.nper;
    it.hi = min(t.cols, it.lo + t.nper);
    it.v = -1;
  }
  out[pos] = it;
}

}  // namespace

hipError_t launch_emit_items(const ItemRun* runs, int32_t nruns, const TaskItems* ti, const uint32_t* hstart,
                             const HeavyCol* hrec, const uint32_t* hcum, uint32_t chunk, DevItem* out,
                             uint32_t nitems, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(k_emit_items, dim3((nitems + kThreads - 1) / kThreads), dim3(kThreads), 0, s, runs, nruns, ti,
                     hstart, hrec, hcum, chunk, out, nitems);
  return hipGetLastError();
}

}  // namespace bbtc
