// Per-task triangle counting kernels (arXiv 2009.12457, Sec. 4.3).
//
// A task {i,j,k} sums |N(G_ik,u) cap N(G_jk,v)| over the edges (u,v) of G_ij.
// The kernels visit those edges grouped by their head v (the columns of G_ij
// that have an in-neighbour in V_i, from the active-column list) rather than
// by their tail u: the sum is the same, and the list N(G_jk,v), which is the
// long one under degree ordering, is staged once per v and probed by the
// short lists N(G_ik,u) of all of v's in-neighbours u in V_i.
//
// Three mappings (tuning knobs; all exact):
//   * short columns (|N(G_jk,v)| < wave_min): the columns of one pass of the
//     workgroup are packed and split into four runs, one per wavefront; a
//     wavefront copies the sorted lists of a window of its columns side by
//     side into its LDS stage and flattens the probes of all their
//     in-neighbours over its 64 lanes (segments of kSegW entries, each
//     lane's owner from per-round start marks and a DPP running maximum),
//     each probe a binary search in its own column's run;
//   * long columns: one 64-lane wavefront per v stages N(G_jk,v) alone and
//     the lanes share the probes of all in-neighbours u (the same segments,
//     handed out by a wavefront prefix sum);
//   * hub columns (in-slice longer than `split`): the host cuts the in-slice
//     into chunks that are separate work items; a whole workgroup stages
//     N(G_jk,v) once and its four wavefronts share the chunk's in-neighbours.
// A column's own stage is either the Intersect form (a sorted LDS copy,
// binary search) or the HMap form (a dense LDS bitmap over the columns of
// V_k -- the paper's dense hash map of the block's column range -- or, when
// V_k is too wide for LDS, an open-addressing LDS hash).  Lists longer than
// the LDS buffer are staged in disjoint pieces; a probe matches at most one
// piece, so the count stays exact.
#include "bbtc_internal.h"
#include "dev_common.h"

namespace bbtc {

namespace {

#ifndef BBTC_STAGE_WORDS
#define BBTC_STAGE_WORDS 512
#endif
constexpr int kABuf = BBTC_STAGE_WORDS;       // LDS words per wavefront
constexpr uint32_t kGroupWords = 4 * kABuf;   // the four wavefront buffers as one workgroup stage
constexpr int log2i(int x) { return x <= 1 ? 0 : 1 + log2i(x / 2); }
static_assert((1 << log2i(kABuf)) == kABuf, "stage size must be a power of two");

// Out-rows are read in 16-byte aligned blocks of kSeg entries, by single
// 128-bit loads (the blocks of N(G_ik,u) are aligned on the absolute
// positions of the oriented CSR, whose base is 16-byte aligned).
constexpr uint32_t kSeg = 4;

struct WaveScratch {        // per wave: one batch of 64 in-neighbours
  uint32_t sa0[4][kWave];   // start of N(G_ik,u)
  uint32_t sa1[4][kWave];   // end of N(G_ik,u)
  uint32_t sex[4][kWave];   // exclusive prefix of the segment counts
  uint32_t scol[4][kWave];  // short columns: the packed column of u
  uint32_t sown[4][kWave];  // owner marks of a probe round
};

struct CountLds {
  // first member, and the struct aligned to 4 kGroupWords bytes: every stage
  // buffer starts at a multiple of its own size (bitmap loads OR their offset in)
  uint32_t abuf[4][kABuf];         // per wave: sorted copy / bitmap / hash; all-zero between uses
  WaveScratch w;
  uint32_t c0s[kThreads];          // short columns of a pass, packed: start of N(G_jk,v)
  uint32_t i0s[kThreads];          // start of the in-slice
  uint32_t soff[kThreads + 1];     // exclusive prefix of list lengths
  uint32_t ioff[kThreads + 1];     // exclusive prefix of in-slice lengths
  uint32_t q[kThreads];            // long columns of a pass (active-column index): from the
                                   // front those of one wavefront, from the back the wide ones
  uint32_t qn, qw;
  uint32_t item;
  unsigned long long red[4];
};

struct TaskCtx {
  int32_t ci, ci1, cj, ck, ck1;
  int32_t kb;               // ck rounded down to a multiple of 32 (the bitmap covers [kb, ck1))
  int32_t i, dk, dkj;       // i, k-i, k-j
  int32_t si, sj;           // first rows of parts i and j with stored boundaries
  // stored boundaries, column-major per part: column b holds, for every
  // stored row, the first position of block b; column k and k+1 of part i
  // (bik0, bik1) bound N(G_ik,u), those of part j (bjk0, bjk1) N(G_jk,v),
  // indexed by the row's rank minus si (sj)
  const uint32_t* bik0;
  const uint32_t* bik1;
  const uint32_t* bjk0;
  const uint32_t* bjk1;
  const uint32_t* orow;
  const int32_t* coli;      // out-rows of part i (N(G_ik,u)), absolute positions
  const int32_t* colj;      // out-rows of part j (N(G_jk,v)), absolute positions
  const int32_t* icolj;     // block-major in-side, absolute positions
  const int32_t* acb;       // active columns, absolute indices
  const uint32_t* aob;      // their in-slice offsets, absolute indices
  const uint16_t* col16;    // resident plans with |V_k| <= 65536: out-rows relative to c_k (else null)
  // dense slices of block k as bitmaps over V_k (16-bit tasks only; else
  // dslot null): slot of row u at dslot[(u - du0) * dnk], dwords words each
  const uint32_t* dslot;
  const uint32_t* dbits;
  int32_t du0;
  uint32_t dnk, dwords;
  const int32_t* ac;        // active columns of block (i,j): acb + acp[cid(i,j)]
  const uint32_t* ao;       // their in-slice offsets (one more entry than columns)
};

// Read through the constant address space: with a wave-uniform address this
// is a scalar load into scalar registers.  Only for data that no kernel
// writes while the count runs (plan tables, items, graph arrays).
template <class T>
__device__ __forceinline__ T ld_const(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized records only");
  typedef const __attribute__((address_space(4))) uint32_t* cword;
  const cword q = (cword)p;
  T r;
  uint32_t* d = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
  for (uint32_t x = 0; x < sizeof(T) / 4; ++x) d[x] = q[x];
  return r;
}

__device__ __forceinline__ TaskCtx make_ctx(const GraphView& g, const DevTask& t) {
  TaskCtx c;
  c.ci = ld_const(g.cuts + t.i);
  c.ci1 = ld_const(g.cuts + t.i + 1);
  c.cj = ld_const(g.cuts + t.j);
  c.ck = ld_const(g.cuts + t.k);
  c.ck1 = ld_const(g.cuts + t.k + 1);
  c.kb = c.ck & ~31;
  c.i = t.i;
  c.dk = t.k - t.i;
  c.dkj = t.k - t.j;
  c.si = max(c.ci, g.rT);
  c.sj = max(c.cj, g.rT);
  // stored rows of parts i and j: the column length of their boundary tables
  const uint32_t ni = (uint32_t)max(c.ci1 - c.si, 0), nj = (uint32_t)max(ld_const(g.cuts + t.j + 1) - c.sj, 0);
  c.orow = g.orow;
  if (g.gi >= 0) {  // streamed: the launch's parts come from cached stripes
    c.bik0 = g.botI;
    c.bjk0 = g.botJ;
    c.coli = g.colI;
    c.colj = g.colJ;
    c.icolj = g.icolJ;
    c.acb = g.acolJ;
    c.aob = g.aoffJ;
  } else {
    c.bik0 = g.bot + ld_const(g.botp + t.i);
    c.bjk0 = g.bot + ld_const(g.botp + t.j);
    c.coli = g.ocol;
    c.colj = g.ocol;
    c.icolj = g.icol;
    c.acb = g.acol;
    c.aob = g.aoff;
  }
  c.bik0 += (uint64_t)c.dk * ni;
  c.bik1 = c.bik0 + ni;
  c.bjk0 += (uint64_t)c.dkj * nj;
  c.bjk1 = c.bjk0 + nj;
  c.col16 = (g.gi < 0 && g.ocol16 != nullptr && c.ck1 - c.ck <= 65536) ? g.ocol16 : nullptr;
  c.dslot = nullptr;
  c.dbits = g.dbits;
  c.du0 = g.dense_u0;
  c.dnk = (uint32_t)(g.p - g.dense_k0);
  c.dwords = ((uint32_t)(c.ck1 - c.ck + 31) / 32 + 7) & ~7u;
  if (c.col16 != nullptr && g.dslot != nullptr && t.k >= g.dense_k0) c.dslot = g.dslot + (t.k - g.dense_k0);
  const uint64_t a0 = ld_const(g.acp + col_block_id(t.i, t.j));
  c.ac = c.acb + a0;
  c.ao = c.aob + a0;
  return c;
}

__device__ __forceinline__ uint32_t hash_slot(uint32_t w, int hbits) { return (w * 0x9E3779B1u) >> (32 - hbits); }

// LDS byte address of a pointer into shared memory, and a load from one.
typedef __attribute__((address_space(3))) const uint32_t* lds_cptr;
__device__ __forceinline__ uint32_t lds_addr(const uint32_t* p) { return (uint32_t)(uintptr_t)(lds_cptr)p; }
__device__ __forceinline__ uint32_t lds_load(uint32_t a) { return *(lds_cptr)(uintptr_t)a; }

// Rows up to this many entries are scanned for their block slices, longer
// ones searched.
constexpr uint32_t kScanRow = 32;

// First position in col[rb, re) whose entry is >= key, for a row in which
// "entry < key" holds on a prefix (sorted out-rows; in-rows grouped by part,
// with key a cut point).
__device__ __forceinline__ uint32_t first_at_least(const int32_t* __restrict__ col, uint32_t rb, uint32_t re,
                                                   int32_t key) {
  while (rb < re) {
    const uint32_t mid = (rb + re) >> 1;
    if (col[mid] < key) rb = mid + 1; else re = mid;
  }
  return rb;
}

// The slice [a0, a1) of the row col[rb, re) with entries in [k0, k1), for a
// row without stored boundaries.  Short rows are counted in aligned 16-byte
// blocks (positions outside the row are masked; the arrays are aligned on
// absolute positions and padded), longer ones searched.
__device__ __forceinline__ void row_slice(const int32_t* __restrict__ col, uint32_t rb, uint32_t re, int32_t k0,
                                          int32_t k1, uint32_t& a0, uint32_t& a1) {
  if (re - rb <= kScanRow) {
    uint32_t n0 = 0, n1 = 0;
    for (uint32_t q = rb & ~3u; q < re; q += 4) {
      const int4 v = *reinterpret_cast<const int4*>(col + q);
      const int32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (uint32_t t = 0; t < 4; ++t) {
        const bool in = q + t >= rb && q + t < re;
        n0 += (in && w[t] < k0) ? 1u : 0u;
        n1 += (in && w[t] < k1) ? 1u : 0u;
      }
    }
    a0 = rb + n0;
    a1 = rb + n1;
  } else {
    a0 = first_at_least(col, rb, re, k0);
    a1 = first_at_least(col, a0, re, k1);
  }
}

// N(G_ik,u) = coli[a0, a1) for an in-neighbour u in V_i.
__device__ __forceinline__ void out_slice_i(const TaskCtx& c, int32_t u, uint32_t& a0, uint32_t& a1) {
  if (u >= c.si) {
    a0 = c.bik0[u - c.si];
    a1 = c.bik1[u - c.si];
  } else {
    row_slice(c.coli, c.orow[u], c.orow[u + 1], c.ck, c.ck1, a0, a1);
  }
}

// Largest k in [a, b) with off[k] <= x (off non-decreasing, off[a] <= x).
__device__ __forceinline__ uint32_t owner_of(const uint32_t* off, uint32_t a, uint32_t b, uint32_t x) {
  uint32_t lo = a, hi = b - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// How a stage of N(G_jk,v) is held in a buffer of nw words (a power of
// two): 0 sorted copy, 1 bitmap over V_k, 2 open-addressing hash at load at
// most 1/2.  The bitmap holds id x at bit x mod 32 of word (x / 32) mod nw,
// with x = w - c_k when the task reads the 16-bit out-rows (col16) and x = w
// otherwise; either way the list's ids map to distinct bits when they span
// at most 32 nw consecutive values from a multiple of 32 (or from c_k).
struct Stage {
  int mode;
  uint32_t piece;  // entries staged at a time
  uint32_t nw;     // buffer words
  int hbits;       // log2(nw)
};

template <uint32_t NW>
__device__ __forceinline__ Stage pick_stage(const TaskCtx& c, bool use_hash, uint32_t len) {
  constexpr int hb = log2i((int)NW);
  if (!use_hash) return Stage{0, NW, NW, hb};
  const uint32_t span = c.col16 ? (uint32_t)(c.ck1 - c.ck) : (uint32_t)(c.ck1 - c.kb);
  if (span <= NW * 32u) return Stage{1, len, NW, hb};
  return Stage{2, NW / 2, NW, hb};
}

// Pieces a list of len entries needs in a buffer of NW words.
template <uint32_t NW>
__device__ __forceinline__ uint32_t pieces(const TaskCtx& c, bool use_hash, uint32_t len) {
  const Stage st = pick_stage<NW>(c, use_hash, len);
  return (len + st.piece - 1) / st.piece;
}

// Fills buf with col[lo, lo+sn) by `nthr` cooperating threads numbered tid
// (a bitmap from the 16-bit copy col16 of the same positions when given).
__device__ __forceinline__ void stage_fill(const Stage& st, uint32_t* buf, const int32_t* __restrict__ col,
                                           const uint16_t* __restrict__ col16, uint32_t lo, uint32_t sn,
                                           uint32_t tid, uint32_t nthr) {
  if (st.mode == 0) {
    for (uint32_t t = tid; t < sn; t += nthr) buf[t] = (uint32_t)col[lo + t];
  } else if (st.mode == 1) {  // bit x mod 32 of word (x / 32) mod nw
    for (uint32_t t = tid; t < sn; t += nthr) {
      const uint32_t x = col16 ? (uint32_t)col16[lo + t] : (uint32_t)col[lo + t];
      atomicOr(&buf[(x >> 5) & (st.nw - 1)], 1u << (x & 31));
    }
  } else {
    for (uint32_t t = tid; t < sn; t += nthr) {
      const uint32_t key = (uint32_t)col[lo + t] + 1u;  // 0 marks an empty slot
      uint32_t s = hash_slot(key - 1u, st.hbits);
      for (uint32_t guard = 0; guard < st.nw && atomicCAS(&buf[s], 0u, key) != 0u; ++guard) s = (s + 1) & (st.nw - 1);
    }
  }
}

// Restores the all-zero buffer after stage_fill.
__device__ __forceinline__ void stage_clear(const Stage& st, uint32_t* buf, const int32_t* __restrict__ col,
                                            const uint16_t* __restrict__ col16, uint32_t lo, uint32_t sn,
                                            uint32_t tid, uint32_t nthr) {
  if (st.mode == 0) {
    for (uint32_t t = tid; t < sn; t += nthr) buf[t] = 0;
  } else if (st.mode == 1) {
    for (uint32_t t = tid; t < sn; t += nthr) {
      const uint32_t x = col16 ? (uint32_t)col16[lo + t] : (uint32_t)col[lo + t];
      buf[(x >> 5) & (st.nw - 1)] = 0;
    }
  } else {
    for (uint32_t t = tid; t < st.nw; t += nthr) buf[t] = 0;
  }
}

// Wavefront probes use wider segments: kSegW entries, two aligned 16-byte
// blocks (the second is read only if it holds part of the list).
constexpr uint32_t kSegW = 8;

__device__ __forceinline__ uint32_t seg_count_w(uint32_t a0, uint32_t a1) {
  return a1 > a0 ? (a1 - (a0 & ~(kSeg - 1)) + kSegW - 1) / kSegW : 0u;
}

// Segment q of the list col[a0, a1) as read, entries outside the list
// included (neighbouring rows); returns the mask of the positions that belong
// to the list.  Both 16-byte blocks are always read, without branches: the
// second block is the first one again when the list ends inside the first,
// and a q past the list (which the owner search never yields) reads the
// list's first block under an empty mask.
__device__ __forceinline__ uint32_t load_seg_raw(const int32_t* __restrict__ col, uint32_t a0, uint32_t a1,
                                                 uint32_t q, uint32_t w[kSegW]) {
  const uint32_t s = (a0 & ~(kSeg - 1)) + q * kSegW;
  const bool in = s < a1;
  const uint32_t s0 = in ? s : (a0 & ~(kSeg - 1));
  const uint32_t s1 = s0 + kSeg < a1 ? s0 + kSeg : s0;
  const int4 v0 = *reinterpret_cast<const int4*>(col + s0);
  const int4 v1 = *reinterpret_cast<const int4*>(col + s1);
  w[0] = (uint32_t)v0.x;
  w[1] = (uint32_t)v0.y;
  w[2] = (uint32_t)v0.z;
  w[3] = (uint32_t)v0.w;
  w[4] = (uint32_t)v1.x;
  w[5] = (uint32_t)v1.y;
  w[6] = (uint32_t)v1.z;
  w[7] = (uint32_t)v1.w;
  // [a0 - s0, a1 - s0) within [0, 8)
  const uint32_t lo = a0 > s0 ? a0 - s0 : 0u, hi = min(a1 - s0, kSegW);
  return in ? ((1u << hi) - 1u) & ~((1u << lo) - 1u) : 0u;
}

// The same with the positions outside the list set to all ones.
__device__ __forceinline__ void load_seg_w(const int32_t* __restrict__ col, uint32_t a0, uint32_t a1, uint32_t q,
                                           uint32_t w[kSegW]) {
  const uint32_t vm = load_seg_raw(col, a0, a1, q, w);
#pragma unroll
  for (uint32_t x = 0; x < kSegW; ++x)
    if (!((vm >> x) & 1u)) w[x] = 0xFFFFFFFFu;
}

// The owner of segment qb + lane in a round of a batch (lane l of the batch
// holds in-neighbour l, its segments [sx, sx + ns) of the batch): every
// in-neighbour whose segments meet the round marks its first position in it
// with (round number, l + 1), and the running maximum over the positions is
// the owner's mark (marks of earlier rounds are smaller; position 0 is always
// marked).  sown is cleared when the batch counter rnd starts.
__device__ __forceinline__ uint32_t round_owner(uint32_t* sown, uint32_t sx, uint32_t ns, uint32_t qb, uint32_t rnd,
                                                uint32_t l) {
  if (ns && sx < qb + kWave && sx + ns > qb) sown[sx > qb ? sx - qb : 0u] = (rnd << 7) | (l + 1u);
  wave_sync();
  const uint32_t o = ((wave_incl_max_u32(sown[l]) & 127u) - 1u) & (kWave - 1);
  wave_sync();
  return o;
}

// The probe rounds of one batch: segment q of the batch goes to lane q mod 64,
// its owner (the in-neighbour whose list holds it) from round_owner.  MODE is the stage
// form, fixed for the whole loop: 1 = bitmap over V_k, 2 = hash, 0 = sorted
// copy; for 0 and 2 entries outside [smin, smax] cannot match and are
// skipped.  The bitmap tests all eight positions without branches (every
// position indexes some word of the buffer) and keeps the hits of the list's
// own positions.
template <int MODE>
__device__ __forceinline__ uint32_t probe_rounds(const int32_t* __restrict__ col, uint32_t tot, const uint32_t* sa0,
                                                 const uint32_t* sa1, const uint32_t* sex, uint32_t* sown, uint32_t sx,
                                                 uint32_t ns, uint32_t& rnd, const Stage& st,
                                                 const uint32_t* buf, uint32_t sn, uint32_t smin, uint32_t smax) {
  const uint32_t l = (uint32_t)lane_id();
  uint32_t cnt = 0;
  for (uint32_t qb = 0; qb < tot; qb += kWave) {
    const uint32_t o = round_owner(sown, sx, ns, qb, ++rnd, l);
    const uint32_t q = qb + l;
    if (q < tot && MODE == 1) {
      uint32_t w[kSegW];
      const uint32_t vm = load_seg_raw(col, sa0[o], sa1[o], q - sex[o], w);
      // bit w mod 32 of word (w / 32) mod nw: one word per 32 consecutive
      // ids, distinct for the list's ids (all within 32 nw consecutive ids
      // from a multiple of 32); the other positions read some word of the
      // buffer and the mask drops their hits
      // LDS byte address of the word: the buffer's base (aligned to its size)
      // ORed with the word offset, two instructions per position
      const uint32_t base = lds_addr(buf), omask = (st.nw - 1) << 2;
      uint32_t wd[kSegW];
#pragma unroll
      for (uint32_t t = 0; t < kSegW; ++t) wd[t] = lds_load(base | ((w[t] >> 3) & omask));
      uint32_t hit = 0;
#pragma unroll
      for (uint32_t t = 0; t < kSegW; ++t) hit |= __builtin_amdgcn_ubfe(wd[t], w[t], 1u) << t;  // offset taken mod 32
      cnt += __popc(hit & vm);
    } else if (q < tot) {
      uint32_t w[kSegW];
      load_seg_w(col, sa0[o], sa1[o], q - sex[o], w);
#pragma unroll
      for (uint32_t t = 0; t < kSegW; ++t) {
        if (w[t] >= smin && w[t] <= smax) {
          if (MODE == 2) {
            const uint32_t key = w[t] + 1u;
            uint32_t h = hash_slot(w[t], st.hbits);
            for (uint32_t guard = 0; guard < st.nw; ++guard) {
              const uint32_t kk = buf[h];
              if (kk == key) {
                ++cnt;
                break;
              }
              if (kk == 0u) break;
              h = (h + 1) & (st.nw - 1);
            }
          } else {
            uint32_t x = 0, y = sn;
            while (x < y) {
              const uint32_t mid = (x + y) >> 1;
              if (buf[mid] < w[t]) x = mid + 1; else y = mid;
            }
            cnt += (x < sn && buf[x] == w[t]) ? 1u : 0u;
          }
        }
      }
    }
  }
  return cnt;
}

// A dense slice (stored as a bitmap over V_k) is marked by sa1 = kDenseMark
// and probed kDenseSeg words per segment.
constexpr uint32_t kDenseMark = 0xFFFFFFFFu;
constexpr uint32_t kDenseSeg = 8;

// Segments of the 16-bit out-rows: kSeg16 entries, aligned 16-byte blocks
// of 8 entries each (the owner search and the segment bounds of a probe
// round are paid once per segment).
constexpr uint32_t kSeg16 = 16;
__device__ __forceinline__ uint32_t seg_count16(uint32_t a0, uint32_t a1) {
  return a1 > a0 ? (a1 - (a0 & ~7u) + kSeg16 - 1u) / kSeg16 : 0u;
}

// Segment q of the list col16[a0, a1) as kSeg16/2 words of two entries each
// (entry 2h in the low half of x[h]); returns the mask of the positions that
// belong to the list.  A block past the list end rereads the segment's first
// block, and a q past the list reads the list's first block, both under an
// empty mask for those positions.
__device__ __forceinline__ uint32_t load_seg16(const uint16_t* __restrict__ col, uint32_t a0, uint32_t a1, uint32_t q,
                                               uint32_t x[kSeg16 / 2]) {
  const uint32_t s = (a0 & ~7u) + q * kSeg16;
  const bool in = s < a1;
  const uint32_t s0 = in ? s : (a0 & ~7u);
#pragma unroll
  for (uint32_t h = 0; h < kSeg16 / 8; ++h) {
    const uint32_t sh = s0 + 8 * h < a1 ? s0 + 8 * h : s0;
    const uint4 v = *reinterpret_cast<const uint4*>(col + sh);
    x[4 * h + 0] = v.x;
    x[4 * h + 1] = v.y;
    x[4 * h + 2] = v.z;
    x[4 * h + 3] = v.w;
  }
  const uint32_t lo = a0 > s0 ? a0 - s0 : 0u, hi = min(a1 - s0, kSeg16);
  return in ? ((hi >= 32u ? 0xFFFFFFFFu : (1u << hi) - 1u) & ~((1u << lo) - 1u)) : 0u;
}

// probe_rounds<1> over the 16-bit out-rows: the bitmap holds x = w - c_k.
// Word (x / 32) mod nw as a byte address: bits 5.. of the entry shifted to
// bits 2.. (low half: x >> 3, high half: x >> 19), masked and ORed into the
// aligned base; the bit is x mod 32.
__device__ __forceinline__ uint32_t probe_rounds16(const uint16_t* __restrict__ col,
                                                   const uint32_t* __restrict__ dbits, uint32_t tot,
                                                   const uint32_t* sa0, const uint32_t* sa1, const uint32_t* sex,
                                                   uint32_t* sown, uint32_t sx, uint32_t ns, uint32_t& rnd,
                                                   const Stage& st, const uint32_t* buf) {
  const uint32_t l = (uint32_t)lane_id();
  const uint32_t base = lds_addr(buf), omask = (st.nw - 1) << 2;
  uint32_t cnt = 0;
  for (uint32_t qb = 0; qb < tot; qb += kWave) {
    const uint32_t o = round_owner(sown, sx, ns, qb, ++rnd, l);
    const uint32_t q = qb + l;
    if (q < tot && sa1[o] == kDenseMark) {
      // a dense N(G_ik,u): 8 words of its bitmap against the same 8 words of
      // the staged bitmap of V_k (word t covers c_k + 32t .. c_k + 32t + 31)
      const uint32_t t0 = (q - sex[o]) * kDenseSeg;
      const uint4* src = reinterpret_cast<const uint4*>(dbits + sa0[o] + t0);
      const uint4 x0 = src[0], x1 = src[1];
      const uint32_t xw[kDenseSeg] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
      for (uint32_t h = 0; h < kDenseSeg; ++h) cnt += __popc(xw[h] & lds_load(base | (((t0 + h) << 2) & omask)));
    } else if (q < tot) {
      uint32_t x[kSeg16 / 2];
      const uint32_t vm = load_seg16(col, sa0[o], sa1[o], q - sex[o], x);
      uint32_t wl[kSeg16 / 2], wh[kSeg16 / 2];
#pragma unroll
      for (uint32_t h = 0; h < kSeg16 / 2; ++h) {
        wl[h] = lds_load(base | ((x[h] >> 3) & omask));
        wh[h] = lds_load(base | ((x[h] >> 19) & omask));
      }
      uint32_t hit = 0;
#pragma unroll
      for (uint32_t h = 0; h < kSeg16 / 2; ++h) {
        hit |= __builtin_amdgcn_ubfe(wl[h], x[h], 1u) << (2 * h);
        hit |= __builtin_amdgcn_ubfe(wh[h], x[h] >> 16, 1u) << (2 * h + 1);
      }
      cnt += __popc(hit & vm);
    }
  }
  return cnt;
}

// One wavefront tests every w of N(G_ik,u), for the in-neighbours
// u = icol[i0..i1), against the stage.  The probe space is cut into segments
// of kSegW consecutive entries of one N(G_ik,u); a wavefront prefix sum over
// the segment counts of 64 in-neighbours at a time lets all lanes share the
// segments, however unequal the lists are.
__device__ uint64_t probe_flat(const TaskCtx& c, uint32_t i0, uint32_t i1, const Stage& st, const uint32_t* buf,
                               uint32_t sn, int32_t smin, int32_t smax, uint32_t* sa0, uint32_t* sa1, uint32_t* sex,
                               uint32_t* sown) {
  const int32_t* __restrict__ col = c.coli;
  const int32_t* __restrict__ icol = c.icolj;
  const uint32_t l = (uint32_t)lane_id();
  // a bitmap stage probed with the 16-bit out-rows: 8 entries per 16 bytes
  const bool c16 = c.col16 != nullptr && st.mode == 1;
  uint64_t cnt = 0;
  uint32_t rnd = 0;
  sown[l] = 0;
  const bool dense = c16 && c.dslot != nullptr;
  for (uint32_t eb = i0; eb < i1; eb += kWave) {
    const uint32_t e = eb + l;
    uint32_t a0 = 0, a1 = 0;
    if (e < i1) {
      const int32_t u = icol[e];
      const uint32_t slot = dense && u >= c.du0 ? c.dslot[(uint32_t)(u - c.du0) * c.dnk] : 0u;
      out_slice_i(c, u, a0, a1);
      if (slot && a1 > a0) {
        a0 = slot - 1;
        a1 = kDenseMark;
      }
    }
    const uint32_t nseg = a1 == kDenseMark ? c.dwords / kDenseSeg : (c16 ? seg_count16(a0, a1) : seg_count_w(a0, a1));
    const uint32_t inc = wave_incl_scan_u32(nseg);
    const uint32_t tot = last_lane(inc);
    sa0[l] = a0;
    sa1[l] = a1;
    sex[l] = inc - nseg;
    wave_sync();
    if (c16)
      cnt += probe_rounds16(c.col16, c.dbits, tot, sa0, sa1, sex, sown, inc - nseg, nseg, rnd, st, buf);
    else if (st.mode == 1)
      cnt += probe_rounds<1>(col, tot, sa0, sa1, sex, sown, inc - nseg, nseg, rnd, st, buf, sn, (uint32_t)smin,
                               (uint32_t)smax);
    else if (st.mode == 2)
      cnt += probe_rounds<2>(col, tot, sa0, sa1, sex, sown, inc - nseg, nseg, rnd, st, buf, sn, (uint32_t)smin,
                               (uint32_t)smax);
    else
      cnt += probe_rounds<0>(col, tot, sa0, sa1, sex, sown, inc - nseg, nseg, rnd, st, buf, sn, (uint32_t)smin,
                               (uint32_t)smax);
    wave_sync();
  }
  return cnt;
}

// One wavefront: in-slice [i0,i1) of v against N(G_jk,v) = ocol[c0..c1).
__device__ uint64_t wave_col(const TaskCtx& c, uint32_t i0, uint32_t i1, uint32_t c0, uint32_t c1, bool use_hash,
                             uint32_t* abuf, uint32_t* sa0, uint32_t* sa1, uint32_t* sex, uint32_t* sown) {
  const int32_t* __restrict__ col = c.colj;
  const uint32_t l = (uint32_t)lane_id();
  uint64_t cnt = 0;
  const Stage st = pick_stage<kABuf>(c, use_hash, c1 - c0);
  for (uint32_t s_lo = c0; s_lo < c1; s_lo += st.piece) {
    const uint32_t sn = min(st.piece, c1 - s_lo);
    stage_fill(st, abuf, col, c.col16, s_lo, sn, l, kWave);
    wave_sync();
    cnt += probe_flat(c, i0, i1, st, abuf, sn, col[s_lo], col[s_lo + sn - 1], sa0, sa1, sex, sown);
    stage_clear(st, abuf, col, c.col16, s_lo, sn, l, kWave);
    wave_sync();
  }
  return cnt;
}

// Bounds of active column x of block (i,j): N(G_jk,v) = col[c0,c1) and the
// in-slice [i0,i1) of v in V_i.
// N(G_jk,v) = colj[c0, c1) for a column v in V_j.
__device__ __forceinline__ void out_slice_j(const TaskCtx& c, int32_t v, uint32_t& c0, uint32_t& c1) {
  if (v >= c.sj) {
    c0 = c.bjk0[v - c.sj];
    c1 = c.bjk1[v - c.sj];
  } else {
    row_slice(c.colj, c.orow[v], c.orow[v + 1], c.ck, c.ck1, c0, c1);
  }
}

__device__ __forceinline__ void col_bounds(const TaskCtx& c, uint32_t x, uint32_t& c0, uint32_t& c1, uint32_t& i0,
                                           uint32_t& i1) {
  out_slice_j(c, c.ac[x], c0, c1);
  i0 = c.ao[x];
  i1 = c.ao[x + 1];
}

// col_bounds for a column index that is the same on every lane: scalar loads.
__device__ __forceinline__ void col_bounds_uniform(const TaskCtx& c, uint32_t x, uint32_t& c0, uint32_t& c1,
                                                   uint32_t& i0, uint32_t& i1) {
  x = __builtin_amdgcn_readfirstlane(x);
  const int32_t v = ld_const(c.ac + x);
  i0 = ld_const(c.ao + x);
  i1 = ld_const(c.ao + x + 1);
  if (v >= c.sj) {
    c0 = ld_const(c.bjk0 + (v - c.sj));
    c1 = ld_const(c.bjk1 + (v - c.sj));
  } else {
    out_slice_j(c, v, c0, c1);
    c0 = __builtin_amdgcn_readfirstlane(c0);
    c1 = __builtin_amdgcn_readfirstlane(c1);
  }
}

// Packed short columns [a0, b0) of a pass (bounds in c0s/i0s, prefixes in
// soff/ioff), by one wavefront, window by window: a window is the longest run
// of columns whose lists fit the wavefront's stage together.  The lists are
// copied, sorted, side by side; every probe is a binary search in its own
// column's run, in fixed halving steps from the window's longest run so that
// the eight searches of a segment advance together.
__device__ uint64_t short_cols(const TaskCtx& c, CountLds& s, uint32_t a0, uint32_t b0, int w) {
  const int32_t* __restrict__ colj = c.colj;
  const int32_t* __restrict__ coli = c.coli;
  const int32_t* __restrict__ icol = c.icolj;
  const uint32_t l = (uint32_t)lane_id();
  uint32_t* stage = s.abuf[w];
  uint32_t* sa0 = s.w.sa0[w];
  uint32_t* sa1 = s.w.sa1[w];
  uint32_t* sex = s.w.sex[w];
  uint32_t* scol = s.w.scol[w];
  uint32_t* sown = s.w.sown[w];
  uint64_t cnt = 0;
  uint32_t rnd = 0;
  sown[l] = 0;
  for (uint32_t a = a0; a < b0;) {  // uniform across the wavefront
    const uint32_t sbase = s.soff[a];
    uint32_t b = a + 1, hi = b0;  // largest b in [a+1, b0] with soff[b] - sbase <= kABuf
    while (b < hi) {
      const uint32_t mid = (b + hi + 1) >> 1;
      if (s.soff[mid] - sbase <= (uint32_t)kABuf) b = mid; else hi = mid - 1;
    }
    const uint32_t span = s.soff[b] - sbase;
    uint32_t mx = 0;
    for (uint32_t k = a + l; k < b; k += kWave) mx = max(mx, s.soff[k + 1] - s.soff[k]);
    mx = wave_max_u32(mx);
    const uint32_t top = mx > 1 ? 1u << (31 - __clz(mx - 1)) : 0u;  // 2*top > longest run - 1
    for (uint32_t g = l; g < span; g += kWave) {
      const uint32_t k = owner_of(s.soff, a, b, sbase + g);
      stage[g] = (uint32_t)colj[s.c0s[k] + (sbase + g - s.soff[k])];
    }
    wave_sync();
    const uint32_t iend = s.ioff[b];
    for (uint32_t eb = s.ioff[a]; eb < iend; eb += kWave) {  // uniform
      const uint32_t e = eb + l;
      uint32_t u0 = 0, u1 = 0, k = a;
      if (e < iend) {
        k = owner_of(s.ioff, a, b, e);
        out_slice_i(c, icol[s.i0s[k] + (e - s.ioff[k])], u0, u1);
      }
      const uint32_t nseg = seg_count_w(u0, u1);
      const uint32_t inc = wave_incl_scan_u32(nseg);
      const uint32_t tot = last_lane(inc);
      sa0[l] = u0;
      sa1[l] = u1;
      sex[l] = inc - nseg;
      scol[l] = k;
      wave_sync();
      uint32_t lc = 0;
      for (uint32_t qb = 0; qb < tot; qb += kWave) {
        const uint32_t o = round_owner(sown, inc - nseg, nseg, qb, ++rnd, l);
        const uint32_t q = qb + l;
        if (q < tot) {
          const uint32_t k2 = scol[o];
          const uint32_t lo = s.soff[k2] - sbase, hi2 = s.soff[k2 + 1] - sbase;
          uint32_t wv[kSegW];
          const uint32_t vm = load_seg_raw(coli, sa0[o], sa1[o], q - sex[o], wv);
          // pos: the last position of the run whose value is <= w (lo if none is)
          uint32_t pos[kSegW];
#pragma unroll
          for (uint32_t x = 0; x < kSegW; ++x) pos[x] = lo;
          for (uint32_t step = top; step > 0; step >>= 1) {
#pragma unroll
            for (uint32_t x = 0; x < kSegW; ++x) {
              const uint32_t nx = pos[x] + step;
              if (nx < hi2 && stage[nx] <= wv[x]) pos[x] = nx;
            }
          }
          uint32_t hit = 0;
#pragma unroll
          for (uint32_t x = 0; x < kSegW; ++x) hit |= (stage[pos[x]] == wv[x] ? 1u : 0u) << x;
          lc += __popc(hit & vm);
        }
      }
      cnt += lc;
      wave_sync();
    }
    for (uint32_t g = l; g < span; g += kWave) stage[g] = 0;
    wave_sync();
    a = b;
  }
  return cnt;
}

__device__ uint64_t group_col(const PlanCtx& cp, const TaskCtx& c, uint32_t i0, uint32_t i1, uint32_t c0, uint32_t c1,
                              CountLds& s);

// Active columns [lo, hi) of block (i,j), by the whole workgroup, 256 per
// pass.  Columns with in-slices longer than cp.split are left to their split
// items; columns whose lists reach wave_min get a wavefront of their own (a
// shared queue hands them out) or, if only the four buffers together hold
// their list in fewer pieces, the whole workgroup; the others are packed and
// split into four runs of about equal in-slice volume, one per wavefront
// (short_cols).
__device__ uint64_t process_cols(const PlanCtx& cp, const TaskCtx& c, uint32_t lo, uint32_t hi, CountLds& s) {
  const int t = threadIdx.x, w = t / kWave;
  const uint32_t own_min = min((uint32_t)cp.wave_min, (uint32_t)kABuf);
  uint64_t cnt = 0;
  for (uint32_t base = lo; base < hi; base += kThreads) {
    const uint32_t x = base + t;
    uint32_t c0 = 0, c1 = 0, i0 = 0, i1 = 0;
    if (x < hi) col_bounds(c, x, c0, c1, i0, i1);
    const bool live = c1 > c0 && i1 > i0 && (cp.split == 0 || i1 - i0 <= cp.split);
    // in-slices up to 2^24 keep the packed prefix below in range
    const bool own = live && ((c1 - c0) >= own_min || (i1 - i0) >= (1u << 24) / kThreads);
    if (own) {
      // lists that a wavefront's buffer holds only in pieces go to the whole
      // workgroup when its four buffers need fewer pieces
      const bool use_hash = cp.hash_min >= 0 && (c1 - c0) >= (uint32_t)cp.hash_min;
      const uint32_t pw = pieces<kABuf>(c, use_hash, c1 - c0);
      if (pw > 1 && pieces<kGroupWords>(c, use_hash, c1 - c0) < pw)
        s.q[kThreads - 1 - atomicAdd(&s.qw, 1u)] = x;
      else
        s.q[atomicAdd(&s.qn, 1u)] = x;
    }
    const bool sh = live && !own;
    // one 64-bit scan packs: count (bits 0-8), in-slice length (9-33), list length (34-63)
    const unsigned long long pk =
        sh ? (1ull | ((unsigned long long)(i1 - i0) << 9) | ((unsigned long long)(c1 - c0) << 34)) : 0ull;
    unsigned long long tot;
    const unsigned long long ex = block256_excl_scan(pk, s.red, &tot);
    const uint32_t ns = (uint32_t)(tot & 511u);
    if (sh) {
      const uint32_t k = (uint32_t)(ex & 511u);
      s.c0s[k] = c0;
      s.i0s[k] = i0;
      s.soff[k] = (uint32_t)(ex >> 34);
      s.ioff[k] = (uint32_t)((ex >> 9) & 0x1FFFFFFu);
    }
    if (t == 0) {
      s.soff[ns] = (uint32_t)(tot >> 34);
      s.ioff[ns] = (uint32_t)((tot >> 9) & 0x1FFFFFFu);
    }
    __syncthreads();
    const uint32_t nq = s.qn;
    for (uint32_t h = w; h < nq; h += 4) {
      uint32_t qc0, qc1, qi0, qi1;
      col_bounds_uniform(c, s.q[h], qc0, qc1, qi0, qi1);
      const bool use_hash = cp.hash_min >= 0 && (qc1 - qc0) >= (uint32_t)cp.hash_min;
      cnt += wave_col(c, qi0, qi1, qc0, qc1, use_hash, s.abuf[w], s.w.sa0[w], s.w.sa1[w], s.w.sex[w], s.w.sown[w]);
    }
    if (ns) {
      // this wavefront's run: the columns whose in-slices start in its quarter
      const uint32_t itot = s.ioff[ns];
      uint32_t ab[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t target = (uint32_t)(((uint64_t)itot * (uint32_t)(w + h)) / 4u);
        uint32_t x0 = 0, x1 = ns;  // first column with ioff >= target
        while (x0 < x1) {
          const uint32_t mid = (x0 + x1) >> 1;
          if (s.ioff[mid] < target) x0 = mid + 1; else x1 = mid;
        }
        ab[h] = (w + h == 4) ? ns : x0;
      }
      if (ab[0] < ab[1]) cnt += short_cols(c, s, ab[0], ab[1], w);
    }
    __syncthreads();  // every wavefront buffer is clear again: they form one stage now
    const uint32_t nwide = s.qw;
    for (uint32_t h = 0; h < nwide; ++h) {
      uint32_t qc0, qc1, qi0, qi1;
      col_bounds_uniform(c, s.q[kThreads - 1 - h], qc0, qc1, qi0, qi1);
      cnt += group_col(cp, c, qi0, qi1, qc0, qc1, s);
    }
    if (t == 0) s.qn = s.qw = 0;
    __syncthreads();
  }
  return cnt;
}

// In-slice [i0, i1) of column v against N(G_jk,v) = col[c0, c1), by the
// whole workgroup: the four wavefront buffers form one stage of kGroupWords
// words (all zero on entry and on exit), filled once per piece by all
// threads, and each wavefront probes a quarter of the in-neighbours.
__device__ uint64_t group_col(const PlanCtx& cp, const TaskCtx& c, uint32_t i0, uint32_t i1, uint32_t c0, uint32_t c1,
                              CountLds& s) {
  const int32_t* __restrict__ col = c.colj;
  const int w = threadIdx.x / kWave;
  uint64_t cnt = 0;
  const uint32_t per = (i1 - i0 + 3) / 4;
  const uint32_t w0 = min(i0 + per * w, i1), w1 = min(w0 + per, i1);
  const bool use_hash = cp.hash_min >= 0 && (c1 - c0) >= (uint32_t)cp.hash_min;
  const Stage st = pick_stage<kGroupWords>(c, use_hash, c1 - c0);
  uint32_t* buf = &s.abuf[0][0];
  for (uint32_t s_lo = c0; s_lo < c1; s_lo += st.piece) {
    const uint32_t sn = min(st.piece, c1 - s_lo);
    stage_fill(st, buf, col, c.col16, s_lo, sn, threadIdx.x, kThreads);
    __syncthreads();
    cnt += probe_flat(c, w0, w1, st, buf, sn, col[s_lo], col[s_lo + sn - 1], s.w.sa0[w], s.w.sa1[w],
                      s.w.sex[w], s.w.sown[w]);
    __syncthreads();
    stage_clear(st, buf, col, c.col16, s_lo, sn, threadIdx.x, kThreads);
    __syncthreads();
  }
  return cnt;
}

// One chunk [lo, hi) of the in-slice of the hub column with absolute
// active-column index x, by the whole workgroup.
__device__ uint64_t hub_chunk(const PlanCtx& cp, const TaskCtx& c, uint32_t x, uint32_t lo, uint32_t hi,
                              CountLds& s) {
  const int32_t v = ld_const(c.acb + x);
  const uint32_t ib = ld_const(c.aob + x), ie = ld_const(c.aob + x + 1);
  uint32_t c0, c1;
  out_slice_j(c, v, c0, c1);
  c0 = __builtin_amdgcn_readfirstlane(c0);
  c1 = __builtin_amdgcn_readfirstlane(c1);
  const uint32_t i0 = min(ib + lo, ie), i1 = min(ib + hi, ie);
  if (c1 <= c0 || i1 <= i0) return 0;  // uniform across the workgroup
  return group_col(cp, c, i0, i1, c0, c1, s);
}

__device__ __forceinline__ void init_lds(CountLds& s) {
  uint32_t* a = &s.abuf[0][0];
  for (int t = threadIdx.x; t < 4 * kABuf; t += kThreads) a[t] = 0;
  if (threadIdx.x == 0) s.qn = s.qw = 0;
  __syncthreads();
}

__device__ __forceinline__ void flush(const PlanCtx& cp, int32_t out, uint64_t cnt, CountLds& s) {
  cnt = block256_sum_u64(cnt, s.red);
  if (threadIdx.x == 0 && cnt) {
    atomicAdd((unsigned long long*)&cp.per_task[out], (unsigned long long)cnt);
    atomicAdd((unsigned long long*)cp.total, (unsigned long long)cnt);
  }
}

__device__ __forceinline__ uint64_t run_item(const PlanCtx& pc, const DevItem& item, CountLds& s, int32_t* out) {
  const DevTask t = ld_const(pc.tasks + item.task);
  const TaskCtx c = make_ctx(pc.g, t);
  *out = t.out;
  if (item.v >= 0) return hub_chunk(pc, c, (uint32_t)item.v, item.lo, item.hi, s);
  return process_cols(pc, c, item.lo, item.hi, s);
}

// Items [first, first + gridDim.x) of the item list, one workgroup each.
// Eight workgroups per CU fit the LDS; the register budget is held to match.
#define BBTC_COUNT_KERNEL __global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8)))

BBTC_COUNT_KERNEL void k_count_items(CountParams cp, uint32_t first) {
  __shared__ __attribute__((aligned(kGroupWords * 4))) CountLds s;
  init_lds(s);
  const PlanCtx& pc = cp.one;
  const DevItem item = ld_const(cp.items + first + blockIdx.x);
  int32_t out = 0;
  const uint64_t cnt = run_item(pc, item, s, &out);
  flush(pc, out, cnt, s);
}

// Persistent work-stealing form: every workgroup claims work items from a
// global cursor until none are left.  MULTI: items of several plans, each
// read from its own plan's item list.
template <bool MULTI>
BBTC_COUNT_KERNEL void k_count_persistent(CountParams cp) {
  __shared__ __attribute__((aligned(kGroupWords * 4))) CountLds s;
  init_lds(s);
  // workgroups are dispatched to the XCDs round robin: start on this one's queue
  uint32_t x = blockIdx.x % cp.nq, tried = 0;
  while (true) {
    if (threadIdx.x == 0) {
      uint32_t it = 0xFFFFFFFFu;
      while (tried < cp.nq) {
        const uint32_t r = atomicAdd(&cp.cursor[x], 1u);
        if (r < cp.qlen[x]) {
          it = cp.qbeg[x] + r;
          break;
        }
        ++tried;  // this queue is drained: move on to the next
        x = x + 1 == cp.nq ? 0 : x + 1;
      }
      s.item = it;
    }
    __syncthreads();
    // the claimed item is uniform: keep it (and all that derives from it) in scalar registers
    const uint32_t it = __builtin_amdgcn_readfirstlane(s.item);
    __syncthreads();
    if (it >= cp.nitems) break;
    DevItem item;
    PlanCtx pc;
    if constexpr (MULTI) {
      uint32_t a = 0, b = (uint32_t)cp.nplans - 1;  // the plan whose item range holds it
      while (a < b) {
        const uint32_t mid = (a + b + 1) >> 1;
        if (ld_const(cp.plan_off + mid) <= it) a = mid; else b = mid - 1;
      }
      pc = ld_const(cp.many + a);
      item = ld_const(pc.items + (it - ld_const(cp.plan_off + a)));
    } else {
      pc = cp.one;
      item = ld_const(cp.items + it);
    }
    int32_t out = 0;
    const uint64_t cnt = run_item(pc, item, s, &out);
    flush(pc, out, cnt, s);
  }
}

__global__ __launch_bounds__(kThreads) void k_reset(uint64_t* per_task, int64_t ntasks, uint64_t* total,
                                                    uint32_t* cursor) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntasks; t += (int64_t)gridDim.x * blockDim.x)
    per_task[t] = 0;
  if (blockIdx.x == 0 && threadIdx.x < kMaxQueues) {
    if (total && threadIdx.x == 0) *total = 0;
    if (cursor) cursor[threadIdx.x] = 0;
  }
}

__global__ __launch_bounds__(kThreads) void k_reset_multi(const PlanCtx* ctxs, int32_t nplans, uint32_t* cursor) {
  for (int32_t q = blockIdx.x; q < nplans; q += gridDim.x) {
    const PlanCtx c = ctxs[q];
    for (int64_t t = threadIdx.x; t < c.ntasks; t += kThreads) c.per_task[t] = 0;
    if (threadIdx.x == 0) *c.total = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x < kMaxQueues) cursor[threadIdx.x] = 0;
}

__global__ void k_add_u64(uint64_t* __restrict__ x, uint64_t v) {
  if (threadIdx.x == 0) *x += v;
}

}  // namespace

hipError_t launch_add_u64(uint64_t* x, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(64), 0, s, x, v);
  return hipGetLastError();
}

hipError_t launch_reset_multi(const PlanCtx* ctxs, int32_t nplans, uint32_t* cursor, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_multi, dim3(nplans > 0 ? (nplans < 1024 ? nplans : 1024) : 1), dim3(kThreads), 0, s, ctxs,
                     nplans, cursor);
  return hipGetLastError();
}

hipError_t launch_reset(uint64_t* per_task, int64_t ntasks, uint64_t* total, uint32_t* cursor, hipStream_t s) {
  int64_t g = (ntasks + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_reset, dim3((unsigned)g), dim3(kThreads), 0, s, per_task, ntasks, total, cursor);
  return hipGetLastError();
}

hipError_t launch_count_items(const CountParams& cp, uint32_t first, uint32_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_items, dim3(count), dim3(kThreads), 0, s, cp, first);
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
