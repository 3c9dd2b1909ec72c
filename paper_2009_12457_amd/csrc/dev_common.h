// Device helpers shared by the preprocessing and counting kernels (gfx950,
// 64-lane wavefronts).  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bbtc {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Orders LDS traffic of one wavefront: every lane's earlier LDS writes are
// visible to every lane's later LDS reads.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return (uint32_t)__popcll(mask & __lanemask_lt());
}

// Inclusive prefix sum over the 64 lanes of a wavefront, by DPP moves (the
// pattern of wave_incl_max_u32 below: shifts by 1, 2, 4, 8 within rows of
// 16, then the row totals of lanes 15/47 and 31 into the rows above; lanes a
// move does not reach add 0).
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// The value of lane 63 (a wave total after an inclusive scan), uniform.
__device__ __forceinline__ uint32_t last_lane(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1); }

// The 64-bit form: both halves of the source lane's value move by the same
// DPP pattern, and the sums are 64-bit.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_move_u64(unsigned long long v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROW_MASK, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROW_MASK, 0xf, false);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long v) {
  v += dpp_move_u64<0x111, 0xf>(v);  // row_shr:1
  v += dpp_move_u64<0x112, 0xf>(v);  // row_shr:2
  v += dpp_move_u64<0x114, 0xf>(v);  // row_shr:4
  v += dpp_move_u64<0x118, 0xf>(v);  // row_shr:8
  v += dpp_move_u64<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_move_u64<0x143, 0xc>(v);  // row_bcast:31
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    uint32_t t = __shfl_xor(v, o, kWave);
    v = t > v ? t : v;
  }
  return v;
}

// Inclusive running maximum over the 64 lanes of a wavefront, by DPP moves:
// shifts by 1, 2, 4 and 8 lanes within each row of 16, then the last lane of
// row 0 into row 1 and of row 2 into row 3, then lane 31 into rows 2 and 3
// (lanes a move does not reach take 0, the identity for unsigned maximum).
__device__ __forceinline__ uint32_t wave_incl_max_u32(uint32_t v) {
  uint32_t t;
  t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v = t > v ? t : v;
  t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v = t > v ? t : v;
  t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v = t > v ? t : v;
  t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v = t > v ? t : v;
  t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v = t > v ? t : v;
  t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  v = t > v ? t : v;
  return v;
}

// Exclusive scan of one value per thread over a 256-thread workgroup.
// `lds` needs 4 slots.  Contains barriers: call from uniform control flow.
template <typename T>
__device__ __forceinline__ T block256_excl_scan(T v, T* lds, T* total) {
  const int l = lane_id(), w = threadIdx.x / kWave;
  T inc;
  if constexpr (sizeof(T) == 8)
    inc = (T)wave_incl_scan_u64((unsigned long long)v);
  else
    inc = (T)wave_incl_scan_u32((uint32_t)v);
  if (l == kWave - 1) lds[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T s = lds[q];
    if (q < w) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__device__ __forceinline__ unsigned long long block256_sum_u64(unsigned long long v,
                                                               unsigned long long* lds) {
  v = wave_sum_u64(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) lds[w] = v;
  __syncthreads();
  unsigned long long s = lds[0] + lds[1] + lds[2] + lds[3];
  __syncthreads();
  return s;
}

}  // namespace bbtc
