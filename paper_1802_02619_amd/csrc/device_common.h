// Device-side helpers shared by the HIP kernels (wave64 primitives).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lco_internal.h"

namespace lco {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Wave-wide scans and reductions on DPP lane moves (no LDS traffic, no lane
// address registers).  row_shr:n moves each lane's value n lanes up within its
// row of 16 (lanes with no source read 0); row_bcast:15 copies lane 15 of each
// row into the next row and row_bcast:31 copies lane 31 into rows 2 and 3,
// each only into the rows the row mask selects.  All 64 lanes must be active.
template <int CTRL, int ROWS, bool ZERO>
__device__ __forceinline__ uint32_t dpp_move(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xf, ZERO);
}
template <int CTRL, int ROWS, bool ZERO>
__device__ __forceinline__ uint64_t dpp_move(uint64_t x) {
  return ((uint64_t)dpp_move<CTRL, ROWS, ZERO>((uint32_t)(x >> 32)) << 32) | dpp_move<CTRL, ROWS, ZERO>((uint32_t)x);
}
constexpr int kDppRowShr = 0x110, kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

// Inclusive prefix sum over the wave (lane order): Hillis-Steele steps of 1,
// 2, 4 and 8 lanes within each row, then the totals of rows 0 and 2 into rows
// 1 and 3, then the total of rows 0-1 into rows 2 and 3.
template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  x += dpp_move<kDppRowShr + 1, 0xf, true>(x);
  x += dpp_move<kDppRowShr + 2, 0xf, true>(x);
  x += dpp_move<kDppRowShr + 4, 0xf, true>(x);
  x += dpp_move<kDppRowShr + 8, 0xf, true>(x);
  x += dpp_move<kDppRowBcast15, 0xa, false>(x);
  x += dpp_move<kDppRowBcast31, 0xc, false>(x);
  return x;
}

// Inclusive running maximum over the wave (lane order), the same steps with
// max in place of +; lanes a step does not reach see 0, so the values must
// be unsigned.
__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t x) {
  uint32_t y;
  y = dpp_move<kDppRowShr + 1, 0xf, true>(x); x = x > y ? x : y;
  y = dpp_move<kDppRowShr + 2, 0xf, true>(x); x = x > y ? x : y;
  y = dpp_move<kDppRowShr + 4, 0xf, true>(x); x = x > y ? x : y;
  y = dpp_move<kDppRowShr + 8, 0xf, true>(x); x = x > y ? x : y;
  y = dpp_move<kDppRowBcast15, 0xa, false>(x); x = x > y ? x : y;
  y = dpp_move<kDppRowBcast31, 0xc, false>(x); x = x > y ? x : y;
  return x;
}

__device__ __forceinline__ uint32_t lane_value(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
__device__ __forceinline__ uint64_t lane_value(uint64_t x, int l) {
  return ((uint64_t)lane_value((uint32_t)(x >> 32), l) << 32) | lane_value((uint32_t)x, l);
}

// Sum over the wave, returned to every lane.
template <class T>
__device__ __forceinline__ T wave_reduce_sum(T x) {
  return lane_value(wave_inclusive_scan(x), kWave - 1);
}

// Exclusive scan of one value per thread over the block; returns the block total
// through `total`.  `wsum` must hold blockDim/64 + 1 elements of LDS.
template <class T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* wsum, T& total) {
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  T inc = wave_inclusive_scan(x);
  if (lane == kWave - 1) wsum[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    T v = lane < nw ? wsum[lane] : T(0);
    T vi = wave_inclusive_scan(v);
    if (lane < nw) wsum[lane] = vi - v;
    if (lane == nw - 1) wsum[nw] = vi;  // block total after the per-wave offsets
  }
  __syncthreads();
  total = wsum[nw];
  T res = wsum[wave] + inc - x;
  __syncthreads();
  return res;
}

// The LIV shuffle (Section 3.1): decode an old-order LIV into coordinates by
// repeated invariant division, then re-linearise with the new order's weights.
__device__ __forceinline__ uint64_t shuffle_liv(const ShuffleParams& sp, uint64_t x) {
  uint64_t out = 0;
  if (sp.all_pow2) {
    for (int q = 0; q < sp.order; ++q) out |= ((x >> sp.in_shift[q]) & sp.in_mask[q]) << sp.out_shift[q];
    return out;
  }
  for (int q = 0; q < sp.order - 1; ++q) {
    uint64_t c;
    x = fd_divmod(sp.dim[q], x, c);
    out += c * sp.new_weight[q];
  }
  if (sp.order > 0) out += x * sp.new_weight[sp.order - 1];
  return out;
}

}  // namespace lco
