// Device-side helpers shared by the HIP kernels (wave64 primitives).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lco_internal.h"

namespace lco {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T t = __shfl_up(x, o, kWave);
    if (lane >= o) x += t;
  }
  return x;
}

template <class T>
__device__ __forceinline__ T wave_reduce_sum(T x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

template <class T>
__device__ __forceinline__ T wave_reduce_max(T x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T y = __shfl_xor(x, o, kWave);
    x = y > x ? y : x;
  }
  return x;
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
