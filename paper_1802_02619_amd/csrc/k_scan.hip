// Device-wide exclusive prefix sums (reduce -> scan partials -> scan tiles).
// Used for radix bucket offsets, compaction positions and per-row output offsets.
#include "device_common.h"

namespace lco {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
// Up to this many tiles, each tile sums the partials before it itself (at most
// 16 loads per thread) instead of a separate scan of the partials.
constexpr int64_t kSumPartialsMax = 4096;

template <class Tin, class T>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const Tin* __restrict__ in, int64_t n,
                                                                   T* __restrict__ partials) {
  __shared__ T wsum[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T s = 0;
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    const int64_t i = base + it * kScanThreads + threadIdx.x;
    if (i < n) s += (T)in[i];
  }
  T total;
  block_exclusive_scan<T>(s, wsum, total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// Scans one tile per block.  A tile's starting value is offsets[tile] when
// `offsets` is given, else the sum of partials[0, tile) when `partials` is
// given (each block adds up the tile sums before it), else 0.
template <class Tin, class T>
__global__ __launch_bounds__(kScanThreads) void scan_tile_kernel(const Tin* __restrict__ in, T* __restrict__ out,
                                                                 int64_t n, const T* __restrict__ offsets,
                                                                 const T* __restrict__ partials,
                                                                 T* __restrict__ total_out) {
  __shared__ T tile[kScanTile];
  __shared__ T wsum[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T off = 0;
  if (offsets) {
    off = offsets[blockIdx.x];
  } else if (partials) {
    T p = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kScanThreads) p += partials[b];
    block_exclusive_scan<T>(p, wsum, off);
  }
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    const int64_t i = base + it * kScanThreads + threadIdx.x;
    tile[it * kScanThreads + threadIdx.x] = i < n ? (T)in[i] : T(0);
  }
  __syncthreads();
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    v[it] = tile[threadIdx.x * kScanItems + it];
    s += v[it];
  }
  T total;
  T run = block_exclusive_scan<T>(s, wsum, total);
  run += off;
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    tile[threadIdx.x * kScanItems + it] = run;
    run += v[it];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    const int64_t i = base + it * kScanThreads + threadIdx.x;
    if (i < n) out[i] = tile[it * kScanThreads + threadIdx.x];
  }
  if (total_out && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total_out = off + total;
}

template <class Tin, class T>
void scan_impl(lco_ctx ctx, const Tin* in, T* out, int64_t n, T* total, const char* name) {
  if (n <= 0) {
    if (total) memset_async(ctx, total, 0, sizeof(T));
    return;
  }
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    LCO_LAUNCH(ctx, name, (scan_tile_kernel<Tin, T>), 1, kScanThreads, 0, in, out, n, (const T*)nullptr,
               (const T*)nullptr, total);
    return;
  }
  Scratch s(ctx);
  T* partials = s.get<T>(tiles);
  LCO_LAUNCH(ctx, "scan_reduce", (scan_reduce_kernel<Tin, T>), tiles, kScanThreads, 0, in, n, partials);
  if (tiles <= kSumPartialsMax) {
    // each tile adds up the partial sums before it (two launches instead of three)
    LCO_LAUNCH(ctx, name, (scan_tile_kernel<Tin, T>), tiles, kScanThreads, 0, in, out, n, (const T*)nullptr,
               (const T*)partials, total);
    return;
  }
  T* poff = s.get<T>(tiles);
  scan_impl<T, T>(ctx, partials, poff, tiles, (T*)nullptr, name);
  LCO_LAUNCH(ctx, name, (scan_tile_kernel<Tin, T>), tiles, kScanThreads, 0, in, out, n, (const T*)poff,
             (const T*)nullptr, total);
}

}  // namespace

void scan_u32(lco_ctx ctx, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total) {
  scan_impl<uint32_t, uint32_t>(ctx, in, out, n, total, "scan_u32");
}

void scan_u64(lco_ctx ctx, const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total) {
  scan_impl<uint64_t, uint64_t>(ctx, in, out, n, total, "scan_u64");
}

void scan_u32_u64(lco_ctx ctx, const uint32_t* in, uint64_t* out, int64_t n, uint64_t* total) {
  scan_impl<uint32_t, uint64_t>(ctx, in, out, n, total, "scan_u64");
}

}  // namespace lco
