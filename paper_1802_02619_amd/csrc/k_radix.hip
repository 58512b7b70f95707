// Radix permutation engine (Section 4.1) and the stable LSD radix sort it is built on.
//
// The paper's RP sorts, stably, only the digit groups a permutation disturbs.
// Here every pass is a stable least-significant-digit pass over a tile of
// (LIV, value) pairs: each wave ranks its elements per digit with ballot
// matching (all lanes holding the same digit are found with one ballot per
// digit bit), waves are combined with per-digit counters in LDS, the tile is
// reordered by digit in LDS, and then written out in digit runs so that
// consecutive lanes store consecutive addresses.  Tile bucket offsets come from
// a device-wide scan of per-tile digit counts (reduce-then-scan).  The LIV
// shuffle (recomputing LIVs in the new lexicographical order) is fused into the
// first pass's loads.
#include <algorithm>
#include <cstdlib>

#include "device_common.h"

namespace lco {

namespace {

constexpr int kRxWaves = 16;
constexpr int kRxThreads = kRxWaves * kWave;
constexpr int kRxItems = 4;
constexpr int kRxTile = kRxThreads * kRxItems;  // 4096
constexpr int kRxBins = 256;                    // digits of at most 8 bits
// the digit-count kernel covers the same 4096-element tiles with fewer, longer waves
constexpr int kCntWaves = 4;
constexpr int kCntThreads = kCntWaves * kWave;
constexpr int kCntItems = kRxTile / kCntThreads;

constexpr int kLdsWaves = 8;
constexpr int kLdsThreads = kLdsWaves * kWave;
constexpr int kLdsItems = 16;
constexpr int kLdsTile = kLdsThreads * kLdsItems;  // 8192: single-tile and segmented sorts

__device__ __forceinline__ uint32_t digit_of(uint64_t key, int shift, uint32_t mask) {
  return (uint32_t)(key >> shift) & mask;
}

// Peers: lanes of this wave holding the same digit (one ballot per digit bit).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int dbits) {
  uint64_t peers = ~0ull;
  for (int b = 0; b < dbits; ++b) {
    const int bit = (d >> b) & 1;
    const uint64_t bal = __ballot(bit);
    peers &= bit ? bal : ~bal;
  }
  return peers;
}

// Stable rank of ITEMS elements per lane within the block, by digit.  Element
// order is (wave, item, lane).  On return pos[it] is the element's position in
// the tile sorted by digit; dstart[d] is the first position of digit d.
template <int WAVES, int ITEMS>
__device__ __forceinline__ void block_rank(const uint32_t (&dg)[ITEMS], uint32_t (&pos)[ITEMS], int dbits,
                                           uint32_t (*cnt)[kRxBins], uint32_t* dstart, uint32_t* wsum) {
  const int wave = threadIdx.x / kWave;
  const uint32_t bins = 1u << dbits;
  for (int i = threadIdx.x; i < WAVES * kRxBins; i += WAVES * kWave) (&cnt[0][0])[i] = 0;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t peers = match_digit(dg[it], dbits);
    const uint32_t before = (uint32_t)__popcll(peers & lanemask_lt());
    const uint32_t c = cnt[wave][dg[it]];
    pos[it] = c + before;
    if (before == 0) cnt[wave][dg[it]] = c + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  uint32_t tot = 0;
  for (uint32_t d = threadIdx.x; d < (uint32_t)kRxBins; d += WAVES * kWave) {
    // only threads d < bins hold digits; WAVES*64 >= 256 so each thread has at most one digit
    if (d < bins) {
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = cnt[w][d];
        cnt[w][d] = run;
        run += c;
      }
      tot = run;
    }
  }
  uint32_t all;
  const uint32_t ex = block_exclusive_scan<uint32_t>(tot, wsum, all);
  if (threadIdx.x < bins) dstart[threadIdx.x] = ex;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) pos[it] += dstart[dg[it]] + cnt[wave][dg[it]];
}

// ---------------------------------------------------------------- global passes

template <bool SHUF>
__global__ __launch_bounds__(kCntThreads) void rx_count_kernel(const uint64_t* __restrict__ livs, int64_t n,
                                                              ShuffleParams sp, KeyParams kp, int shift,
                                                              uint32_t mask, uint32_t* __restrict__ counts,
                                                              int64_t num_tiles) {
  __shared__ uint32_t hist[kCntWaves][kRxBins];
  for (int i = threadIdx.x; i < kCntWaves * kRxBins; i += kCntThreads) (&hist[0][0])[i] = 0;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int64_t base = (int64_t)blockIdx.x * kRxTile + (int64_t)wave * kCntItems * kWave + lane;
  uint64_t x[kCntItems];
#pragma unroll
  for (int it = 0; it < kCntItems; ++it) {
    const int64_t e = base + it * kWave;
    x[it] = e < n ? livs[e] : 0;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kCntItems; ++it) {
    const int64_t e = base + it * kWave;
    if (e < n) {
      uint64_t v = x[it];
      if (SHUF) v = shuffle_liv(sp, v);
      const uint64_t key = fd_div(kp.key_div, v) - kp.key_base;
      atomicAdd(&hist[wave][digit_of(key, shift, mask)], 1u);
    }
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d <= mask; d += kCntThreads) {
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < kCntWaves; ++w) s += hist[w][d];
    counts[(int64_t)d * num_tiles + blockIdx.x] = s;
  }
}

template <bool SHUF>
__global__ __launch_bounds__(kRxThreads) void rx_scatter_kernel(
    const uint64_t* __restrict__ livs, const double* __restrict__ vals, int64_t n, ShuffleParams sp, KeyParams kp,
    int shift, int dbits, const uint32_t* __restrict__ offsets, int64_t num_tiles, uint64_t* __restrict__ out_livs,
    double* __restrict__ out_vals) {
  __shared__ uint32_t cnt[kRxWaves][kRxBins];
  __shared__ uint32_t dstart[kRxBins];
  __shared__ uint32_t gbase[kRxBins];
  __shared__ uint32_t wsum[kRxWaves + 1];
  __shared__ uint64_t s_buf[kRxTile];  // the tile in digit order: LIVs, then values
  __shared__ uint8_t s_dig[kRxTile];
  const uint32_t mask = (1u << dbits) - 1u;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int64_t tile0 = (int64_t)blockIdx.x * kRxTile;
  const int64_t base = tile0 + (int64_t)wave * kRxItems * kWave + lane;
  for (uint32_t d = threadIdx.x; d <= mask; d += kRxThreads) gbase[d] = offsets[(int64_t)d * num_tiles + blockIdx.x];
  uint64_t lv[kRxItems];
  double vv[kRxItems];
  const uint64_t* lp = livs + base;
  const double* vp = vals + base;
#pragma unroll
  for (int it = 0; it < kRxItems; ++it) lv[it] = base + it * kWave < n ? lp[it * kWave] : 0;
  uint32_t dg[kRxItems], pos[kRxItems];
#pragma unroll
  for (int it = 0; it < kRxItems; ++it) {
    const int64_t e = base + it * kWave;
    if (SHUF) lv[it] = shuffle_liv(sp, lv[it]);
    dg[it] = e < n ? digit_of(fd_div(kp.key_div, lv[it]) - kp.key_base, shift, mask) : mask;
  }
  // the values are needed only after the LIVs are written: their loads overlap the ranking
#pragma unroll
  for (int it = 0; it < kRxItems; ++it) vv[it] = base + it * kWave < n ? vp[it * kWave] : 0.0;
  block_rank<kRxWaves, kRxItems>(dg, pos, dbits, cnt, dstart, wsum);
  // LIVs and then values pass through one LDS buffer (half the LDS of staging
  // both at once, so more workgroups fit on a compute unit); each is written
  // out in digit runs, consecutive lanes to consecutive addresses
#pragma unroll
  for (int it = 0; it < kRxItems; ++it) {
    s_buf[pos[it]] = lv[it];
    s_dig[pos[it]] = (uint8_t)dg[it];
  }
  __syncthreads();
  const int valid = (int)((n - tile0) < kRxTile ? (n - tile0) : kRxTile);
  for (int i = threadIdx.x; i < valid; i += kRxThreads) {
    const uint32_t d = s_dig[i];
    out_livs[(uint64_t)gbase[d] + (uint32_t)(i - (int)dstart[d])] = s_buf[i];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kRxItems; ++it) s_buf[pos[it]] = (uint64_t)__double_as_longlong(vv[it]);
  __syncthreads();
  for (int i = threadIdx.x; i < valid; i += kRxThreads) {
    const uint32_t d = s_dig[i];
    out_vals[(uint64_t)gbase[d] + (uint32_t)(i - (int)dstart[d])] = __longlong_as_double((long long)s_buf[i]);
  }
}

// ---------------------------------------------------------------- LDS-resident sorts

// Sorts up to kLdsThreads * ITEMS elements held in registers (element order
// (wave, item, lane)) by bits [0, bits) of key(x) = x / key_div - key_base,
// stably, leaving the result in s_liv / s_val positions [0, valid).
template <int ITEMS = kLdsItems>
__device__ __forceinline__ void lds_sort(uint64_t (&lv)[ITEMS], double (&vv)[ITEMS], int valid, int bits,
                                         int digit_cap, const FastDiv& key_div, uint64_t key_base,
                                         uint32_t (*cnt)[kRxBins], uint32_t* dstart, uint32_t* wsum,
                                         uint64_t* s_liv, double* s_val) {
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int passes = bits > 0 ? (bits + digit_cap - 1) / digit_cap : 0;
  const int dbits = passes ? (bits + passes - 1) / passes : 1;
  const uint32_t mask = (1u << dbits) - 1u;
  const int ebase = wave * ITEMS * kWave + lane;
  if (passes == 0) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int e = ebase + it * kWave;
      s_liv[e] = lv[it];
      s_val[e] = vv[it];
    }
    __syncthreads();
    return;
  }
  for (int p = 0; p < passes; ++p) {
    uint32_t dg[ITEMS], pos[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int e = ebase + it * kWave;
      dg[it] = e < valid ? digit_of(fd_div(key_div, lv[it]) - key_base, p * dbits, mask) : mask;
    }
    block_rank<kLdsWaves, ITEMS>(dg, pos, dbits, cnt, dstart, wsum);
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      s_liv[pos[it]] = lv[it];
      s_val[pos[it]] = vv[it];
    }
    __syncthreads();
    if (p + 1 < passes) {
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) {
        const int e = ebase + it * kWave;
        lv[it] = s_liv[e];
        vv[it] = s_val[e];
      }
      __syncthreads();
    }
  }
}

template <bool SHUF>
__global__ __launch_bounds__(kLdsThreads) void rx_single_kernel(const uint64_t* __restrict__ livs,
                                                                const double* __restrict__ vals, int n,
                                                                ShuffleParams sp, KeyParams kp, int bits,
                                                                int digit_cap, uint64_t* __restrict__ out_livs,
                                                                double* __restrict__ out_vals) {
  __shared__ uint32_t cnt[kLdsWaves][kRxBins];
  __shared__ uint32_t dstart[kRxBins];
  __shared__ uint32_t wsum[kLdsWaves + 1];
  __shared__ uint64_t s_liv[kLdsTile];
  __shared__ double s_val[kLdsTile];
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int ebase = wave * kLdsItems * kWave + lane;
  uint64_t lv[kLdsItems];
  double vv[kLdsItems];
#pragma unroll
  for (int it = 0; it < kLdsItems; ++it) {
    const int e = ebase + it * kWave;
    lv[it] = e < n ? livs[e] : 0;
    vv[it] = e < n ? vals[e] : 0.0;
    if (SHUF && e < n) lv[it] = shuffle_liv(sp, lv[it]);
  }
  lds_sort(lv, vv, n, bits, digit_cap, kp.key_div, kp.key_base, cnt, dstart, wsum, s_liv, s_val);
  for (int i = threadIdx.x; i < n; i += kLdsThreads) {
    out_livs[i] = s_liv[i];
    out_vals[i] = s_val[i];
  }
}

// First index >= x that starts a segment (segment id = old LIV / seg_div), or n.
__device__ int64_t seg_start_at_or_after(const uint64_t* __restrict__ livs, int64_t n, const FastDiv& seg_div,
                                         int64_t x) {
  if (x >= n) return n;
  const uint64_t s = fd_div(seg_div, livs[x]);
  if (x == 0 || fd_div(seg_div, livs[x - 1]) != s) return x;
  // gallop forward to bracket the segment's end, then bisect: the number of
  // dependent loads grows with the log of the segment's length, not of n
  int64_t lo = x, hi = n, step = 1;  // livs[lo] lies in segment s; the answer lies in (lo, hi]
  while (lo + step < n) {
    if (fd_div(seg_div, livs[lo + step]) != s) {
      hi = lo + step;
      break;
    }
    lo += step;
    step *= 2;
  }
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (fd_div(seg_div, livs[mid]) == s) lo = mid;
    else hi = mid;
  }
  return hi;
}

// Segmented radix permutation: tiles hold whole segments of constant leading
// resting modes (Section 4.1: such regions sort independently), each sorted in
// LDS by the tile-relative key.  Sets *overflow if a tile exceeds capacity.
// Two tile sizes: kLdsThreads x 8 (64 KB of LDS, two blocks per compute unit)
// and kLdsThreads x 16 (one block per compute unit).
template <int ITEMS>
__global__ __launch_bounds__(kLdsThreads, ITEMS <= kLdsItems / 2 ? 4 : 1) void rx_segmented_kernel(
    const uint64_t* __restrict__ livs, const double* __restrict__ vals, int64_t n, ShuffleParams sp,
    FastDiv seg_div, FastDiv key_div, uint64_t key_range, int64_t nominal, int digit_cap,
    uint64_t* __restrict__ out_livs, double* __restrict__ out_vals, uint32_t* __restrict__ overflow) {
  constexpr int kTile = kLdsThreads * ITEMS;
  __shared__ uint32_t cnt[kLdsWaves][kRxBins];
  __shared__ uint32_t dstart[kRxBins];
  __shared__ uint32_t wsum[kLdsWaves + 1];
  __shared__ uint64_t s_liv[kTile];
  __shared__ double s_val[kTile];
  __shared__ int64_t bounds[2];
  if (threadIdx.x < 2) bounds[threadIdx.x] = seg_start_at_or_after(livs, n, seg_div, ((int64_t)blockIdx.x + threadIdx.x) * nominal);
  __syncthreads();
  const int64_t s0 = bounds[0], s1 = bounds[1];
  const int64_t len = s1 - s0;
  if (len <= 0) return;
  if (len > kTile) {
    if (threadIdx.x == 0) atomicOr(overflow, 1u);
    return;
  }
  const int valid = (int)len;
  const uint64_t seg_first = fd_div(seg_div, livs[s0]);
  const uint64_t seg_last = fd_div(seg_div, livs[s1 - 1]);
  const uint64_t key_base = seg_first * key_range;
  const uint64_t range_max = (seg_last - seg_first + 1) * key_range - 1;
  const int bits = range_max ? 64 - __builtin_clzll(range_max) : 0;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int ebase = wave * ITEMS * kWave + lane;
  uint64_t lv[ITEMS];
  double vv[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int e = ebase + it * kWave;
    lv[it] = e < valid ? shuffle_liv(sp, livs[s0 + e]) : 0;
    vv[it] = e < valid ? vals[s0 + e] : 0.0;
  }
  lds_sort<ITEMS>(lv, vv, valid, bits, digit_cap, key_div, key_base, cnt, dstart, wsum, s_liv, s_val);
  for (int i = threadIdx.x; i < valid; i += kLdsThreads) {
    out_livs[s0 + i] = s_liv[i];
    out_vals[s0 + i] = s_val[i];
  }
}

// Segmented permutation for short segments: every entry of a segment of at
// most kSmallSeg entries finds its place directly, as the segment's start plus
// the number of the segment's entries with a smaller (key, input position).
// Segments stay where they are (they are the leading resting modes), so one
// read and one write per entry suffice.  Tiles hold the segments that start in
// a nominal range of kSegTile / 2 entries.  Sets *overflow if a tile exceeds
// kSegTile entries or holds a longer segment.
constexpr int kSegThreads = 512;
constexpr int kSegItems = 8;
constexpr int kSegTile = kSegThreads * kSegItems;  // 4096
constexpr int kSmallSeg = 32;

__global__ __launch_bounds__(kSegThreads) void rx_smallseg_kernel(
    const uint64_t* __restrict__ livs, const double* __restrict__ vals, int64_t n, ShuffleParams sp,
    FastDiv seg_div, FastDiv key_div, uint64_t key_range, int64_t nominal, uint64_t* __restrict__ out_livs,
    double* __restrict__ out_vals, uint32_t* __restrict__ overflow) {
  __shared__ uint64_t s_a[kSegTile];  // tile-relative keys, then the output LIVs
  __shared__ uint64_t s_b[kSegTile];  // tile-relative segment ids, then the output values
  __shared__ int64_t bounds[2];
  __shared__ int too_long;
  if (threadIdx.x == 0) {
    // a segment holding both ends of a 33-entry stretch at the nominal cut is too long (two loads)
    const int64_t x = (int64_t)blockIdx.x * nominal;
    too_long = x + kSmallSeg < n && fd_div(seg_div, livs[x]) == fd_div(seg_div, livs[x + kSmallSeg]);
  }
  __syncthreads();
  if (too_long) {
    if (threadIdx.x == 0) atomicOr(overflow, 1u);
    return;
  }
  if (threadIdx.x < 2)
    bounds[threadIdx.x] = seg_start_at_or_after(livs, n, seg_div, ((int64_t)blockIdx.x + threadIdx.x) * nominal);
  __syncthreads();
  const int64_t s0 = bounds[0], s1 = bounds[1];
  const int64_t len64 = s1 - s0;
  if (len64 <= 0) return;
  if (len64 > kSegTile) {
    if (threadIdx.x == 0) atomicOr(overflow, 1u);
    return;
  }
  const int len = (int)len64;
  const uint64_t seg_first = fd_div(seg_div, livs[s0]);
  // give up at once when the tile's first segment is already too long (one load)
  if (len > kSmallSeg && fd_div(seg_div, livs[s0 + kSmallSeg]) == seg_first) {
    if (threadIdx.x == 0) atomicOr(overflow, 1u);
    return;
  }
  const uint64_t key_base = seg_first * key_range;
  uint64_t lv[kSegItems], key[kSegItems], sg[kSegItems];
  double vv[kSegItems];
#pragma unroll
  for (int it = 0; it < kSegItems; ++it) {
    const int e = threadIdx.x + it * kSegThreads;
    lv[it] = 0;
    key[it] = 0;
    sg[it] = 0;
    vv[it] = 0.0;
    if (e < len) {
      const uint64_t old = livs[s0 + e];
      lv[it] = shuffle_liv(sp, old);
      vv[it] = vals[s0 + e];
      sg[it] = fd_div(seg_div, old) - seg_first;
      key[it] = fd_div(key_div, lv[it]) - key_base;
      s_a[e] = key[it];
      s_b[e] = sg[it];
    }
  }
  __syncthreads();
  int pos[kSegItems];
#pragma unroll
  for (int it = 0; it < kSegItems; ++it) {
    const int e = threadIdx.x + it * kSegThreads;
    pos[it] = 0;
    if (e < len) {
      int lo = e, hi = e + 1;
      while (lo > 0 && e - lo < kSmallSeg && s_b[lo - 1] == sg[it]) --lo;
      while (hi < len && hi - lo <= kSmallSeg && s_b[hi] == sg[it]) ++hi;
      if (hi - lo > kSmallSeg || (lo > 0 && s_b[lo - 1] == sg[it])) {
        too_long = 1;
      } else {
        int r = lo;
        for (int j = lo; j < hi; ++j) {
          const uint64_t kj = s_a[j];
          r += (kj < key[it] || (kj == key[it] && j < e)) ? 1 : 0;
        }
        pos[it] = r;
      }
    }
  }
  __syncthreads();
  if (too_long) {
    if (threadIdx.x == 0) atomicOr(overflow, 1u);
    return;
  }
#pragma unroll
  for (int it = 0; it < kSegItems; ++it) {
    const int e = threadIdx.x + it * kSegThreads;
    if (e < len) {
      s_a[pos[it]] = lv[it];
      s_b[pos[it]] = (uint64_t)__double_as_longlong(vv[it]);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < len; i += kSegThreads) {
    out_livs[s0 + i] = s_a[i];
    out_vals[s0 + i] = __longlong_as_double((long long)s_b[i]);
  }
}

template <bool SHUF>
__global__ void shuffle_copy_kernel(const uint64_t* __restrict__ livs, const double* __restrict__ vals, int64_t n,
                                    ShuffleParams sp, uint64_t* __restrict__ out_livs,
                                    double* __restrict__ out_vals) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t x = livs[i];
    out_livs[i] = SHUF ? shuffle_liv(sp, x) : x;
    out_vals[i] = vals[i];
  }
}

int grid_for(lco_ctx ctx, int64_t n, int threads) {
  const int64_t want = (n + threads - 1) / threads;
  const int64_t cap = (int64_t)ctx->num_cus * 16;
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, cap));
}

}  // namespace

ShuffleParams make_shuffle(int order, const uint64_t* dims, const uint64_t* new_weight_of_input_mode) {
  ShuffleParams sp;
  sp.order = order;
  sp.all_pow2 = 1;
  uint32_t at = 0;
  for (int q = 0; q < order; ++q) {
    sp.dim[q] = make_fastdiv(dims[q]);
    sp.new_weight[q] = new_weight_of_input_mode[q];
    const uint64_t w = new_weight_of_input_mode[q];
    if (!sp.dim[q].pow2 || (w & (w - 1)) != 0) {
      sp.all_pow2 = 0;
      continue;
    }
    sp.in_shift[q] = at;
    sp.in_mask[q] = dims[q] - 1;
    sp.out_shift[q] = (uint32_t)__builtin_ctzll(w);
    at += sp.dim[q].shift;
  }
  return sp;
}

int default_digit_cap() {
  static int cap = [] {
    const char* e = std::getenv("LCO_DIGIT_BITS");
    int v = e ? std::atoi(e) : 8;
    return std::min(8, std::max(1, v));
  }();
  return cap;
}

void shuffle_copy(lco_ctx ctx, const uint64_t* in_livs, const double* in_vals, uint64_t* out_livs,
                  double* out_vals, int64_t n, const ShuffleParams* shuffle) {
  if (n <= 0) return;
  if (shuffle) {
    LCO_LAUNCH(ctx, "shuffle_copy", shuffle_copy_kernel<true>, grid_for(ctx, n, 256), 256, 0, in_livs, in_vals, n,
               *shuffle, out_livs, out_vals);
  } else {
    LCO_LAUNCH(ctx, "shuffle_copy", shuffle_copy_kernel<false>, grid_for(ctx, n, 256), 256, 0, in_livs, in_vals, n,
               ShuffleParams{}, out_livs, out_vals);
  }
}

void radix_sort_pairs(lco_ctx ctx, const uint64_t* in_livs, const double* in_vals, uint64_t* out_livs,
                      double* out_vals, int64_t n, const ShuffleParams* shuffle, const KeyParams& key, int bits,
                      int digit_cap) {
  if (n <= 0) return;
  if (bits <= 0) {
    shuffle_copy(ctx, in_livs, in_vals, out_livs, out_vals, n, shuffle);
    return;
  }
  if (n > (int64_t)UINT32_MAX) fail(LCO_E_UNSUPPORTED, "radix sort: more than 2^32-1 elements");
  if (digit_cap < 1 || digit_cap > 8) digit_cap = default_digit_cap();
  const ShuffleParams sp = shuffle ? *shuffle : ShuffleParams{};
  if (n <= kLdsTile) {
    if (shuffle) {
      LCO_LAUNCH(ctx, "rx_single", rx_single_kernel<true>, 1, kLdsThreads, 0, in_livs, in_vals, (int)n, sp, key, bits,
                 digit_cap, out_livs, out_vals);
    } else {
      LCO_LAUNCH(ctx, "rx_single", rx_single_kernel<false>, 1, kLdsThreads, 0, in_livs, in_vals, (int)n, sp, key,
                 bits, digit_cap, out_livs, out_vals);
    }
    return;
  }
  const int passes = (bits + digit_cap - 1) / digit_cap;
  const int dbits = (bits + passes - 1) / passes;
  const uint32_t bins = 1u << dbits;
  const int64_t num_tiles = (n + kRxTile - 1) / kRxTile;
  Scratch s(ctx);
  uint32_t* counts = s.get<uint32_t>((size_t)bins * num_tiles);
  uint32_t* offs = s.get<uint32_t>((size_t)bins * num_tiles);
  uint64_t* tl = nullptr;
  double* tv = nullptr;
  if (passes >= 2) {
    tl = s.get<uint64_t>(n);
    tv = s.get<double>(n);
  }
  const uint64_t* src_l = in_livs;
  const double* src_v = in_vals;
  for (int p = 0; p < passes; ++p) {
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    uint64_t* dl = to_out ? out_livs : tl;
    double* dv = to_out ? out_vals : tv;
    const int shift = p * dbits;
    if (p == 0 && shuffle) {
      LCO_LAUNCH(ctx, "rx_count", rx_count_kernel<true>, num_tiles, kCntThreads, 0, src_l, n, sp, key, shift,
                 bins - 1, counts, num_tiles);
      scan_u32(ctx, counts, offs, (int64_t)bins * num_tiles, nullptr);
      LCO_LAUNCH(ctx, "rx_scatter", rx_scatter_kernel<true>, num_tiles, kRxThreads, 0, src_l, src_v, n, sp, key,
                 shift, dbits, offs, num_tiles, dl, dv);
    } else {
      LCO_LAUNCH(ctx, "rx_count", rx_count_kernel<false>, num_tiles, kCntThreads, 0, src_l, n, sp, key, shift,
                 bins - 1, counts, num_tiles);
      scan_u32(ctx, counts, offs, (int64_t)bins * num_tiles, nullptr);
      LCO_LAUNCH(ctx, "rx_scatter", rx_scatter_kernel<false>, num_tiles, kRxThreads, 0, src_l, src_v, n, sp, key,
                 shift, dbits, offs, num_tiles, dl, dv);
    }
    src_l = dl;
    src_v = dv;
  }
}

bool segmented_permute(lco_ctx ctx, const uint64_t* in_livs, const double* in_vals, uint64_t* out_livs,
                       double* out_vals, int64_t n, const ShuffleParams& shuffle, const FastDiv& seg_div,
                       const FastDiv& key_div, uint64_t key_range, bool small_first, bool half_first) {
  if (n <= 0) return true;
  Scratch s(ctx);
  uint64_t* word = s.get<uint64_t>(1);  // the kernel ORs its flag into the low half
  if (small_first) {
    memset_async(ctx, word, 0, sizeof(uint64_t));
    const int64_t nominal = kSegTile / 2;
    const int64_t tiles = (n + nominal - 1) / nominal;
    LCO_LAUNCH(ctx, "rx_smallseg", rx_smallseg_kernel, tiles, kSegThreads, 0, in_livs, in_vals, n, shuffle, seg_div,
               key_div, key_range, nominal, out_livs, out_vals, (uint32_t*)word);
    const uint64_t* words[1] = {word};
    if (readback(ctx, words, 1)[0] == 0) return true;
  }
  // the half-size tile first when segments are expected to fit it
  if (half_first) {
    memset_async(ctx, word, 0, sizeof(uint64_t));
    const int64_t nominal = kLdsTile / 4;
    const int64_t tiles = (n + nominal - 1) / nominal;
    LCO_LAUNCH(ctx, "rx_segmented", rx_segmented_kernel<kLdsItems / 2>, tiles, kLdsThreads, 0, in_livs, in_vals, n,
               shuffle, seg_div, key_div, key_range, nominal, default_digit_cap(), out_livs, out_vals,
               (uint32_t*)word);
    const uint64_t* words[1] = {word};
    if (readback(ctx, words, 1)[0] == 0) return true;
  }
  memset_async(ctx, word, 0, sizeof(uint64_t));
  const int64_t nominal = kLdsTile / 2;
  const int64_t tiles = (n + nominal - 1) / nominal;
  LCO_LAUNCH(ctx, "rx_segmented", rx_segmented_kernel<kLdsItems>, tiles, kLdsThreads, 0, in_livs, in_vals, n, shuffle,
             seg_div, key_div, key_range, nominal, default_digit_cap(), out_livs, out_vals, (uint32_t*)word);
  const uint64_t* words[1] = {word};
  const uint64_t* r = readback(ctx, words, 1);
  return r[0] == 0;
}

void permute_storage(lco_ctx ctx, const lco_tensor_s* in, const RpDetail& plan, uint64_t* out_livs,
                     double* out_vals) {
  const int64_t n = in->nnz;
  if (n == 0) return;
  const ShuffleParams sp = make_shuffle(in->order, in->dims, plan.new_weight_of_input_mode);
  KeyParams kp;
  kp.key_div = make_fastdiv(plan.pub.key_div);
  kp.key_base = 0;
  const int cap = default_digit_cap();
  switch (plan.pub.method) {
    case 0:
      shuffle_copy(ctx, in->livs, in->vals, out_livs, out_vals, n, &sp);
      return;
    case 1:
    case 2:
    case 4:
      radix_sort_pairs(ctx, in->livs, in->vals, out_livs, out_vals, n, &sp, kp, plan.sort_bits, cap);
      return;
    case 3:
      // segments larger than a tile on average: some segment is, and the tile sort would only give up
      if (plan.avg_segment <= (double)kLdsTile &&
          segmented_permute(ctx, in->livs, in->vals, out_livs, out_vals, n, sp, make_fastdiv(plan.pub.seg_div),
                            kp.key_div, plan.pub.key_range, plan.avg_segment <= 8.0,
                            plan.avg_segment <= (double)kLdsTile / 4))
        return;
      radix_sort_pairs(ctx, in->livs, in->vals, out_livs, out_vals, n, &sp, kp, plan.sort_bits, cap);
      return;
    default:
      fail(LCO_E_ARG, "permute: unknown method");
  }
}

}  // namespace lco
