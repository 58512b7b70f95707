// Device code of the one-wave-per-row product, shared by the per-call row
// engine and the batched engine so that both compute every row identically.
#pragma once

#include "device_common.h"
#include "rows.h"

namespace lco {
namespace {

constexpr int kRowThreads = kRowWaves * kWave;
constexpr uint64_t kEmpty = ~0ull;

// Rows handled by one wave.  Workgroups are dispatched round-robin over the
// eight XCDs (block b runs on XCD b % 8), each with its own L2; giving every
// XCD one contiguous share of the rows keeps neighbouring rows, which gather
// the same rows of B', in one L2.  Every row in [0, n) is visited exactly once
// for any grid size.
constexpr uint32_t kXcds = 8;
struct RowSpan {
  uint64_t first, end, step;
};
__device__ __forceinline__ RowSpan xcd_row_span(uint64_t n, int w) {
  const uint32_t G = gridDim.x, b = blockIdx.x;
  if (G < kXcds) return {(uint64_t)b * kRowWaves + w, n, (uint64_t)G * kRowWaves};
  const uint32_t x = b % kXcds, slot = b / kXcds, nb = (G - x + kXcds - 1) / kXcds;
  const uint64_t chunk = (n + kXcds - 1) / kXcds;
  const uint64_t begin = x * chunk < n ? x * chunk : n;
  const uint64_t end = begin + chunk < n ? begin + chunk : n;
  return {begin + (uint64_t)slot * kRowWaves + w, end, (uint64_t)nb * kRowWaves};
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const uint64_t b = __double_as_longlong(x);
  const uint32_t lo = readlane_u32((uint32_t)b, l), hi = readlane_u32((uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Bitonic sort of one (key, idx, val) triple per lane across the wave, ascending
// by (key, idx).
__device__ __forceinline__ void wave_bitonic(uint64_t& key, uint32_t& idx, double& val) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint64_t ok = __shfl_xor(key, j, kWave);
      const uint32_t oi = __shfl_xor(idx, j, kWave);
      const double ov = __shfl_xor(val, j, kWave);
      const bool up = (lane & k) == 0;
      const bool lower = (lane & j) == 0;
      const bool other_less = ok < key || (ok == key && oi < idx);
      const bool take = (lower == up) ? other_less : !other_less;
      if (take) {
        key = ok;
        idx = oi;
        val = ov;
      }
    }
  }
}

__device__ __forceinline__ uint32_t hash_slot(uint64_t c) {
  return (uint32_t)((c * 0x9E3779B97F4A7C15ull) >> 57);  // 7 bits
}

// Per-row shape codes of the one-wave kernel.
constexpr uint8_t kShapeSearch = 7;    // at most 64 products, located by search
constexpr uint8_t kShapeTiny = 8;      // at most kTinyEntries entries and kTinyProducts products: one lane per row
constexpr uint8_t kShapeCopy = 9;      // one entry (more than kTinyProducts products): the row is a scaled B' row
constexpr uint8_t kShapeSkip = 0xFF;   // no products, or a long row
constexpr int kTinyEntries = 4;
constexpr int kTinyProducts = 16;
// Rows with at most 64 products and 64 entries run one wave per row.  When the
// row's entries times W (the next power of two at least its longest B' row) fit
// the 64 lanes, lane = entry * W + position ("entry-major"): each lane knows its
// product without any search.  The shape code is log2 W for those rows.
__device__ __forceinline__ bool small_row(uint64_t f, uint32_t t) {
  return f <= (uint64_t)kWave && t <= (uint32_t)kWave;
}

// Shared memory of the one-wave-per-row kernels (one row table per wave).
struct RowSmem {
  uint64_t (*hash)[2 * kWave];
  uint32_t (*hash32)[2 * kWave];
  double (*vals)[kWave + 8];      // each lane's product value, and a zero at index kWave
  uint64_t (*lanes)[2 * kWave];   // per hash slot: the lanes whose product has that column
  uint32_t (*own)[kWave];
};

__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int l) {
  return ((uint64_t)readlane_u32((uint32_t)(x >> 32), l) << 32) | readlane_u32((uint32_t)x, l);
}

// The products of one small row from the entry window (lane l holds entry w0 + l:
// its product count, B' row start, value, and its A' LIV (numeric pass) or
// j * n' (symbolic pass: the LIV of its B' row's first position)); each lane
// ends up with at most one product: its A' entry `ent` within the row, its
// column and (numeric) value.
template <bool NUMERIC>
__device__ __forceinline__ void window_products(const uint64_t* __restrict__ b_livs, const double* __restrict__ b_vals,
                                                uint64_t np, uint64_t kp, uint32_t e0, int t, uint64_t row,
                                                uint8_t sh, int lane, int64_t w0, uint32_t x_len, uint32_t x_bs,
                                                uint64_t x_jn, double x_av, bool& valid, int& ent, uint64_t& col,
                                                double& v) {
  valid = false;
  ent = 0;
  col = kEmpty;
  v = 0.0;
  const int first = (int)((int64_t)e0 - w0);  // window lane of the row's first entry
  if (sh != kShapeSearch) {
    // entry-major lanes: lane = entry * W + position
    const int e = lane >> sh, k = lane & ((1 << sh) - 1);
    const int src = (first + e) & (kWave - 1);
    const uint32_t len = (uint32_t)__shfl((int)x_len, src, kWave);
    const uint32_t bs = (uint32_t)__shfl((int)x_bs, src, kWave);
    const uint64_t jn = __shfl(x_jn, src, kWave);
    const double av = NUMERIC ? __shfl(x_av, src, kWave) : 0.0;
    if (e < t && (uint32_t)k < len) {
      const uint32_t q = bs + (uint32_t)k;
      valid = true;
      ent = e;
      col = b_livs[q] - (NUMERIC ? np * (jn - kp * row) : jn);
      if (NUMERIC) v = av * b_vals[q];
    }
    return;
  }
  // general small row: lane p takes product p, found by a binary search over the
  // entries' inclusive product counts
  const int src = (first + lane) & (kWave - 1);
  uint32_t len = (uint32_t)__shfl((int)x_len, src, kWave);
  const uint32_t bs = (uint32_t)__shfl((int)x_bs, src, kWave);
  const uint64_t jn = __shfl(x_jn, src, kWave);
  const double av = NUMERIC ? __shfl(x_av, src, kWave) : 0.0;
  if (lane >= t) len = 0;
  const uint32_t incl = wave_inclusive_scan(len);
  const uint32_t rel = incl - len;
  const uint32_t f = (uint32_t)__shfl((int)incl, t - 1, kWave);
  const uint32_t p = (uint32_t)lane;
  int lo = 0, hi = t - 1;
#pragma unroll
  for (int it = 0; it < 6; ++it) {
    const int mid = (lo + hi) >> 1;
    const uint32_t x = (uint32_t)__shfl((int)incl, mid, kWave);
    if (lo < hi) {
      if (x > p) hi = mid;
      else lo = mid + 1;
    }
  }
  const uint32_t excl_e = (uint32_t)__shfl((int)rel, lo, kWave);
  const uint32_t bs_e = (uint32_t)__shfl((int)bs, lo, kWave);
  const uint64_t jn_e = __shfl(jn, lo, kWave);
  const double av_e = NUMERIC ? __shfl(av, lo, kWave) : 0.0;
  if (p < f) {
    const uint32_t q = bs_e + (p - excl_e);
    valid = true;
    ent = lo;
    col = b_livs[q] - (NUMERIC ? np * (jn_e - kp * row) : jn_e);
    if (NUMERIC) v = av_e * b_vals[q];
  }
}

// One lane's share of a small row's product: at most one output entry.
struct RowOut {
  bool own = false;   // this lane holds an output entry
  uint32_t rank = 0;  // its position in the sorted row (numeric only)
  uint64_t col = 0;   // its column of B'
  double val = 0.0;   // its summed value (numeric only)
};

// The product of one small row of A' by one wave.  Returns the number of
// distinct columns (the row's output count); when NUMERIC, `o` receives this
// lane's output entry.
// The reduction of one small row's products (one per lane: `valid`, its A'
// entry `ent` in the row, column `col`, value `v`) into the row's output.
template <bool ACC, bool NUMERIC>
__device__ __forceinline__ uint32_t row_reduce(bool valid, int ent, uint64_t col, double v, int t, bool narrow, int w,
                                               int lane, const RowSmem& sm, RowOut& o) {
  if (ACC) {
    // sparse accumulator: an LDS hash table maps a column to a slot (32-bit
    // keys when the columns allow), and one FP64 accumulator per slot
    if (narrow) {
      sm.hash32[w][lane] = 0xFFFFFFFFu;
      sm.hash32[w][lane + kWave] = 0xFFFFFFFFu;
    } else {
      sm.hash[w][lane] = kEmpty;
      sm.hash[w][lane + kWave] = kEmpty;
    }
    if (NUMERIC) {
      sm.lanes[w][lane] = 0;
      sm.lanes[w][lane + kWave] = 0;
      if (lane == 0) sm.vals[w][kWave] = 0.0;
    }
    wave_lds_sync();
    uint32_t slot = valid ? hash_slot(col) : 0;
    bool isnew = false;
    if (valid) {
      if (narrow) {
        const uint32_t c32 = (uint32_t)col;
        for (int probe = 0; probe < 2 * kWave; ++probe) {
          const uint32_t prev = atomicCAS(&sm.hash32[w][slot], 0xFFFFFFFFu, c32);
          if (prev == 0xFFFFFFFFu) {
            isnew = true;
            break;
          }
          if (prev == c32) break;
          slot = (slot + 1) & (2 * kWave - 1);
        }
      } else {
        for (int probe = 0; probe < 2 * kWave; ++probe) {
          const uint64_t prev = atomicCAS((unsigned long long*)&sm.hash[w][slot], (unsigned long long)kEmpty,
                                          (unsigned long long)col);
          if (prev == kEmpty) {
            isnew = true;
            break;
          }
          if (prev == col) break;
          slot = (slot + 1) & (2 * kWave - 1);
        }
      }
    }
    const uint64_t newmask = __ballot(isnew);
    const uint32_t distinct = (uint32_t)__popcll(newmask);
    if (NUMERIC) {
      // Every product records its lane in its column's slot and stages its value
      // by lane.  The owner of a column (the lane that inserted it, i.e. its
      // first product) then sums the column's products in ascending lane order,
      // which is ascending A' entry (contracted index) order, starting from 0.0:
      // the values are read eight at a time (absent ones read the staged zero,
      // and adding +0.0 to a sum that started at +0.0 changes nothing), so the
      // reads of a group are independent and overlap.
      if (valid) atomicOr((unsigned long long*)&sm.lanes[w][slot], 1ull << lane);
      sm.vals[w][lane] = v;
      wave_lds_sync();
      double mine = 0.0;
      uint64_t m = isnew ? sm.lanes[w][slot] : 0ull;
      const int groups = (t + 7) >> 3;  // a column has at most one product per entry
      for (int g = 0; g < groups; ++g) {
        double x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int l = m ? __builtin_ctzll(m) : kWave;
          m &= m - 1;
          x[k] = sm.vals[w][l];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) mine += x[k];
      }
      uint32_t rank = 0;
      if (narrow && distinct <= 32) {
        // owners' columns compacted into slots [0, distinct) of a 32-slot list
        // padded with the largest column, then compared by every lane with
        // broadcast 16-byte LDS reads (no loop, no branches)
        if (isnew) sm.own[w][__popcll(newmask & lanemask_lt())] = (uint32_t)col;
        if (lane >= (int)distinct && lane < 32) sm.own[w][lane] = 0xFFFFFFFFu;
        wave_lds_sync();
        const uint32_t c32 = (uint32_t)col;
        const uint4* ol = reinterpret_cast<const uint4*>(sm.own[w]);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint4 x = ol[q];
          rank += (x.x < c32 ? 1u : 0u) + (x.y < c32 ? 1u : 0u) + (x.z < c32 ? 1u : 0u) + (x.w < c32 ? 1u : 0u);
        }
      } else {
        for (uint64_t mm = newmask; mm; mm &= mm - 1) {
          const int b = __builtin_ctzll(mm);
          const uint64_t cb = ((uint64_t)readlane_u32((uint32_t)(col >> 32), b) << 32) |
                              readlane_u32((uint32_t)col, b);
          rank += cb < col ? 1u : 0u;
        }
      }
      o.own = isnew;
      o.rank = rank;
      o.col = col;
      o.val = mine;
    }
    wave_lds_sync();
    return distinct;
  }
  // no accumulator: sort (column, product index), then each run head sums its
  // run (invalid lanes carry the largest key and sort last)
  uint64_t key = col;
  uint32_t idx = (uint32_t)lane;
  double val = v;
  wave_bitonic(key, idx, val);
  const uint64_t prev = __shfl_up(key, 1, kWave);
  const bool head = key != kEmpty && (lane == 0 || prev != key);
  const uint64_t hmask = __ballot(head);
  if (NUMERIC) {
    double acc = 0.0;
    bool active = head;
    if (head) acc += val;
    for (int s = 1; s < kWave; ++s) {
      const uint64_t ks = __shfl_down(key, s, kWave);
      const double vs = __shfl_down(val, s, kWave);
      if (active) {
        if (lane + s < kWave && ks == key) acc += vs;
        else active = false;
      }
      if (!__any(active)) break;
    }
    o.own = head;
    o.rank = (uint32_t)__popcll(hmask & lanemask_lt());
    o.col = key;
    o.val = acc;
  }
  return (uint32_t)__popcll(hmask);
}

}  // namespace
}  // namespace lco
