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

// Pointer arrays (row pointers, row starts, bucket indexes) are filled from
// the entries: entry e owns the pointer slots [lo, hi) of the rows (or
// buckets) from just after the previous entry's row up to its own, and writes
// e into them.  A lane fills its own
// slots when there are at most kFillLane of them; longer runs (clustered rows
// leave long runs of empty rows) are written by the whole wave, so no lane
// writes millions of slots alone.  Every lane of the wave must call this.
constexpr uint64_t kFillLane = 256;
__device__ __forceinline__ void fill_slots(uint32_t* __restrict__ out, bool active, uint64_t lo, uint64_t hi,
                                           uint32_t v) {
  const bool wide = active && hi - lo > kFillLane;
  if (active && !wide)
    for (uint64_t r = lo; r < hi; ++r) out[r] = v;
  const int lane = lane_id();
  for (uint64_t m = __ballot(wide); m; m &= m - 1) {
    const int src = __builtin_ctzll(m);
    const uint64_t a = __shfl(lo, src, kWave), b = __shfl(hi, src, kWave);
    const uint32_t x = __shfl(v, src, kWave);
    for (uint64_t r = a + lane; r < b; r += kWave) out[r] = x;
  }
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

// Hash slots per wave, two per lane (at most 64 columns per row: at most half
// full).
constexpr int kHashBits = 7;
constexpr int kHashSlots = 1 << kHashBits;
static_assert(kHashSlots == 2 * kWave, "two hash slots per lane");
__device__ __forceinline__ uint32_t hash_slot(uint64_t c) {
  return (uint32_t)((c * 0x9E3779B97F4A7C15ull) >> (64 - kHashBits));
}
__device__ __forceinline__ uint32_t hash_slot32(uint32_t c) {
  return (c * 0x9E3779B1u) >> (32 - kHashBits);
}

// Per-row shape codes of the one-wave kernel.
constexpr uint8_t kShapeSearch = 7;    // at most 64 products, located by search
constexpr uint8_t kShapeTiny = 8;      // at most kTinyEntries entries and kTinyProducts products: one lane per row
constexpr uint8_t kShapeCopy = 9;      // one entry (more than kTinyProducts products): the row is a scaled B' row
constexpr uint8_t kShapeLong = 0xFE;   // more than 64 products or entries (not one entry): the long-row path
constexpr uint8_t kShapeSkip = 0xFF;   // no products
constexpr int kTinyEntries = 4;
constexpr int kTinyProducts = 16;
// Rows with at most 64 products and 64 entries run one wave per row.  When the
// row's entries times W (the next power of two at least its longest B' row) fit
// the 64 lanes, lane = entry * W + position ("entry-major"): each lane knows its
// product without any search.  The shape code is log2 W for those rows.
__device__ __forceinline__ bool small_row(uint64_t f, uint32_t t) {
  return f <= (uint64_t)kWave && t <= (uint32_t)kWave;
}

// LDS of one wave of the one-wave-per-row kernels.  The hash table has
// kHashSlots slots.
// Numeric: a row with at most kTabEntries entries and 32-bit columns sums
// through the table tab[entry][owner number], which is all +0.0 between rows;
// other accumulator rows use the lane masks and staged values that share its
// space and clear them again when done.
constexpr int kTabEntries = 7;
template <bool NUMERIC>
struct RowLds;
template <>
struct alignas(16) RowLds<false> {
  union {
    uint64_t hash[kHashSlots];    // columns
    uint32_t hash32[kHashSlots];  // 32-bit columns
  };
};
template <>
struct alignas(16) RowLds<true> {
  union {
    uint64_t hash[kHashSlots];    // column (with the owner lane above 32-bit columns in table rows)
    uint32_t hash32[kHashSlots];  // (32-bit keys: the symbolic pass only)
  };
  uint32_t own[kWave];  // owners' columns (rank by broadcast compares)
  union {
    double tab[kTabEntries][kWave + 1];  // per A' entry, per owner number: the product's value (rows padded by one
                                         // value, so that one owner's cells fall in different banks)
    struct {
      uint64_t lanes[kHashSlots];  // per hash slot: the lanes whose product has that column
      double vals[kWave + 8];      // each lane's product value, and a zero at index kWave
    } mask;
  };
};
static_assert(offsetof(RowLds<true>, own) % 16 == 0, "RowLds alignment");

// Clears a wave's table (once, before its first row).
__device__ __forceinline__ void tab_clear(RowLds<true>& L, int lane) {
#pragma unroll
  for (int e = 0; e < kTabEntries; ++e) {
    L.tab[e][lane] = 0.0;
    if (lane == 0) L.tab[e][kWave] = 0.0;
  }
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int l) {
  return ((uint64_t)readlane_u32((uint32_t)(x >> 32), l) << 32) | readlane_u32((uint32_t)x, l);
}

// Locates the products of one small row in the entry window (lane l holds
// entry w0 + l: its product count, B' row start, value, and j * n', the LIV of
// its B' row's first position, j = its contracted index).
// Each lane ends up with at most one product: its A' entry `ent` within the
// row, its B' position `q`, the amount `off` (= j * n') its B' LIV exceeds its
// column by, and (numeric) the A' value `av` that scales it.  The caller loads
// B' at q.
template <bool NUMERIC>
__device__ __forceinline__ void window_locate(uint32_t e0, int t, uint8_t sh, int lane, int64_t w0, uint32_t x_len,
                                              uint32_t x_bs, uint64_t x_jn, double x_av, bool& valid, int& ent,
                                              uint32_t& q, uint64_t& off, double& av) {
  valid = false;
  ent = 0;
  q = 0;
  off = 0;
  av = 0.0;
  const int first = (int)((int64_t)e0 - w0);  // window lane of the row's first entry
  if (sh != kShapeSearch) {
    // entry-major lanes: lane = entry * W + position
    const int e = lane >> sh, k = lane & ((1 << sh) - 1);
    const int src = (first + e) & (kWave - 1);
    const uint32_t len = (uint32_t)__shfl((int)x_len, src, kWave);
    const uint32_t bs = (uint32_t)__shfl((int)x_bs, src, kWave);
    const uint64_t jn = __shfl(x_jn, src, kWave);
    if (NUMERIC) av = __shfl(x_av, src, kWave);
    if (e < t && (uint32_t)k < len) {
      valid = true;
      ent = e;
      q = bs + (uint32_t)k;
      off = jn;
    }
    return;
  }
  // general small row: lane p takes product p, found by a binary search over the
  // entries' inclusive product counts
  const int src = (first + lane) & (kWave - 1);
  uint32_t len = (uint32_t)__shfl((int)x_len, src, kWave);
  const uint32_t bs = (uint32_t)__shfl((int)x_bs, src, kWave);
  const uint64_t jn = __shfl(x_jn, src, kWave);
  const double a = NUMERIC ? __shfl(x_av, src, kWave) : 0.0;
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
  if (NUMERIC) av = __shfl(a, lo, kWave);
  if (p < f) {
    valid = true;
    ent = lo;
    q = bs_e + (p - excl_e);
    off = jn_e;
  }
}

// One lane's product of a small row: where it is, and its B' entry once loaded.
template <bool NUMERIC>
struct RowProduct {
  bool valid = false;
  int ent = 0;
  uint64_t off = 0;
  double av = 0.0;
  uint64_t liv = 0;    // B' LIV (in flight until first use)
  double bval = 0.0;   // B' value (numeric)

  __device__ __forceinline__ void load(const uint64_t* __restrict__ b_livs, const double* __restrict__ b_vals,
                                       uint32_t q) {
    if (valid) {
      liv = b_livs[q];
      if (NUMERIC) bval = b_vals[q];
    }
  }
  // the product's column (kEmpty when this lane holds none) and value
  __device__ __forceinline__ uint64_t col() const { return valid ? liv - off : kEmpty; }
  __device__ __forceinline__ double val() const { return (NUMERIC && valid) ? av * bval : 0.0; }
};

// Locates a small row's products in the window and issues their B' loads.
template <bool NUMERIC>
__device__ __forceinline__ void window_products(const uint64_t* __restrict__ b_livs, const double* __restrict__ b_vals,
                                                uint32_t e0, int t, uint8_t sh, int lane, int64_t w0, uint32_t x_len,
                                                uint32_t x_bs, uint64_t x_jn, double x_av, RowProduct<NUMERIC>& pr) {
  uint32_t q;
  window_locate<NUMERIC>(e0, t, sh, lane, w0, x_len, x_bs, x_jn, x_av, pr.valid, pr.ent, q, pr.off, pr.av);
  pr.load(b_livs, b_vals, q);
}

// One lane's share of a small row's product: at most one output entry.
struct RowOut {
  bool own = false;   // this lane holds an output entry
  uint32_t rank = 0;  // its position in the sorted row (numeric only)
  uint64_t col = 0;   // its column of B'
  double val = 0.0;   // its summed value (numeric only)
};

// The reduction of one small row's products by one wave (one product per
// lane: `valid`, its A' entry `ent` in the row, column `col`, value `v`; the
// row has t entries).  Returns the number of distinct columns (the row's output
// count); when NUMERIC, `o` receives this lane's output entry.
template <bool ACC, bool NUMERIC>
__device__ __forceinline__ uint32_t row_reduce(bool valid, int ent, uint64_t col, double v, int t, bool narrow,
                                               int lane, RowLds<NUMERIC>& L, RowOut& o) {
  if (ACC) {
    // Sparse accumulator: an LDS hash table maps a column to a slot, and the
    // lane that inserts a column owns it.  Numeric rows of at most kTabEntries
    // entries with 32-bit columns ("table rows") store the owner lane beside
    // the column, so that every product learns its owner.
    const bool table = NUMERIC && narrow && t <= kTabEntries;
    const bool key32 = !NUMERIC && narrow;
    if constexpr (!NUMERIC) {
      if (key32) {
        L.hash32[lane] = 0xFFFFFFFFu;
        L.hash32[lane + kWave] = 0xFFFFFFFFu;
      } else {
        L.hash[lane] = kEmpty;
        L.hash[lane + kWave] = kEmpty;
      }
    } else {
      L.hash[lane] = kEmpty;
      L.hash[lane + kWave] = kEmpty;
      if (!table) {
        L.mask.lanes[lane] = 0;
        L.mask.lanes[lane + kWave] = 0;
        if (lane == 0) L.mask.vals[kWave] = 0.0;
      }
    }
    wave_lds_sync();
    uint32_t slot = valid ? (narrow ? hash_slot32((uint32_t)col) : hash_slot(col)) : 0;
    uint32_t owner = 0;  // the lane that inserted the column (table rows)
    bool isnew = false;
    if constexpr (NUMERIC) {
      // Probe until the slot is empty (this lane inserts the column) or holds
      // the column; at most 64 columns in 128 slots, so a free slot always
      // exists and every probe sequence ends.  Only lanes still probing take
      // part in a probe.  Lanes with one column probe the same slots in
      // lockstep, so exactly one of them inserts it.
      if (valid) {
        uint64_t p;
        if (table) {
          // key: the owner lane above the 32-bit column (never kEmpty)
          const uint32_t c32 = (uint32_t)col;
          const uint64_t key = ((uint64_t)lane << 32) | c32;
          while (true) {
            p = atomicCAS((unsigned long long*)&L.hash[slot], (unsigned long long)kEmpty, (unsigned long long)key);
            if (p == kEmpty || (uint32_t)p == c32) break;
            slot = (slot + 1) & (kHashSlots - 1);
          }
        } else {
          while (true) {
            p = atomicCAS((unsigned long long*)&L.hash[slot], (unsigned long long)kEmpty, (unsigned long long)col);
            if (p == kEmpty || p == col) break;
            slot = (slot + 1) & (kHashSlots - 1);
          }
        }
        isnew = p == kEmpty;
        owner = isnew ? (uint32_t)lane : (uint32_t)(p >> 32);
      }
    } else {
      // The same probing as the numeric pass, with only the column stored
      // (32-bit columns in 32-bit slots).
      if (valid) {
        if (key32) {
          const uint32_t c32 = (uint32_t)col;
          while (true) {
            const uint32_t p = atomicCAS(&L.hash32[slot], 0xFFFFFFFFu, c32);
            if (p == 0xFFFFFFFFu) {
              isnew = true;
              break;
            }
            if (p == c32) break;
            slot = (slot + 1) & (kHashSlots - 1);
          }
        } else {
          while (true) {
            const uint64_t p =
                atomicCAS((unsigned long long*)&L.hash[slot], (unsigned long long)kEmpty, (unsigned long long)col);
            if (p == kEmpty) {
              isnew = true;
              break;
            }
            if (p == col) break;
            slot = (slot + 1) & (kHashSlots - 1);
          }
        }
      }
    }
    const uint64_t newmask = __ballot(isnew);
    const uint32_t distinct = (uint32_t)__popcll(newmask);
    if constexpr (NUMERIC) {
      if (table) {
        // Owners are numbered d = 0, 1, ... in lane order, and output d is
        // computed by lane d (and, when there are at most 32, also by lane
        // d + 32, which shares the rank comparisons).  Each product stores its
        // value at (its entry, its owner's d); owner d stores its column at d.
        const uint32_t d = (uint32_t)__popcll(newmask & ((1ull << owner) - 1ull));
        if (valid) L.tab[ent][d] = v;
        if (isnew) L.own[d] = (uint32_t)col;
        if (lane >= (int)distinct) L.own[lane] = 0xFFFFFFFFu;  // padding: larger than any column
        wave_lds_sync();
        const bool split = distinct <= 32;
        const int me = split ? (lane & 31) : lane;
        const uint32_t c32 = L.own[me];
        // the sum runs over the entries in order, i.e. ascending contracted
        // index, from 0.0; entries without this column hold +0.0, which cannot
        // change a sum that started at +0.0
        double x[kTabEntries];
#pragma unroll
        for (int e = 0; e < kTabEntries; ++e) x[e] = L.tab[e][me];
        double mine = 0.0;
#pragma unroll
        for (int e = 0; e < kTabEntries; ++e) mine += x[e];
        // rank: the number of smaller columns, by broadcast 16-byte LDS reads
        // of the column list (each half of the wave takes 16 of at most 32)
        const uint4* ol = reinterpret_cast<const uint4*>(L.own);
        uint32_t rank = 0;
        if (split) {
          // all four reads at once; columns past the distinct ones are padding,
          // which is never smaller
          uint4 y[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) y[q] = ol[(lane >> 5) * 4 + q];
#pragma unroll
          for (int q = 0; q < 4; ++q)
            rank += (y[q].x < c32 ? 1u : 0u) + (y[q].y < c32 ? 1u : 0u) + (y[q].z < c32 ? 1u : 0u) +
                    (y[q].w < c32 ? 1u : 0u);
          rank += (uint32_t)__shfl_xor((int)rank, 32, kWave);
        } else {
          const uint32_t nq = (distinct + 3) >> 2;
#pragma unroll
          for (uint32_t q = 0; q < kWave / 4; ++q) {
            if (q < nq) {
              const uint4 y = ol[q];
              rank += (y.x < c32 ? 1u : 0u) + (y.y < c32 ? 1u : 0u) + (y.z < c32 ? 1u : 0u) + (y.w < c32 ? 1u : 0u);
            }
          }
        }
        wave_lds_sync();
        if (valid) L.tab[ent][d] = 0.0;  // every product clears its cell for the next row
        o.own = lane < (int)distinct;
        o.rank = rank;
        o.col = c32;
        o.val = mine;
        return distinct;
      }
      // Every product records its lane in its column's slot and stages its
      // value by lane.  The owner (the inserting lane) then sums the column's
      // products in ascending lane order, which is ascending A' entry
      // (contracted index) order, starting from 0.0: the values are read eight
      // at a time (absent ones read the staged zero, and adding +0.0 to a sum
      // that started at +0.0 changes nothing), so the reads of a group are
      // independent.
      if (valid) atomicOr((unsigned long long*)&L.mask.lanes[slot], 1ull << lane);
      L.mask.vals[lane] = v;
      wave_lds_sync();
      double mine = 0.0;
      uint64_t m = isnew ? L.mask.lanes[slot] : 0ull;
      const int groups = (t + 7) >> 3;  // a column has at most one product per entry
      for (int g = 0; g < groups; ++g) {
        double x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int l = m ? __builtin_ctzll(m) : kWave;
          m &= m - 1;
          x[k] = L.mask.vals[l];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) mine += x[k];
      }
      uint32_t rank = 0;
      if (narrow && distinct <= 32) {
        // owners' columns compacted into slots [0, distinct) of a 32-slot list
        // padded with the largest column, then compared by every lane with
        // broadcast 16-byte LDS reads
        if (isnew) L.own[__popcll(newmask & lanemask_lt())] = (uint32_t)col;
        if (lane >= (int)distinct && lane < 32) L.own[lane] = 0xFFFFFFFFu;
        wave_lds_sync();
        const uint32_t c32 = (uint32_t)col;
        const uint4* ol = reinterpret_cast<const uint4*>(L.own);
        const uint32_t nq = (distinct + 3) >> 2;
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) {
          if (q < nq) {
            const uint4 y = ol[q];
            rank += (y.x < c32 ? 1u : 0u) + (y.y < c32 ? 1u : 0u) + (y.z < c32 ? 1u : 0u) + (y.w < c32 ? 1u : 0u);
          }
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
      wave_lds_sync();
      // the table's space is all +0.0 again
      L.mask.lanes[lane] = 0;
      L.mask.lanes[lane + kWave] = 0;
      L.mask.vals[lane] = 0.0;
      return distinct;
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
