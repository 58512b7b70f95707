// Persistent batched contraction: every phase of every instance of a batch in
// one launch of a persistent grid, with no host synchronisation between phases.
//
// The instances are the row-wise products of the batch (singly compressed B',
// rows of A' listed densely, every row of A' with at most 64 products and 64
// entries), i.e. the three steps of Section 5.2 applied per instance with the
// row engine of Sections 5.2.2 and 5.2.4.  The work of an instance is cut into
// items of six phases:
//   0  row pointers of B' (tiles of B' entries),
//   1  row starts of A' and each A' entry's product count and B' row start
//      (tiles of A' entries),
//   2  row shapes and the symbolic count of every row (groups of 64-row chunks),
//   3  each instance's scan of its chunk counts (one item per instance),
//   4  the scan over instances: every instance's place in the output pool (one item),
//   5  the numeric product, written to the pool (groups of 64-row chunks).
// Items are taken from 64 queues, eight per XCD: the eight queues of XCD x
// share the x-th eighth of every phase's items in instance order, interleaved
// (queue j takes every eighth item from the j-th on), so the waves of one XCD
// work on neighbouring chunks of the same instances (rows that gather the same
// rows of B' share that XCD's L2) while the queue heads, one atomic per item
// taken, are spread over 64 addresses.  A wave takes items of phase p from a
// queue of its own XCD, then from any queue with items left, and moves on to
// phase p + 1 only when every queue has handed out all of phase p; it then
// waits until every item of phase p is complete.  A wave waits only for items that running waves have
// already taken, so the grid never deadlocks, whatever part of it is resident
// and whatever else runs on the device; every wait is also bounded and reports
// through the device error word when it gives up.
//
// Rows are computed by the same device code as the per-call engine
// (row_core.h), so each result is bit-identical to the per-call result.
#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <mutex>

#include "row_core.h"

namespace lco {

namespace {

constexpr int kPhases = 6;
constexpr int64_t kSetupTile = 8192;  // entries per item of phases 0 and 1
constexpr int kCtlStride = 32;         // control words sit 256 bytes apart
// Work queues: kSubQueues per XCD, interleaved over the XCD's range of a
// phase's items (so that the queue heads, one atomic per item taken, are
// spread over many addresses).
constexpr uint32_t kSubQueues = 8;
constexpr uint32_t kQueues = kXcds * kSubQueues;
static_assert(kQueues == (uint32_t)kWave, "one queue per lane in the search for leftover items");
// control block: queue heads [phase][queue], done counts [phase], results
constexpr int kCtlDone = kPhases * (int)kQueues;
constexpr int kCtlRes = kCtlDone + kPhases;
constexpr int kCtlWords = (kCtlRes + 1) * kCtlStride;
constexpr uint64_t kSpinLimit = 1ull << 24;  // polls of a completion count before giving up

struct PInst {
  const uint64_t* a_livs;
  const double* a_vals;
  const uint64_t* b_livs;
  const double* b_vals;
  int64_t nnz_a, nnz_b;
  uint64_t mp, kp, np;
  FastDiv kdiv, ndiv;
  int64_t eoff;  // first slot of this instance in the per-entry arrays
  int64_t koff;  // first of its k' + 1 row pointers of B'
  int64_t roff;  // first of its m' + 1 row slots (row starts, shapes, counts)
  int64_t coff;  // first of its chunks
  uint32_t nchunks;
  uint32_t group;  // chunks per item in phases 2 and 5
  uint32_t acc;    // 1: accumulator (CSR/CSC), 0: none (CSRNA/CSCNA)
  uint32_t pad;
};

struct PArgs {
  const PInst* inst;
  int count;
  int first, last;     // phases run by this launch
  const uint32_t* ipre;  // items before each instance in phases 0, 1, 2 and 5 (4 x (count + 1))
  uint64_t n[kPhases];   // items per phase in this launch
  uint32_t* bptr;
  uint32_t* row_start;
  uint32_t* elen;
  uint32_t* bstart;
  uint8_t* shape;
  uint32_t* cnt;
  uint32_t* chunk_sum;
  uint64_t* chunk_off;
  uint64_t* total;
  uint64_t* base;
  uint32_t* fallback;
  uint64_t* ctl;
  uint32_t* err;
  uint64_t* out_livs;
  double* out_vals;
  uint64_t capacity;  // entries the output pool holds
};

__device__ __forceinline__ uint64_t* ctl_head(uint64_t* ctl, int p, uint32_t q) {
  return ctl + (p * (int)kQueues + (int)q) * kCtlStride;
}
__device__ __forceinline__ uint64_t* ctl_done(uint64_t* ctl, int p) { return ctl + (kCtlDone + p) * kCtlStride; }
__device__ __forceinline__ uint64_t* ctl_res(uint64_t* ctl) { return ctl + kCtlRes * kCtlStride; }

__device__ __forceinline__ uint64_t shfl0_u64(uint64_t x) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(x >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// An instance descriptor in scalar registers: every word is read by the wave
// and made uniform, so that the fields need no vector registers.
__device__ __forceinline__ PInst load_inst(const PInst* __restrict__ inst, int i) {
  static_assert(sizeof(PInst) % 4 == 0, "PInst is read in 32-bit words");
  const uint32_t* src = reinterpret_cast<const uint32_t*>(inst + i);
  PInst x;
  uint32_t* dst = reinterpret_cast<uint32_t*>(&x);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(PInst) / 4); ++k) dst[k] = (uint32_t)__builtin_amdgcn_readfirstlane((int)src[k]);
  return x;
}

// Items of queue q among a phase's n items: lo, lo + kSubQueues, ... (len of them).
__device__ __forceinline__ void queue_range(uint64_t n, uint32_t q, uint64_t& lo, uint64_t& len) {
  const uint32_t x = q / kSubQueues, j = q % kSubQueues;
  const uint64_t xlo = n * x / kXcds, xhi = n * (x + 1) / kXcds;
  lo = xlo + j;
  len = xhi > lo ? (xhi - lo + kSubQueues - 1) / kSubQueues : 0;
}

// Instance owning item k of a phase: the largest i < count with pre[i] <= k
// (pre ascending, pre[0] = 0, k < pre[count]); a 64-way search per round.
__device__ __forceinline__ int find_owner(const uint32_t* __restrict__ pre, int count, uint32_t k) {
  const int lane = lane_id();
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int step = (hi - lo + kWave - 1) / kWave;
    const int pos = lo + lane * step;
    const bool le = pos < hi && pre[pos] <= k;
    const uint64_t m = __ballot(le);  // lanes 0.. are true, lane 0 always
    const int last = 63 - __builtin_clzll(m);
    lo += last * step;
    hi = lo + step < hi ? lo + step : hi;
  }
  return lo;
}

// ---------------------------------------------------------------- phases 0 and 1

// Entries per lane and step of the setup phases: every load of a step is
// issued before its stores, so a wave keeps several loads in flight.
constexpr int kSetupUnroll = 4;

// Row pointers of B' from B' entries [e_lo, e_hi) (entry nnz_b is the terminal).
__device__ __forceinline__ void p_bptr(const PArgs& g, const PInst& x, int64_t e_lo, int64_t e_hi, int lane) {
  const int64_t n = x.nnz_b;
  uint32_t* bp = g.bptr + x.koff;
  const uint64_t* __restrict__ bl = x.b_livs;
  for (int64_t e0 = e_lo; e0 < e_hi; e0 += kSetupUnroll * kWave) {
    uint64_t lo[kSetupUnroll], hi[kSetupUnroll];
    bool valid[kSetupUnroll];
#pragma unroll
    for (int u = 0; u < kSetupUnroll; ++u) {
      const int64_t e = e0 + u * kWave + lane;
      valid[u] = e < e_hi;
      lo[u] = 0;
      hi[u] = 0;
      if (valid[u]) {
        lo[u] = e == 0 ? 0 : fd_div(x.ndiv, bl[e - 1]) + 1;
        hi[u] = (e == n ? x.kp : fd_div(x.ndiv, bl[e])) + 1;
      }
    }
#pragma unroll
    for (int u = 0; u < kSetupUnroll; ++u) fill_slots(bp, valid[u], lo[u], hi[u], (uint32_t)(e0 + u * kWave + lane));
  }
}

// Row starts of A' (all m' rows, empty ones included) and each A' entry's B'
// row start and length, from A' entries [e_lo, e_hi) (entry nnz_a is the terminal).
__device__ __forceinline__ void p_rows(const PArgs& g, const PInst& x, int64_t e_lo, int64_t e_hi, int lane) {
  const int64_t n = x.nnz_a;
  const uint32_t* __restrict__ bp = g.bptr + x.koff;
  const uint64_t* __restrict__ al = x.a_livs;
  uint32_t* rs = g.row_start + x.roff;
  for (int64_t e0 = e_lo; e0 < e_hi; e0 += kSetupUnroll * kWave) {
    uint64_t lo[kSetupUnroll], hi[kSetupUnroll], j[kSetupUnroll];
    uint32_t st[kSetupUnroll], en[kSetupUnroll];
    bool valid[kSetupUnroll];
#pragma unroll
    for (int u = 0; u < kSetupUnroll; ++u) {
      const int64_t e = e0 + u * kWave + lane;
      valid[u] = e < e_hi;
      lo[u] = 0;
      hi[u] = x.mp;
      j[u] = 0;
      if (valid[u]) {
        if (e < n) hi[u] = fd_divmod(x.kdiv, al[e], j[u]);
        lo[u] = e == 0 ? 0 : fd_div(x.kdiv, al[e - 1]) + 1;
      }
    }
#pragma unroll
    for (int u = 0; u < kSetupUnroll; ++u) {
      const int64_t e = e0 + u * kWave + lane;
      st[u] = 0;
      en[u] = 0;
      if (valid[u] && e < n) {
        st[u] = bp[j[u]];
        en[u] = bp[j[u] + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < kSetupUnroll; ++u) {
      const int64_t e = e0 + u * kWave + lane;
      if (valid[u] && e < n) {
        g.elen[x.eoff + e] = en[u] - st[u];
        g.bstart[x.eoff + e] = st[u];
      }
      fill_slots(rs, valid[u], lo[u], valid[u] ? hi[u] + 1 : 0, (uint32_t)e);
    }
  }
}

// ---------------------------------------------------------------- phases 2 and 5: one chunk of 64 rows

union PLds {
  RowLds<true> num;
  RowLds<false> sym;
};

template <bool ACC, bool NUMERIC, bool NARROW>
__device__ __forceinline__ void p_chunk(const PArgs& g, const PInst& x, int inst, uint64_t c, RowLds<NUMERIC>& L,
                                        int lane) {
  const uint64_t r0 = c * kWave;
  const int rows = (int)(x.mp - r0 < (uint64_t)kWave ? x.mp - r0 : (uint64_t)kWave);
  const uint32_t* rs = g.row_start + x.roff;
  const uint32_t* elen = g.elen + x.eoff;
  const uint32_t* bst = g.bstart + x.eoff;
  uint32_t m_s0 = 0, m_s1 = 0, m_sh = kShapeSkip;
  uint64_t m_off = 0;
  if (lane < rows) {
    m_s0 = rs[r0 + lane];
    m_s1 = rs[r0 + lane + 1];
  }
  if (NUMERIC) {
    uint32_t m_cnt = 0;
    if (lane < rows) {
      m_sh = g.shape[x.roff + r0 + lane];
      m_cnt = g.cnt[x.roff + r0 + lane];
    }
    const uint32_t incl = wave_inclusive_scan(m_cnt);
    m_off = g.base[inst] + g.chunk_off[x.coff + c] + (incl - m_cnt);
  } else if (lane < rows) {
    // the row's shape; a row the one-wave engine cannot take sends the
    // instance to the per-call path
    const uint32_t ne = m_s1 - m_s0;
    uint8_t sh = kShapeSkip;
    bool out = ne > (uint32_t)kWave;
    if (!out) {
      uint64_t f = 0, mx = 0;
      for (uint32_t e0 = m_s0; e0 < m_s1; e0 += 8) {
        uint32_t l[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) l[k] = e0 + k < m_s1 ? elen[e0 + k] : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          f += l[k];
          mx = l[k] > mx ? l[k] : mx;
        }
      }
      if (f > 0 && small_row(f, ne)) {
        uint32_t lw = 0;
        while ((1ull << lw) < mx) ++lw;
        sh = ((uint64_t)ne << lw) <= (uint64_t)kWave ? (uint8_t)lw : kShapeSearch;
      } else if (f > 0) {
        out = true;
      }
    }
    if (out) atomicOr(&g.fallback[inst], 1u);
    g.shape[x.roff + r0 + lane] = sh;
    m_sh = sh;
  }
  uint32_t my_cnt = 0;
  // entry window [w0, w0 + 64) (none before the first row; entry indexes are
  // 32-bit, so the tests are scalar compares)
  bool have = false;
  uint32_t w0 = 0;
  uint32_t x_len = 0, x_bs = 0;
  uint64_t x_jn = 0;
  double x_av = 0.0;
  uint64_t todo = __ballot(lane < rows && m_sh <= kShapeSearch);
  RowProduct<NUMERIC> next;
  int t_next = 0;
  auto stage = [&](int i) {
    const uint8_t sh = (uint8_t)readlane_u32(m_sh, i);
    const uint32_t e0 = readlane_u32(m_s0, i), e1 = readlane_u32(m_s1, i);
    t_next = (int)(e1 - e0);  // at most 64 for the rows of this engine
    if (!have || e0 - w0 > (uint32_t)(kWave - t_next)) {
      have = true;
      w0 = e0;
      const int64_t e = (int64_t)w0 + lane;
      if (e < x.nnz_a) {
        x_len = elen[e];
        x_bs = bst[e];
        uint64_t j;
        fd_divmod(x.kdiv, x.a_livs[e], j);
        x_jn = j * x.np;
        if (NUMERIC) x_av = x.a_vals[e];
      }
    }
    window_products<NUMERIC>(x.b_livs, x.b_vals, e0, t_next, sh, lane, (int64_t)w0, x_len, x_bs, x_jn, x_av,
                             next);
  };
  if (todo) stage(__builtin_ctzll(todo));
  const bool narrow = NARROW || x.np < (1ull << 32);
  while (todo) {
    const int i = __builtin_ctzll(todo);
    todo &= todo - 1;
    const bool valid = next.valid;
    const int ent = next.ent;
    const uint64_t col = next.col();
    const double v = next.val();
    const int t = t_next;
    if (todo) stage(__builtin_ctzll(todo));
    RowOut o;
    const uint32_t d = row_reduce<ACC, NUMERIC>(valid, ent, col, v, t, narrow, lane, L, o);
    if (!NUMERIC) {
      if (lane == i) my_cnt = d;
    } else if (o.own) {
      // scalar row base, 32-bit lane offset (the rank is below 64)
      const uint64_t r_off = readlane_u64(m_off, i);
      const uint32_t boff = o.rank * 8u;
      *reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(g.out_livs + r_off) + boff) =
          o.col + x.np * (r0 + (uint64_t)i);
      *reinterpret_cast<double*>(reinterpret_cast<char*>(g.out_vals + r_off) + boff) = o.val;
    }
  }
  if (!NUMERIC) {
    if (lane < rows) g.cnt[x.roff + r0 + lane] = my_cnt;
    const uint32_t sum = wave_reduce_sum(my_cnt);
    if (lane == 0) g.chunk_sum[x.coff + c] = sum;
  }
}

// ---------------------------------------------------------------- phases 3 and 4: scans by one wave

// Exclusive scan of n 32-bit counts into 64-bit offsets; returns the total.
// Each lane takes 16 consecutive counts per step (independent loads), so a
// step covers 1024 counts with one wave-wide scan.
constexpr int kScanPerLane = 16;
__device__ __forceinline__ uint64_t wave_scan_counts(const uint32_t* __restrict__ in, uint64_t* __restrict__ out,
                                                     uint64_t n, int lane) {
  uint64_t run = 0;
  for (uint64_t b = 0; b < n; b += (uint64_t)kScanPerLane * kWave) {
    const uint64_t first = b + (uint64_t)lane * kScanPerLane;
    uint32_t v[kScanPerLane];
#pragma unroll
    for (int k = 0; k < kScanPerLane; ++k) v[k] = first + k < n ? in[first + k] : 0u;
    uint64_t mine = 0;
#pragma unroll
    for (int k = 0; k < kScanPerLane; ++k) mine += v[k];
    const uint64_t incl = wave_inclusive_scan(mine);
    uint64_t at = run + incl - mine;
#pragma unroll
    for (int k = 0; k < kScanPerLane; ++k) {
      if (first + k < n) out[first + k] = at;
      at += v[k];
    }
    run += lane_value(incl, kWave - 1);
  }
  return run;
}

// ---------------------------------------------------------------- the persistent grid

// MODE: bit 0 compiles phases 0-4 (setup, symbolic, scans), bit 1 phase 5 (numeric).
constexpr int kModeSize = 1, kModeNumeric = 2, kModeAll = 3;
// BRANCH: the numeric row code compiled in: the accumulator only, the
// sort-based branch only, or both (chosen per instance).  Each is compiled
// alone where the batch allows it, since the code of both together needs more
// registers.  The symbolic count is the same for both branches, so phase 2
// always counts with the accumulator.
constexpr int kBranchNa = 0, kBranchAcc = 1, kBranchBoth = 2;

template <bool NARROW, int MODE, int BRANCH>
__device__ __forceinline__ void run_item(const PArgs& g, int p, uint64_t k, PLds& L, int lane) {
  if constexpr ((MODE & kModeSize) == 0) {
    if (p != 5) return;
  }
  if (p == 4) {
    // every instance's place in the pool, in instance order (16 instances per lane per step)
    uint64_t run = 0;
    uint32_t anyfb = 0;
    for (int b = 0; b < g.count; b += kScanPerLane * kWave) {
      const int first = b + lane * kScanPerLane;
      uint64_t v[kScanPerLane];
      uint64_t mine = 0;
#pragma unroll
      for (int k = 0; k < kScanPerLane; ++k) {
        v[k] = first + k < g.count ? g.total[first + k] : 0;
        anyfb |= (first + k < g.count && g.fallback[first + k]) ? 1u : 0u;
        mine += v[k];
      }
      const uint64_t incl = wave_inclusive_scan(mine);
      uint64_t at = run + incl - mine;
#pragma unroll
      for (int k = 0; k < kScanPerLane; ++k) {
        if (first + k < g.count) g.base[first + k] = at;
        at += v[k];
      }
      run += lane_value(incl, kWave - 1);
    }
    anyfb = __ballot(anyfb != 0) ? 1u : 0u;
    if (lane == 0) {
      uint64_t* res = ctl_res(g.ctl);
      res[0] = run;
      res[1] = anyfb;
      res[2] = run > g.capacity ? 1u : 0u;
    }
    return;
  }
  if (p == 3) {
    const int i = (int)k;
    const PInst x = load_inst(g.inst, i);
    const uint64_t t = wave_scan_counts(g.chunk_sum + x.coff, g.chunk_off + x.coff, x.nchunks, lane);
    if (lane == 0) g.total[i] = g.fallback[i] ? 0 : t;
    return;
  }
  const int pi = p == 5 ? 3 : p;
  const uint32_t* pre = g.ipre + (size_t)pi * (g.count + 1);
  const int i = __builtin_amdgcn_readfirstlane(find_owner(pre, g.count, (uint32_t)k));
  const PInst x = load_inst(g.inst, i);
  const uint64_t t = k - pre[i];
  if (p == 0) {
    const int64_t lo = (int64_t)t * kSetupTile, hi = lo + kSetupTile < x.nnz_b + 1 ? lo + kSetupTile : x.nnz_b + 1;
    p_bptr(g, x, lo, hi, lane);
    return;
  }
  if (p == 1) {
    const int64_t lo = (int64_t)t * kSetupTile, hi = lo + kSetupTile < x.nnz_a + 1 ? lo + kSetupTile : x.nnz_a + 1;
    p_rows(g, x, lo, hi, lane);
    return;
  }
  const uint64_t c0 = t * x.group, c1 = c0 + x.group < x.nchunks ? c0 + x.group : (uint64_t)x.nchunks;
  if constexpr ((MODE & kModeNumeric) == 0) p = 2;
  if (p == 2) {
    for (uint64_t c = c0; c < c1; ++c) p_chunk<true, false, NARROW>(g, x, i, c, L.sym, lane);
    return;
  }
  // phase 5: instances sent to the per-call path, or a pool too small, write nothing
  if (g.fallback[i] || ctl_res(g.ctl)[2]) return;
  for (uint64_t c = c0; c < c1; ++c) {
    if (BRANCH == kBranchAcc || (BRANCH == kBranchBoth && x.acc)) p_chunk<true, true, NARROW>(g, x, i, c, L.num, lane);
    else p_chunk<false, true, NARROW>(g, x, i, c, L.num, lane);
  }
}

// Waits until every item of phase p is complete (lane 0 polls), then acquires
// what those items wrote.  Returns false if the wait gave up.
__device__ __forceinline__ bool wait_phase(const PArgs& g, int p, int lane) {
  uint32_t ok = 1;
  if (lane == 0) {
    const uint64_t* d = ctl_done(g.ctl, p);
    uint64_t spins = 0;
    while (__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < g.n[p]) {
      if (++spins > kSpinLimit || __hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
    if (!ok) atomicOr(g.err, 1u);
  }
  ok = (uint32_t)__builtin_amdgcn_readfirstlane((int)ok);
  __threadfence();
  return ok != 0;
}

// Waves per SIMD, the fastest bounds measured on the 4096-instance FD batch:
// the sizing launch 7 (72 VGPRs; at 8 it spills 27 VGPRs), the numeric launch
// 6 (80), and the launch of every phase 5 (96 VGPRs: at 6 it spills 32 and
// takes 13 % longer).
template <bool NARROW, int MODE, int BRANCH>
__global__ __launch_bounds__(kRowThreads, MODE == kModeSize ? 7 : (MODE == kModeAll ? 5 : 6)) void bt_persist_kernel(
    const PArgs* __restrict__ gp) {
  // the arguments are read from device memory where they are used (scalar
  // loads), rather than held in registers for the whole kernel
  const PArgs& g = *gp;
  __shared__ PLds s_lds[kRowWaves];
  const int w = threadIdx.x / kWave, lane = lane_id();
  // queue q = XCD * kSubQueues + sub: XCD x owns the x-th of kXcds contiguous
  // ranges of every phase's items, and its sub-queue j every kSubQueues-th item
  // of that range from the j-th on, so that the waves of one XCD sweep its
  // range together; a wave drains its home queue, then takes leftovers,
  // preferring the other queues of its own XCD
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint32_t sub = ((blockIdx.x / kXcds) * kRowWaves + (uint32_t)w) % kSubQueues;
  const uint32_t cand = ((xcd + (uint32_t)lane / kSubQueues) % kXcds) * kSubQueues + (sub + (uint32_t)lane) % kSubQueues;
  for (int p = g.first; p <= g.last; ++p) {
    if (p > g.first && !wait_phase(g, p - 1, lane)) return;
    if ((MODE & kModeNumeric) && p == 5) tab_clear(s_lds[w].num, lane);
    const uint64_t n = g.n[p];
    uint64_t did = 0;
    uint32_t cur = xcd * kSubQueues + sub;
    for (;;) {
      uint64_t lo, len;
      queue_range(n, cur, lo, len);
      uint64_t* head = ctl_head(g.ctl, p, cur);
      uint64_t k = ~0ull;
      if (lane == 0 && __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < len)
        k = atomicAdd((unsigned long long*)head, 1ull);
      k = shfl0_u64(k);
      if (k < len) {
        run_item<NARROW, MODE, BRANCH>(g, p, lo + k * kSubQueues, s_lds[w], lane);
        ++did;
        continue;
      }
      // this queue is drained: look for a queue with items left, one queue per lane
      uint64_t clo, clen;
      queue_range(n, cand, clo, clen);
      const bool left = __hip_atomic_load(ctl_head(g.ctl, p, cand), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < clen;
      const uint64_t m = __ballot(left);
      if (!m) break;
      cur = readlane_u32(cand, __builtin_ctzll(m));
    }
    if (did) {
      __threadfence();
      if (lane == 0) atomicAdd((unsigned long long*)ctl_done(g.ctl, p), (unsigned long long)did);
    }
  }
}

// Clears the control block and the fallback flags before a launch and stores
// the launch's arguments where the persistent grid reads them (a kernel, so
// that the launch can be captured in a graph).
__global__ void bt_persist_reset_kernel(PArgs a, PArgs* __restrict__ dst, bool clear_fallback) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kCtlWords; i += gridDim.x * blockDim.x) a.ctl[i] = 0;
  if (clear_fallback)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.count; i += gridDim.x * blockDim.x) a.fallback[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst = a;
}

using PersistKernel = void (*)(const PArgs*);
template <bool NARROW>
PersistKernel persist_kernel_w(int mode, int branch) {
  if (mode == kModeSize) return bt_persist_kernel<NARROW, kModeSize, kBranchAcc>;
  if (mode == kModeNumeric) {
    if (branch == kBranchAcc) return bt_persist_kernel<NARROW, kModeNumeric, kBranchAcc>;
    if (branch == kBranchNa) return bt_persist_kernel<NARROW, kModeNumeric, kBranchNa>;
    return bt_persist_kernel<NARROW, kModeNumeric, kBranchBoth>;
  }
  if (branch == kBranchAcc) return bt_persist_kernel<NARROW, kModeAll, kBranchAcc>;
  if (branch == kBranchNa) return bt_persist_kernel<NARROW, kModeAll, kBranchNa>;
  return bt_persist_kernel<NARROW, kModeAll, kBranchBoth>;
}
PersistKernel persist_kernel(bool narrow, int mode, int branch) {
  return narrow ? persist_kernel_w<true>(mode, branch) : persist_kernel_w<false>(mode, branch);
}

template <class T>
T* take(lco_ctx ctx, Scratch* s, KeptBuffers* keep, size_t n) {
  return keep ? keep->get<T>(n) : s->get<T>(n);
}

}  // namespace

bool persist_eligible(uint64_t mp, uint64_t kp, int64_t nnz_a, int64_t nnz_b) {
  return nnz_a > 0 && nnz_b > 0 && mp <= 2 * (uint64_t)nnz_a + kWave && mp <= kPersistMaxRows &&
         nnz_a <= kPersistMaxEntries && kp < ((uint64_t)1 << 34) && nnz_b < (int64_t)UINT32_MAX;
}

struct PersistBatch::Dev {
  std::vector<PInst> host;
  PInst* inst = nullptr;
  uint32_t* ipre = nullptr;
  PArgs* dargs = nullptr;  // the current launch's arguments on the device
  PArgs a{};
  uint64_t items[kPhases] = {};
  bool narrow = true;
  int grid[4][3] = {};  // by mode and branch: blocks that fill every compute unit
  std::vector<bool> active;  // instances whose numeric phase the launches run
};

PersistBatch::PersistBatch(lco_ctx ctx, const std::vector<PJob>& jobs, Scratch* s, KeptBuffers* keep)
    : ctx_(ctx), dev_(new Dev) {
  const int count = (int)jobs.size();
  Dev& D = *dev_;
  D.host.resize(count);
  int64_t E = 0, K = 0, R = 0, C = 0;
  for (int i = 0; i < count; ++i) {
    const PJob& j = jobs[i];
    PInst& x = D.host[i];
    x = PInst{};
    x.a_livs = j.A->livs;
    x.a_vals = j.A->vals;
    x.b_livs = j.B->livs;
    x.b_vals = j.B->vals;
    x.nnz_a = j.A->nnz;
    x.nnz_b = j.B->nnz;
    x.mp = j.mp;
    x.kp = j.kp;
    x.np = j.np;
    x.kdiv = make_fastdiv(j.kp);
    x.ndiv = make_fastdiv(j.np);
    x.eoff = E;
    x.koff = K;
    x.roff = R;
    x.coff = C;
    x.nchunks = (uint32_t)((j.mp + kWave - 1) / kWave);
    x.group = (uint32_t)std::max(1, j.group);
    x.acc = j.acc ? 1u : 0u;
    D.narrow = D.narrow && j.np < ((uint64_t)1 << 32);
    E += x.nnz_a;
    K += (int64_t)j.kp + 1;
    R += (int64_t)j.mp + 1;
    C += x.nchunks;
  }
  PArgs& a = D.a;
  a.count = count;
  D.inst = take<PInst>(ctx, s, keep, count);
  D.ipre = take<uint32_t>(ctx, s, keep, 4 * (size_t)(count + 1));
  D.dargs = take<PArgs>(ctx, s, keep, 1);
  a.inst = D.inst;
  a.ipre = D.ipre;
  a.bptr = take<uint32_t>(ctx, s, keep, K);
  a.row_start = take<uint32_t>(ctx, s, keep, R);
  a.elen = take<uint32_t>(ctx, s, keep, E);
  a.bstart = take<uint32_t>(ctx, s, keep, E);
  a.shape = take<uint8_t>(ctx, s, keep, R);
  a.cnt = take<uint32_t>(ctx, s, keep, R);
  a.chunk_sum = take<uint32_t>(ctx, s, keep, C);
  a.chunk_off = take<uint64_t>(ctx, s, keep, C);
  a.total = take<uint64_t>(ctx, s, keep, count);
  a.base = take<uint64_t>(ctx, s, keep, count);
  a.fallback = take<uint32_t>(ctx, s, keep, count);
  a.ctl = take<uint64_t>(ctx, s, keep, kCtlWords);
  a.err = ctx->dev_err;
  upload_params();
  // blocks that fill every compute unit, by mode and branch (the same for every batch on a device)
  static std::mutex grid_mu;
  static std::map<std::pair<int, int>, std::array<int, 12>> grid_cache;  // (device, narrow) -> grids
  {
    std::lock_guard<std::mutex> lk(grid_mu);
    auto it = grid_cache.find({ctx->device, D.narrow ? 1 : 0});
    if (it == grid_cache.end()) {
      std::array<int, 12> gr{};
      for (int mode : {kModeSize, kModeNumeric, kModeAll}) {
        for (int branch : {kBranchNa, kBranchAcc, kBranchBoth}) {
          int bpc = 0;
          LCO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &bpc, (const void*)persist_kernel(D.narrow, mode, branch), kRowThreads, 0));
          const int g = ctx->num_cus * std::max(1, bpc);
          gr[mode * 3 + branch] = (g + (int)kXcds - 1) / (int)kXcds * (int)kXcds;
        }
      }
      it = grid_cache.emplace(std::make_pair(ctx->device, D.narrow ? 1 : 0), gr).first;
    }
    for (int mode = 0; mode < 4; ++mode)
      for (int branch = 0; branch < 3; ++branch) D.grid[mode][branch] = mode ? it->second[mode * 3 + branch] : 0;
  }
  set_items(std::vector<bool>(count, true));
}

PersistBatch::~PersistBatch() { delete dev_; }

int PersistBatch::grid() const { return dev_->grid[kModeAll][kBranchAcc]; }

void PersistBatch::set_items(const std::vector<bool>& active) {
  Dev& D = *dev_;
  const int count = (int)D.host.size();
  std::vector<uint32_t> pre(4 * (size_t)(count + 1), 0);
  for (int pi = 0; pi < 4; ++pi) {
    uint64_t run = 0;
    for (int i = 0; i < count; ++i) {
      pre[(size_t)pi * (count + 1) + i] = (uint32_t)run;
      const PInst& x = D.host[i];
      uint64_t items = 0;
      if (pi == 0) items = ((uint64_t)x.nnz_b + kSetupTile) / kSetupTile;
      else if (pi == 1) items = ((uint64_t)x.nnz_a + kSetupTile) / kSetupTile;
      else if (pi == 2 || active[i]) items = (x.nchunks + x.group - 1) / x.group;
      run += items;
      if (run >= UINT32_MAX) fail(LCO_E_UNSUPPORTED, "batch: more than 2^32-1 work items in one phase");
    }
    pre[(size_t)pi * (count + 1) + count] = (uint32_t)run;
    D.items[pi == 3 ? 5 : pi] = run;
  }
  D.items[3] = (uint64_t)count;
  D.items[4] = 1;
  D.active = active;
  LCO_HIP(hipMemcpyAsync(D.ipre, pre.data(), sizeof(uint32_t) * pre.size(), hipMemcpyHostToDevice, ctx_->stream));
  pre_.swap(pre);
}

void PersistBatch::set_params(int i, bool acc, int group) {
  PInst& x = dev_->host[i];
  x.acc = acc ? 1u : 0u;
  x.group = (uint32_t)std::max(1, group);
}

void PersistBatch::upload_params() {
  Dev& D = *dev_;
  LCO_HIP(hipMemcpyAsync(D.inst, D.host.data(), sizeof(PInst) * D.host.size(), hipMemcpyHostToDevice,
                         ctx_->stream));
}

void PersistBatch::launch(int first, int last, uint64_t* out_livs, double* out_vals, uint64_t capacity) {
  Dev& D = *dev_;
  PArgs a = D.a;
  a.first = first;
  a.last = last;
  for (int p = 0; p < kPhases; ++p) a.n[p] = (p >= first && p <= last) ? D.items[p] : 0;
  a.out_livs = out_livs;
  a.out_vals = out_vals;
  a.capacity = capacity;
  LCO_LAUNCH(ctx_, "bt_persist_reset", bt_persist_reset_kernel, 1, 256, 0, a, D.dargs, first == 0);
  if (first < 0 || last > 5 || first > last || (first != 0 && first != 5) || (first == 0 && last < 4))
    fail(LCO_E_ARG, "batch: a persistent launch runs phases 0-4, 5 alone, or 0-5");
  const int mode = first == 5 ? kModeNumeric : last == 5 ? kModeAll : kModeSize;
  const char* name = mode == kModeSize ? "bt_persist_size" : mode == kModeNumeric ? "bt_persist_num" : "bt_persist";
  // the numeric branches the launch needs: those of the instances whose numeric phase it runs
  bool any_acc = false, any_na = false;
  for (size_t i = 0; i < D.host.size(); ++i) {
    if (!D.active[i]) continue;
    any_acc = any_acc || D.host[i].acc;
    any_na = any_na || !D.host[i].acc;
  }
  const int branch = mode == kModeSize ? kBranchAcc : any_acc && any_na ? kBranchBoth : any_na ? kBranchNa : kBranchAcc;
  // no more blocks than the largest phase has items for their waves (small batches), at least one per XCD
  uint64_t most = 1;
  for (int p = first; p <= last; ++p) most = std::max<uint64_t>(most, a.n[p]);
  const uint64_t want = (most + kRowWaves - 1) / kRowWaves;
  const int grid = (int)std::min<uint64_t>((uint64_t)D.grid[mode][branch], (want + kXcds - 1) / kXcds * kXcds);
  LCO_LAUNCH(ctx_, name, persist_kernel(D.narrow, mode, branch), grid, kRowThreads, 0, (const PArgs*)D.dargs);
}

void PersistBatch::read_sizes() {
  Dev& D = *dev_;
  const int count = (int)D.host.size();
  sizes_.assign(count, 0);
  fallback_.assign(count, 0);
  uint64_t res[3] = {0, 0, 0};
  LCO_HIP(hipMemcpyAsync(sizes_.data(), D.a.total, sizeof(uint64_t) * count, hipMemcpyDeviceToHost, ctx_->stream));
  LCO_HIP(hipMemcpyAsync(fallback_.data(), D.a.fallback, sizeof(uint32_t) * count, hipMemcpyDeviceToHost,
                         ctx_->stream));
  LCO_HIP(hipMemcpyAsync(res, D.a.ctl + kCtlRes * kCtlStride, sizeof(res), hipMemcpyDeviceToHost, ctx_->stream));
  sync(ctx_);
  total_ = res[0];
  offsets_.assign(count, 0);
  uint64_t run = 0;
  for (int i = 0; i < count; ++i) {
    offsets_[i] = run;
    run += sizes_[i];
  }
  if (run != total_) fail(LCO_E_HIP, "batch: the device's output offsets disagree with its sizes");
}

}  // namespace lco
