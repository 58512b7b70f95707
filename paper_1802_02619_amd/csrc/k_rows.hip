// Row-by-row sparse products (Section 5.2.2-5.2.4): CSR (accumulator, B
// compressed by rows), DCSR (accumulator, B doubly compressed), CSRNA (no
// accumulator: products sorted and summed).  The column-by-column variants
// (CSC, DCSC, CSCNA) are the same kernels run on the transposed roles: a
// column-major A is a row-major A^T over the same LIV array, so C = A*B
// column by column is C^T = B^T * A^T row by row.
//
// Layout: A' is m' x k' with LIV = col + k'*row (rows contiguous, cols
// ascending); B' is k' x n' with LIV = col + n'*row; the product C' gets
// LIV = col + n'*row.  Each output entry sums its products in ascending order
// of the contracted index starting from 0.0.
//
// Setup: the row pointers of B' (or, when doubly compressed, a hash table of
// its non-empty rows keyed by row id), the rows of A' (row starts, and ids
// unless every row is listed), and for every A' entry its product count and B'
// row start.  When
// few rows of A' are empty, one pass over A' lists all m' rows and writes the
// per-entry data; otherwise head flags, a scan and a compaction list the
// non-empty rows.  Small products do the whole setup in one block.
//
// Work split: the rows of A' are binned by their product count f(i).
//  - at most 4 A' entries and f(i) <= 16: one lane per row (k-way merge of the
//    entries' B' rows); from 65536 A' entries up.
//  - one A' entry and f(i) > 16: a wave copies the scaled B' row; idem.
//  - f(i) <= 64 and at most 64 A' entries: one wave per row, rows in chunks
//    (see row_core.h).  CSR/DCSR insert the row's columns into an LDS hash
//    table and sum each column's products in ascending A' entry order; the
//    outputs are ranked by column and written in order.  CSRNA sorts the
//    (column, product index) pairs with a wave bitonic network and sums runs.
//  - larger rows: products are expanded to global memory keyed by (row rank,
//    column), sorted with the stable radix engine and summed per run.
// A symbolic pass counts every row's outputs, a scan places the rows, and the
// numeric pass writes them.
#include <algorithm>
#include <cstring>

#include "row_core.h"

namespace lco {

namespace {
template <bool DENSE>
__device__ __forceinline__ void b_row(const RowArgs& ra, uint64_t j, uint32_t& start, uint32_t& len) {
  if (DENSE) {
    start = ra.bptr[j];
    len = ra.bptr[j + 1] - start;
  } else {
    // linear probing from the id's home slot; the table always holds an empty slot
    uint64_t slot = dc_home(j, ra.dc_shift);
    for (;;) {
      const ulonglong2 e = ra.dc_tab[slot];
      if (e.x == j) {
        start = (uint32_t)e.y;
        len = (uint32_t)(e.y >> 32);
        return;
      }
      if (e.x == kDcEmpty) {
        start = 0;
        len = 0;
        return;
      }
      slot = (slot + 1) & ra.dc_mask;
    }
  }
}

// ---------------------------------------------------------------- setup kernels

__global__ void seg_heads_kernel(const uint64_t* __restrict__ livs, int64_t n, FastDiv div,
                                 uint32_t* __restrict__ head) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (i == 0 || fd_div(div, livs[i]) != fd_div(div, livs[i - 1])) ? 1u : 0u;
}

__global__ void seg_compact_kernel(const uint64_t* __restrict__ livs, int64_t n, FastDiv div,
                                   const uint32_t* __restrict__ head, const uint32_t* __restrict__ pos,
                                   uint64_t* __restrict__ ids, uint32_t* __restrict__ starts) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (head[i]) {
      ids[pos[i]] = fd_div(div, livs[i]);
      starts[pos[i]] = (uint32_t)i;
    }
    if (i == n - 1) starts[pos[i] + head[i]] = (uint32_t)n;
  }
}

// The pointer arrays below are filled from the entries (fill_slots, row_core.h).

// bptr[r] = first B' entry of row r, for r in [0, k'] (bptr[k'] = nnz_b).
__global__ void dense_ptr_kernel(const uint64_t* __restrict__ livs, int64_t n, FastDiv ndiv, uint64_t kp,
                                 uint32_t* __restrict__ bptr) {
  const int lane = lane_id();
  // whole waves step together (fill_slots)
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; e0 <= n;
       e0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = e0 + lane;
    const bool valid = e <= n;
    uint64_t lo = 0, hi = 0;
    if (valid) {
      lo = e == 0 ? 0 : fd_div(ndiv, livs[e - 1]) + 1;
      hi = (e == n ? kp : fd_div(ndiv, livs[e])) + 1;
    }
    fill_slots(bptr, valid, lo, hi, (uint32_t)e);
  }
}

// Hash table of a doubly compressed B' (slots of {row id, start | length << 32},
// cap a power of two above the row count): every slot empty first.
__global__ void dc_clear_kernel(ulonglong2* __restrict__ tab, uint64_t cap) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x)
    tab[i] = make_ulonglong2(kDcEmpty, 0);
}

// Then the first entry of every row inserts the row: its end is the next row's
// first entry, found in the wave's window of 64 entries or, for the window's
// last row, by a galloping search past the window.  Whole waves step together.
__global__ void dc_table_kernel(const uint64_t* __restrict__ livs, int64_t n, FastDiv div,
                                ulonglong2* __restrict__ tab, int shift, uint64_t mask) {
  const int lane = lane_id();
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; e0 < n;
       e0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = e0 + lane;
    const bool valid = e < n;
    uint64_t j = 0;
    bool head = false;
    if (valid) {
      j = fd_div(div, livs[e]);
      head = e == 0 || fd_div(div, livs[e - 1]) != j;
    }
    const uint64_t heads = __ballot(head);
    if (!head) continue;
    const uint64_t later = lane == kWave - 1 ? 0 : heads & (~0ull << (lane + 1));
    int64_t end;
    if (later) {
      end = e0 + __builtin_ctzll(later);
    } else {
      // every entry from e to the window's end lies in row j
      int64_t known = (e0 + kWave < n ? e0 + kWave : n) - 1;
      int64_t step = kWave;
      int64_t hi = known + step;
      while (hi < n && fd_div(div, livs[hi]) == j) {
        known = hi;
        step <<= 1;
        hi = known + step;
      }
      if (hi > n) hi = n;
      int64_t lo = known + 1;  // the end lies in [lo, hi]
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (fd_div(div, livs[mid]) == j) lo = mid + 1;
        else hi = mid;
      }
      end = lo;
    }
    const uint64_t v = (uint64_t)(uint32_t)e | ((uint64_t)(uint32_t)(end - e) << 32);
    uint64_t slot = dc_home(j, shift);
    for (;;) {
      const unsigned long long prev =
          atomicCAS((unsigned long long*)&tab[slot].x, (unsigned long long)kDcEmpty, (unsigned long long)j);
      if (prev == kDcEmpty) {
        tab[slot].y = v;
        break;
      }
      slot = (slot + 1) & mask;
    }
  }
}

// For each A' entry: the start and length of the B' row its column selects.
template <bool DENSE>
__global__ void entry_len_kernel(RowArgs ra, uint32_t* __restrict__ len, uint32_t* __restrict__ bstart) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ra.nnz_a;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t j;
    fd_divmod(ra.kdiv, ra.a_livs[e], j);
    uint32_t s, l;
    b_row<DENSE>(ra, j, s, l);
    len[e] = l;
    bstart[e] = s;
  }
}

// The same, together with the rows of A' taken densely, every row 0..m'-1
// including empty ones (for products where A' has few empty rows):
// row_start[r] = first entry of row r, *count = m' (row r of the list is row r
// of A', so no ids are stored).  Empty rows hold no products and are skipped.
// Also clears the four counter words `zero4` of the classification that
// follows.
template <bool DENSE>
__global__ void dense_rows_len_kernel(RowArgs ra, uint64_t mp, uint32_t* __restrict__ row_start,
                                      uint64_t* __restrict__ count,
                                      uint32_t* __restrict__ len, uint32_t* __restrict__ bstart,
                                      uint64_t* __restrict__ zero4) {
  const int64_t n = ra.nnz_a;
  if (blockIdx.x == 0 && threadIdx.x < 4) zero4[threadIdx.x] = 0;  // the classification's counters
  const int lane = lane_id();
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; e0 <= n;
       e0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = e0 + lane;
    const bool valid = e <= n;
    uint64_t lo = 0, hi = 0;
    if (valid) {
      hi = mp;
      if (e < n) {
        uint64_t j;
        hi = fd_divmod(ra.kdiv, ra.a_livs[e], j);
        uint32_t st, l;
        b_row<DENSE>(ra, j, st, l);
        len[e] = l;
        bstart[e] = st;
      }
      ++hi;
      lo = e == 0 ? 0 : fd_div(ra.kdiv, ra.a_livs[e - 1]) + 1;
      if (e == n) *count = mp;
    }
    fill_slots(row_start, valid, lo, hi, (uint32_t)e);
  }
}

// The class of row r (entries [e0, e1)); `classes` enables the tiny and copy
// classes.  A long row reports its product count through *f_long (else 0).
__device__ __forceinline__ uint8_t classify_row(const RowArgs& ra, uint32_t e0, uint32_t e1, bool classes,
                                                uint64_t* f_long) {
  uint64_t f = 0, mx = 0;
  for (uint32_t e = e0; e < e1; ++e) {
    const uint64_t l = ra.elen[e];
    f += l;
    mx = l > mx ? l : mx;
  }
  *f_long = 0;
  if (f == 0) return kShapeSkip;
  if (classes && e1 - e0 <= (uint32_t)kTinyEntries && f <= (uint64_t)kTinyProducts) return kShapeTiny;
  if (classes && e1 - e0 == 1) return kShapeCopy;
  if (small_row(f, e1 - e0)) {
    uint32_t lw = 0;
    while ((1ull << lw) < mx) ++lw;
    return ((uint64_t)(e1 - e0) << lw) <= (uint64_t)kWave ? (uint8_t)lw : kShapeSearch;
  }
  *f_long = f;
  return kShapeLong;
}

constexpr int kClassifyThreads = 256;

// Writes the shape code of every row and collects the long rows (more than 64
// products or entries, except single-entry rows) in `list2` with their product
// counts `f2`; `*n2` (zero on entry) ends as their number.  List order is
// arbitrary: each long row's result depends only on its own products.
// `*tiny` / `*copy` / `*wave` are set when some row is of that class (`wave`: a
// row of the one-wave kernel).  `fl` (one word per row) holds the product count
// of each long row between the two passes below.
// The first pass classifies the rows and counts the long ones per wave; one
// atomic per block then reserves the block's part of the list, and the second
// pass writes it.  (A reservation per wave and row chunk serialised hundreds of
// thousands of atomics on the one counter word when most chunks hold a long row.)
__global__ __launch_bounds__(kClassifyThreads) void row_classify_kernel(
    RowArgs ra, int64_t upper, bool classes, uint64_t* __restrict__ n2, uint32_t* __restrict__ list2,
    uint64_t* __restrict__ f2, uint64_t* __restrict__ fl, uint8_t* __restrict__ shape, uint32_t* __restrict__ tiny,
    uint32_t* __restrict__ copy, uint32_t* __restrict__ wave) {
  constexpr int kWaves = kClassifyThreads / kWave;
  __shared__ uint64_t s_off[kWaves + 1];
  const int64_t nzr = (int64_t)*ra.nzr_a;
  const int64_t end = nzr < upper ? nzr : upper;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int64_t first = (int64_t)blockIdx.x * kClassifyThreads + threadIdx.x - lane;
  const int64_t stride = (int64_t)gridDim.x * kClassifyThreads;
  uint64_t nlong = 0, any = 0;  // long rows of this wave; classes seen (bit 0 tiny, 1 copy, 2 one-wave)
  // whole waves step together (every lane takes part in the shuffles below)
  for (int64_t r0 = first; r0 < end; r0 += stride) {
    const int64_t r = r0 + lane;
    const bool valid = r < end;
    const uint32_t e0 = valid ? ra.row_start[r] : 0u, e1 = valid ? ra.row_start[r + 1] : 0u;
    // a row of more than 64 entries is long (or has no products): only its
    // product count is needed, summed by the whole wave with coalesced loads
    const bool many = e1 - e0 > (uint32_t)kWave;
    uint64_t f = 0;
    uint8_t sh = kShapeSkip;
    if (valid && !many) sh = classify_row(ra, e0, e1, classes, &f);
    for (uint64_t m = __ballot(many); m; m &= m - 1) {
      const int src = __builtin_ctzll(m);
      const uint32_t b0 = __shfl(e0, src, kWave), b1 = __shfl(e1, src, kWave);
      uint64_t acc = 0;
      uint64_t e = (uint64_t)b0 + lane;
      for (; e + 3 * kWave < b1; e += 4 * kWave)
        acc += (uint64_t)ra.elen[e] + ra.elen[e + kWave] + ra.elen[e + 2 * kWave] + ra.elen[e + 3 * kWave];
      for (; e < b1; e += kWave) acc += ra.elen[e];
      acc = wave_reduce_sum(acc);
      if (lane == src) {
        f = acc;
        sh = acc ? kShapeLong : kShapeSkip;
      }
    }
    if (valid) {
      shape[r] = sh;
      if (sh == kShapeLong) fl[r] = f;
    }
    nlong += (uint64_t)__popcll(__ballot(valid && sh == kShapeLong));
    any |= (__ballot(valid && sh == kShapeTiny) ? 1u : 0u) | (__ballot(valid && sh == kShapeCopy) ? 2u : 0u) |
           (__ballot(valid && sh <= kShapeSearch) ? 4u : 0u);
  }
  if (lane == 0) {
    if (any & 1u) *tiny = 1u;
    if (any & 2u) *copy = 1u;
    if (any & 4u) *wave = 1u;
    s_off[w] = nlong;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tot = 0;
    for (int i = 0; i < kWaves; ++i) {
      const uint64_t c = s_off[i];
      s_off[i] = tot;
      tot += c;
    }
    s_off[kWaves] = tot ? atomicAdd((unsigned long long*)n2, (unsigned long long)tot) : 0ull;
  }
  __syncthreads();
  if (nlong == 0) return;
  // second pass over the same rows: each lane re-reads the codes it wrote
  uint64_t base = s_off[kWaves] + s_off[w];
  for (int64_t r0 = first; r0 < end; r0 += stride) {
    const int64_t r = r0 + lane;
    const bool is_long = r < end && shape[r] == kShapeLong;
    const uint64_t lm = __ballot(is_long);
    if (is_long) {
      const uint64_t i = base + (uint64_t)__popcll(lm & lanemask_lt());
      list2[i] = (uint32_t)r;
      f2[i] = fl[r];
    }
    base += (uint64_t)__popcll(lm);
  }
}

// ---------------------------------------------------------------- small products: all setup in one block
//
// For small operands (singly compressed B') the setup phases run in one block:
// the rows of A' (heads, a block scan, compaction), the row pointers of B',
// each A' entry's product count and B' row start, and the row classes.  The
// kernel writes its counters itself: words[0] rows of A', [1] long rows, [2..4]
// some row is tiny / a copy / of the one-wave kernel.  It also clears the
// per-row output counts cnt[0..nnz_A] (at least as many as there are rows), so
// that the symbolic pass can follow without the row count on the host.
constexpr int kSetupThreads = 1024;
constexpr int64_t kClassMinEntries = 65536;  // A' entries from which the tiny and copy classes are used
constexpr int64_t kSetupMaxEntries = 16384;
constexpr uint64_t kSetupMaxRowPtr = 65536;

__global__ __launch_bounds__(kSetupThreads) void row_setup_small_kernel(
    RowArgs ra, FastDiv ndiv, bool classes, uint32_t* __restrict__ row_start, uint64_t* __restrict__ row_id,
    uint64_t* __restrict__ words, uint32_t* __restrict__ bptr, uint32_t* __restrict__ elen,
    uint32_t* __restrict__ bstart, uint32_t* __restrict__ list2, uint64_t* __restrict__ f2,
    uint8_t* __restrict__ shape, uint64_t* __restrict__ cnt) {
  __shared__ uint32_t wsum[kSetupThreads / kWave + 1];
  __shared__ uint32_t s_cnt[4];  // long rows, tiny, copy, wave
  const int64_t na = ra.nnz_a, nb = ra.nnz_b;
  const int tid = threadIdx.x;
  if (tid < 4) s_cnt[tid] = 0;
  for (int64_t i = tid; i <= na; i += kSetupThreads) cnt[i] = 0;
  // row pointers of B'
  for (int64_t e = tid; e <= nb; e += kSetupThreads) {
    const uint64_t lo = e == 0 ? 0 : fd_div(ndiv, ra.b_livs[e - 1]) + 1;
    const uint64_t hi = e == nb ? ra.kp : fd_div(ndiv, ra.b_livs[e]);
    for (uint64_t r = lo; r <= hi; ++r) bptr[r] = (uint32_t)e;
  }
  // rows of A': each thread counts the row heads of a contiguous run of entries
  const int64_t per = (na + kSetupThreads - 1) / kSetupThreads;
  const int64_t e0 = (int64_t)tid * per < na ? (int64_t)tid * per : na;
  const int64_t e1 = e0 + per < na ? e0 + per : na;
  uint32_t heads = 0;
  for (int64_t e = e0; e < e1; ++e)
    heads += (e == 0 || fd_div(ra.kdiv, ra.a_livs[e]) != fd_div(ra.kdiv, ra.a_livs[e - 1])) ? 1u : 0u;
  uint32_t nzr;
  uint32_t r = block_exclusive_scan(heads, wsum, nzr);
  for (int64_t e = e0; e < e1; ++e) {
    const uint64_t row = fd_div(ra.kdiv, ra.a_livs[e]);
    if (e == 0 || row != fd_div(ra.kdiv, ra.a_livs[e - 1])) {
      row_start[r] = (uint32_t)e;
      row_id[r] = row;
      ++r;
    }
  }
  if (tid == 0) row_start[nzr] = (uint32_t)na;
  __syncthreads();
  // each A' entry: its B' row
  for (int64_t e = tid; e < na; e += kSetupThreads) {
    uint64_t j;
    fd_divmod(ra.kdiv, ra.a_livs[e], j);
    bstart[e] = bptr[j];
    elen[e] = bptr[j + 1] - bptr[j];
  }
  __syncthreads();
  // row classes
  for (uint32_t rr = tid; rr < nzr; rr += kSetupThreads) {
    uint64_t f;
    const uint8_t sh = classify_row(ra, row_start[rr], row_start[rr + 1], classes, &f);
    if (sh == kShapeTiny) s_cnt[1] = 1u;
    else if (sh == kShapeCopy) s_cnt[2] = 1u;
    else if (sh <= kShapeSearch) s_cnt[3] = 1u;
    else if (sh == kShapeLong) {
      const uint32_t i = atomicAdd(&s_cnt[0], 1u);
      list2[i] = rr;
      f2[i] = f;
    }
    shape[rr] = sh;
  }
  __syncthreads();
  if (tid < 5) words[tid] = tid == 0 ? (uint64_t)nzr : (uint64_t)s_cnt[tid - 1];
}

// ---------------------------------------------------------------- one wave per row, rows in chunks
//
// Each wave takes chunks of up to 64 consecutive rows (fewer when there are too
// few rows to give every resident wave a full chunk).  The chunk's row metadata
// (starts, ids, shapes, output offsets) and a window of 64 consecutive A'
// entries (product counts, B' row starts, LIVs, values) are read with one
// coalesced load per array; a row then takes its entries' data from the window
// by lane shuffles, so the only global loads that depend on the row are those
// of its rows of B'.  The window moves forward when a row's entries leave it
// (rows are consecutive, so their entries are too).  The symbolic pass is held
// to 8 waves per SIMD (64 VGPRs) and the numeric pass to 6 (80 VGPRs), the
// fastest bounds measured.  NARROW: columns below 2^32 (n' < 2^32), fixed at
// compile time so that the width is no per-row branch.  With `nzr_dev` the
// row count is the smaller of `nzr` (an upper bound) and *nzr_dev.
constexpr int kChunkRows = kWave;

template <bool ACC, bool NUMERIC, bool NARROW>
__global__ __launch_bounds__(kRowThreads, NUMERIC ? 6 : 8) void row_chunk_kernel(RowArgs ra, uint32_t nzr, int chunk_rows,
                                                                const uint8_t* __restrict__ shape,
                                                                uint64_t* __restrict__ cnt,
                                                                const uint64_t* __restrict__ coff,
                                                                uint64_t* __restrict__ out_livs,
                                                                double* __restrict__ out_vals,
                                                                const uint64_t* __restrict__ nzr_dev) {
  __shared__ RowLds<NUMERIC> s_lds[kRowWaves];
  if (nzr_dev && *nzr_dev < (uint64_t)nzr) nzr = (uint32_t)*nzr_dev;
  const int w = threadIdx.x / kWave, lane = lane_id();
  constexpr bool narrow = NARROW;  // columns below 2^32 (n' < 2^32)
  const uint64_t nchunks = ((uint64_t)nzr + chunk_rows - 1) / chunk_rows;
  const RowSpan span = xcd_row_span(nchunks, w);
  if constexpr (ACC && NUMERIC) tab_clear(s_lds[w], lane);
  for (uint64_t c = span.first; c < span.end; c += span.step) {
    const uint64_t r0 = c * chunk_rows;
    const int rows = (int)((uint64_t)nzr - r0 < (uint64_t)chunk_rows ? (uint64_t)nzr - r0 : (uint64_t)chunk_rows);
    uint32_t m_s0 = 0, m_s1 = 0, m_sh = kShapeSkip;
    uint64_t m_id = 0, m_off = 0;
    if (lane < rows) {
      const uint64_t r = r0 + lane;
      m_s0 = ra.row_start[r];
      m_s1 = ra.row_start[r + 1];
      m_id = row_of(ra, r);
      m_sh = shape[r];
      if (NUMERIC) m_off = coff[r];
    }
    uint32_t my_cnt = 0;
    // The window [w0, w0 + 64) of A' entries (entry indexes are 32-bit here, so
    // the window tests are scalar compares); none is loaded before the first row.
    bool have = false;
    uint32_t w0 = 0;
    // window lane l: entry w0 + l's product count, B' row start, value, and
    // j * n' (the LIV of its B' row's first position, j = its contracted index)
    uint32_t x_len = 0, x_bs = 0;
    uint64_t x_jn = 0;
    double x_av = 0.0;
    // Rows of this kernel (no products, long rows and rows of the lane and copy
    // kernels are skipped).  The B' loads of the next row are issued before the
    // current row is reduced, so that their latency overlaps its LDS work.
    uint64_t todo = __ballot(lane < rows && m_sh <= kShapeSearch);
    RowProduct<NUMERIC> next;
    int t_next = 0;
    auto stage = [&](int i) {
      const uint8_t sh = (uint8_t)readlane_u32(m_sh, i);
      const uint32_t e0 = readlane_u32(m_s0, i), e1 = readlane_u32(m_s1, i);
      t_next = (int)(e1 - e0);  // at most 64 for the rows of this kernel
      if (!have || e0 - w0 > (uint32_t)(kWave - t_next)) {
        have = true;
        w0 = e0;
        const uint64_t e = (uint64_t)w0 + (uint32_t)lane;
        if (e < (uint64_t)ra.nnz_a) {
          x_len = ra.elen[e];
          x_bs = ra.bstart[e];
          uint64_t j;
          fd_divmod(ra.kdiv, ra.a_livs[e], j);
          x_jn = j * ra.np;
          if (NUMERIC) x_av = ra.a_vals[e];
        }
      }
      window_products<NUMERIC>(ra.b_livs, ra.b_vals, e0, t_next, sh, lane, (int64_t)w0, x_len, x_bs, x_jn, x_av,
                               next);
    };
    if (todo) stage(__builtin_ctzll(todo));
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
      const uint32_t d = row_reduce<ACC, NUMERIC>(valid, ent, col, v, t, narrow, lane, s_lds[w], o);
      if (!NUMERIC) {
        if (lane == i) my_cnt = d;
      } else if (o.own) {
        // the row's output range starts at a wave-uniform address; the rank
        // (below 64) is the per-lane offset
        const uint64_t r_off = readlane_u64(m_off, i);
        const uint32_t boff = o.rank * 8u;
        *reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(out_livs + r_off) + boff) =
            o.col + ra.np * readlane_u64(m_id, i);
        *reinterpret_cast<double*>(reinterpret_cast<char*>(out_vals + r_off) + boff) = o.val;
      }
    }
    if (!NUMERIC && lane < rows) cnt[r0 + lane] = my_cnt;
  }
}

// ---------------------------------------------------------------- tiny rows: one lane per row
//
// A row with at most kTinyEntries entries and kTinyProducts products is merged
// by one lane: the entries' B' rows are ascending in column, so a k-way merge
// visits the row's columns in ascending order, and at each column the entries
// that hold it are added in entry order (ascending contracted index) from 0.0.
// Each wave takes 64 consecutive rows.  When all of them are tiny (or have no
// output) and their outputs fit kTinyStage entries, the outputs form one
// contiguous range: they are staged in LDS and stored with coalesced writes.
constexpr int kTinyStage = 512;

template <bool NUMERIC>
__device__ __forceinline__ uint32_t tiny_merge(const RowArgs& ra, uint32_t r, uint64_t base, bool stage, uint64_t* sk,
                                               double* sv, uint64_t* __restrict__ out_livs,
                                               double* __restrict__ out_vals) {
  const uint32_t e0 = ra.row_start[r];
  const int t = (int)(ra.row_start[r + 1] - e0);
  const uint64_t row = row_of(ra, r);
  uint32_t p[kTinyEntries], end[kTinyEntries];
  uint64_t jn[kTinyEntries], col[kTinyEntries];
  double av[kTinyEntries];
#pragma unroll
  for (int e = 0; e < kTinyEntries; ++e) {
    p[e] = 0;
    end[e] = 0;
    jn[e] = 0;
    col[e] = 0;
    av[e] = 0.0;
    if (e < t) {
      const uint32_t ge = e0 + e;
      p[e] = ra.bstart[ge];
      end[e] = p[e] + ra.elen[ge];
      jn[e] = (ra.a_livs[ge] - ra.kp * row) * ra.np;
      if (NUMERIC) av[e] = ra.a_vals[ge];
      if (p[e] < end[e]) col[e] = ra.b_livs[p[e]] - jn[e];
    }
  }
  uint32_t d = 0;
  for (int step = 0; step < kTinyProducts; ++step) {
    bool any = false;
    uint64_t m = 0;
#pragma unroll
    for (int e = 0; e < kTinyEntries; ++e) {
      if (p[e] < end[e] && (!any || col[e] < m)) {
        m = col[e];
        any = true;
      }
    }
    if (!any) break;
    double sum = 0.0;
#pragma unroll
    for (int e = 0; e < kTinyEntries; ++e) {
      if (p[e] < end[e] && col[e] == m) {
        if (NUMERIC) sum += av[e] * ra.b_vals[p[e]];
        ++p[e];
        if (p[e] < end[e]) col[e] = ra.b_livs[p[e]] - jn[e];
      }
    }
    if (NUMERIC) {
      if (stage) {
        sk[base + d] = m + ra.np * row;
        sv[base + d] = sum;
      } else {
        out_livs[base + d] = m + ra.np * row;
        out_vals[base + d] = sum;
      }
    }
    ++d;
  }
  return d;
}

template <bool NUMERIC>
__global__ __launch_bounds__(256) void row_tiny_kernel(RowArgs ra, uint32_t nzr, const uint8_t* __restrict__ shape,
                                                       uint64_t* __restrict__ cnt, const uint64_t* __restrict__ coff,
                                                       uint64_t* __restrict__ out_livs,
                                                       double* __restrict__ out_vals) {
  __shared__ uint64_t s_key[NUMERIC ? 4 : 1][NUMERIC ? kTinyStage : 1];
  __shared__ double s_val[NUMERIC ? 4 : 1][NUMERIC ? kTinyStage : 1];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  for (uint32_t r0 = (blockIdx.x * (blockDim.x / kWave) + w) * kWave; r0 < nzr; r0 += waves * kWave) {
    const uint32_t r = r0 + lane;
    const bool in = r < nzr;
    const bool tiny = in && shape[r] == kShapeTiny;
    if (!NUMERIC) {
      if (tiny) cnt[r] = tiny_merge<false>(ra, r, 0, false, nullptr, nullptr, nullptr, nullptr);
      continue;
    }
    const uint32_t rl = r0 + kWave < nzr ? r0 + kWave : nzr;
    const uint64_t wbase = coff[r0], span = coff[rl] - wbase;
    const bool quiet = !in || tiny || coff[r + 1] == coff[r];
    const bool stage = span <= (uint64_t)kTinyStage && __ballot(quiet) == ~0ull;
    if (tiny)
      tiny_merge<true>(ra, r, stage ? coff[r] - wbase : coff[r], stage, s_key[NUMERIC ? w : 0],
                       s_val[NUMERIC ? w : 0], out_livs, out_vals);
    if (stage) {
      wave_lds_sync();
      for (uint32_t q = lane; q < (uint32_t)span; q += kWave) {
        out_livs[wbase + q] = s_key[NUMERIC ? w : 0][q];
        out_vals[wbase + q] = s_val[NUMERIC ? w : 0][q];
      }
      wave_lds_sync();
    }
  }
}

// ---------------------------------------------------------------- single-entry rows: scaled copies
//
// A row with one A' entry (and more than kTinyProducts products) has as
// products that entry's B' row scaled, already ascending in column and without
// repeats: each output is 0.0 + a*b.  Symbolic pass: one thread per row writes
// the count.  Numeric pass: a wave takes 64 consecutive rows and copies each
// of their copy rows with coalesced loads and stores.
template <bool NUMERIC>
__global__ __launch_bounds__(256) void row_copy_kernel(RowArgs ra, uint32_t nzr, const uint8_t* __restrict__ shape,
                                                       uint64_t* __restrict__ cnt, const uint64_t* __restrict__ coff,
                                                       uint64_t* __restrict__ out_livs,
                                                       double* __restrict__ out_vals) {
  if (!NUMERIC) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nzr; r += gridDim.x * blockDim.x)
      if (shape[r] == kShapeCopy) cnt[r] = ra.elen[ra.row_start[r]];
    return;
  }
  // Each wave takes 64 consecutive rows: one coalesced load of their shapes,
  // and every copy row's metadata loaded by its own lane at once; the wave then
  // copies the chunk's copy rows one after another.
  const int lane = lane_id();
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  for (uint64_t r0 = (uint64_t)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kWave; r0 < nzr;
       r0 += (uint64_t)waves * kWave) {
    const uint32_t r = (uint32_t)(r0 + lane);
    const bool mine = r0 + lane < nzr && shape[r] == kShapeCopy;
    uint32_t len = 0, bs = 0;
    uint64_t jn = 0, base = 0, rowc = 0;
    double a = 0.0;
    if (mine) {
      const uint32_t e0 = ra.row_start[r];
      const uint64_t row = row_of(ra, r);
      len = ra.elen[e0];
      bs = ra.bstart[e0];
      jn = (ra.a_livs[e0] - ra.kp * row) * ra.np;
      a = ra.a_vals[e0];
      base = coff[r];
      rowc = ra.np * row;
    }
    for (uint64_t m = __ballot(mine); m; m &= m - 1) {
      const int src = __builtin_ctzll(m);
      const uint32_t l = readlane_u32(len, src), b = readlane_u32(bs, src);
      const uint64_t j = readlane_u64(jn, src), o = readlane_u64(base, src), rc = readlane_u64(rowc, src);
      const double av = __longlong_as_double((long long)readlane_u64((uint64_t)__double_as_longlong(a), src));
      for (uint32_t q = lane; q < l; q += kWave) {
        out_livs[o + q] = (ra.b_livs[b + q] - j) + rc;
        out_vals[o + q] = 0.0 + av * ra.b_vals[b + q];
      }
    }
  }
}

// ---------------------------------------------------------------- long rows (global sort)

constexpr int kBigThreads = 256;

// Long row number li (list[li]) expands its products at off2[li], keyed by
// (li, column); the key's list position keeps every row's products together.
__global__ __launch_bounds__(kBigThreads) void big_expand_kernel(RowArgs ra, const uint32_t* __restrict__ list,
                                                                 uint32_t count, const uint64_t* __restrict__ off2,
                                                                 int colbits, uint64_t* __restrict__ keys,
                                                                 double* __restrict__ vals) {
  for (uint32_t li = blockIdx.x; li < count; li += gridDim.x) {
    if (off2[li + 1] == off2[li]) continue;  // a row of the in-LDS path
    const uint32_t r = list[li];
    const uint32_t e0 = ra.row_start[r], e1 = ra.row_start[r + 1];
    const uint64_t p0 = ra.poff[e0];
    const uint64_t f = ra.poff[e1] - p0;
    const uint64_t row = row_of(ra, r);
    const uint64_t qk = (uint64_t)li << colbits;
    const uint64_t base = off2[li];
    for (uint64_t p = threadIdx.x; p < f; p += kBigThreads) {
      // last A' entry e in [e0, e1) with poff[e] <= p0 + p
      uint32_t lo = e0, hi = e1 - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (ra.poff[mid] <= p0 + p) lo = mid;
        else hi = mid - 1;
      }
      const uint64_t j = ra.a_livs[lo] - ra.kp * row;
      const uint32_t q = ra.bstart[lo] + (uint32_t)(p0 + p - ra.poff[lo]);
      const uint64_t col = ra.b_livs[q] - ra.np * j;
      keys[base + p] = qk | col;
      vals[base + p] = ra.a_vals[lo] * ra.b_vals[q];
    }
  }
}

// Distinct keys of each long row (symbolic) or their run sums (numeric).
template <bool NUMERIC>
__global__ __launch_bounds__(kBigThreads) void big_reduce_kernel(RowArgs ra, const uint32_t* __restrict__ list,
                                                                 uint32_t count, const uint64_t* __restrict__ off2,
                                                                 const uint64_t* __restrict__ keys,
                                                                 const double* __restrict__ vals,
                                                                 uint64_t colmask, uint64_t* __restrict__ cnt,
                                                                 const uint64_t* __restrict__ coff,
                                                                 uint64_t* __restrict__ out_livs,
                                                                 double* __restrict__ out_vals) {
  __shared__ uint32_t wsum[kBigThreads / kWave + 1];
  for (uint32_t li = blockIdx.x; li < count; li += gridDim.x) {
    const uint64_t f = off2[li + 1] - off2[li];
    if (f == 0) continue;  // a row of the in-LDS path
    const uint32_t r = list[li];
    const uint64_t base = off2[li];
    const uint64_t row = row_of(ra, r);
    uint64_t run = 0;  // heads seen before this chunk
    for (uint64_t c0 = 0; c0 < f; c0 += kBigThreads) {
      const uint64_t p = c0 + threadIdx.x;
      const bool head = p < f && (p == 0 || keys[base + p] != keys[base + p - 1]);
      uint32_t total;
      const uint32_t ex = block_exclusive_scan<uint32_t>(head ? 1u : 0u, wsum, total);
      if (NUMERIC && head) {
        const uint64_t key = keys[base + p];
        double acc = 0.0;
        for (uint64_t q = p; q < f && keys[base + q] == key; ++q) acc += vals[base + q];
        const uint64_t o = coff[r] + run + ex;
        out_livs[o] = (key & colmask) + ra.np * row;
        out_vals[o] = acc;
      }
      run += total;
    }
    if (!NUMERIC && threadIdx.x == 0) cnt[r] = run;
  }
}

// Long rows of at most kMidMax products are computed in LDS, once: the row's
// products are expanded keyed by (column, product index), put in key order by
// a bitonic network, and each column's run is summed in product order, which
// is ascending A' entry order, hence ascending contracted index (the keys are
// distinct, so this is the order the stable global sort gives).  Each row's
// output goes to a staging list at the row's product offset `moff` and its
// count to cnt[r]; once the rows are placed, row_mid_copy moves it to C.
constexpr int kMidThreads = 256;
constexpr int kMidBits = 12;
constexpr int kMidMax = 1 << kMidBits;
constexpr int kMidWaveMax = 256;  // rows of at most this many products take one wave

// Product p of a long row from its A' entry e (absolute index).
__device__ __forceinline__ void mid_product_of(const RowArgs& ra, uint32_t e, uint64_t p0, uint64_t row, uint32_t p,
                                               int pbits, uint64_t& key, double& val) {
  const uint64_t j = ra.a_livs[e] - ra.kp * row;
  const uint32_t q = ra.bstart[e] + (uint32_t)(p0 + p - ra.poff[e]);
  const uint64_t col = ra.b_livs[q] - ra.np * j;
  key = (col << pbits) | p;
  val = ra.a_vals[e] * ra.b_vals[q];
}

__device__ __forceinline__ int mid_bits(uint64_t f) {
  int pbits = 6;
  while (((uint64_t)1 << pbits) < f) ++pbits;
  return pbits;
}

// One wave per row of at most kMidWaveMax products (four rows per block).
__global__ __launch_bounds__(kMidThreads) void row_midw_kernel(RowArgs ra, const uint32_t* __restrict__ list,
                                                               const uint32_t* __restrict__ bin, uint32_t count,
                                                               const uint64_t* __restrict__ f2,
                                                               const uint64_t* __restrict__ moff,
                                                               uint64_t* __restrict__ cnt,
                                                               uint64_t* __restrict__ tmp_livs,
                                                               double* __restrict__ tmp_vals) {
  constexpr int kWaves = kMidThreads / kWave;
  constexpr int kPer = kMidWaveMax / kWave;
  __shared__ uint64_t skey_all[kWaves][kMidWaveMax];
  __shared__ double sval_all[kWaves][kMidWaveMax];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  uint64_t* skey = skey_all[w];
  double* sval = sval_all[w];
  for (uint32_t k = blockIdx.x * kWaves + w; k < count; k += gridDim.x * kWaves) {
    const uint32_t li = bin[k];
    const uint64_t f = f2[li];
    const uint32_t r = list[li];
    const uint32_t e0 = ra.row_start[r], e1 = ra.row_start[r + 1];
    const uint64_t p0 = ra.poff[e0];
    const uint64_t row = row_of(ra, r);
    const int pbits = mid_bits(f);
    const uint32_t P = 1u << pbits;
    // Each product's A' entry: every entry with products marks its first
    // product's position, and a running maximum over the positions (entries
    // come in product order) hands every position its entry.  The marks use
    // the value area, which the expansion fills afterwards.
    uint32_t* ent = reinterpret_cast<uint32_t*>(sval);
#pragma unroll
    for (int i = 0; i < kPer; ++i) ent[i * kWave + lane] = 0;
    wave_lds_sync();
    for (uint32_t e = lane; e < e1 - e0; e += kWave) {
      const uint64_t a = ra.poff[e0 + e] - p0, b = ra.poff[e0 + e + 1] - p0;
      if (b > a) ent[a] = e;
    }
    wave_lds_sync();
    {
      uint32_t top = 0, seg[kPer];
#pragma unroll
      for (int i = 0; i < kPer; ++i) {  // this lane's positions kPer * lane + i
        const uint32_t x = ent[kPer * lane + i];
        top = x > top ? x : top;
        seg[i] = top;
      }
      const uint32_t incl = wave_inclusive_max(top);
      uint32_t before = (uint32_t)__shfl_up((int)incl, 1, kWave);
      if (lane == 0) before = 0;
#pragma unroll
      for (int i = 0; i < kPer; ++i) ent[kPer * lane + i] = seg[i] > before ? seg[i] : before;
    }
    wave_lds_sync();
    uint32_t mine[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) mine[i] = ent[i * kWave + lane];
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const uint32_t p = (uint32_t)(i * kWave + lane);
      if (p < P) {
        uint64_t key = ~0ull;  // padding sorts last
        double v = 0.0;
        if (p < f) mid_product_of(ra, e0 + mine[i], p0, row, p, pbits, key, v);
        skey[p] = key;
        sval[p] = v;
      }
    }
    wave_lds_sync();
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
        for (int h = 0; h < kPer / 2; ++h) {
          const uint32_t i = (uint32_t)(h * kWave + lane);
          if (i < P / 2) {
            const uint32_t lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
            const uint32_t hi = lo | j;
            const uint64_t a = skey[lo], b = skey[hi];
            if ((a > b) == ((lo & k) == 0)) {
              skey[lo] = b;
              skey[hi] = a;
            }
          }
        }
        wave_lds_sync();
      }
    }
    const uint64_t base = moff[li];
    uint64_t run = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const uint32_t q = (uint32_t)(i * kWave + lane);
      const uint64_t col = q < f ? skey[q] >> pbits : 0;
      const bool head = q < f && (q == 0 || (skey[q - 1] >> pbits) != col);
      const uint64_t hm = __ballot(head);
      if (head) {
        double acc = 0.0;
        for (uint32_t t = q; t < (uint32_t)f && (skey[t] >> pbits) == col; ++t) acc += sval[skey[t] & (P - 1)];
        const uint64_t o = base + run + (uint64_t)__popcll(hm & lanemask_lt());
        tmp_livs[o] = col + ra.np * row;
        tmp_vals[o] = acc;
      }
      run += (uint64_t)__popcll(hm);
    }
    if (lane == 0) cnt[r] = run;
    wave_lds_sync();  // every run is summed before the next row is expanded
  }
}

// One block per row of more than fmin and at most MAXP products.
template <int MAXP>
__global__ __launch_bounds__(kMidThreads) void row_mid_kernel(RowArgs ra, const uint32_t* __restrict__ list,
                                                              const uint32_t* __restrict__ bin, uint32_t count,
                                                              const uint64_t* __restrict__ f2,
                                                              const uint64_t* __restrict__ moff,
                                                              uint64_t* __restrict__ cnt,
                                                              uint64_t* __restrict__ tmp_livs,
                                                              double* __restrict__ tmp_vals) {
  __shared__ uint64_t skey[MAXP];
  __shared__ double sval[MAXP];
  __shared__ uint32_t wsum[kMidThreads / kWave + 1];
  const uint32_t tid = threadIdx.x;
  for (uint32_t k = blockIdx.x; k < count; k += gridDim.x) {
    const uint32_t li = bin[k];
    const uint64_t f = f2[li];
    const uint32_t r = list[li];
    const uint32_t e0 = ra.row_start[r], e1 = ra.row_start[r + 1];
    const uint64_t p0 = ra.poff[e0];
    const uint64_t row = row_of(ra, r);
    const int pbits = mid_bits(f);
    const uint32_t P = 1u << pbits;
    // each product's A' entry, as in the one-wave kernel: marks, then a running
    // maximum over the positions (thread i takes positions i*S .. i*S + S - 1)
    constexpr int kMaxPer = MAXP / kMidThreads;
    uint32_t* ent = reinterpret_cast<uint32_t*>(sval);
    for (uint32_t p = tid; p < P; p += kMidThreads) ent[p] = 0;
    __syncthreads();
    for (uint32_t e = tid; e < e1 - e0; e += kMidThreads) {
      const uint64_t a = ra.poff[e0 + e] - p0, b = ra.poff[e0 + e + 1] - p0;
      if (b > a) ent[a] = e;
    }
    __syncthreads();
    {
      const uint32_t S = P / kMidThreads;
      uint32_t run = 0;
      for (uint32_t i = 0; i < S; ++i) {
        const uint32_t x = ent[tid * S + i];
        run = x > run ? x : run;
      }
      const uint32_t incl = wave_inclusive_max(run);
      const int lane = lane_id(), wv = (int)(tid / kWave);
      if (lane == kWave - 1) wsum[wv] = incl;
      uint32_t before = (uint32_t)__shfl_up((int)incl, 1, kWave);
      if (lane == 0) before = 0;
      __syncthreads();
      for (int q = 0; q < wv; ++q) before = wsum[q] > before ? wsum[q] : before;
      run = before;
      for (uint32_t i = 0; i < S; ++i) {
        const uint32_t x = ent[tid * S + i];
        run = x > run ? x : run;
        ent[tid * S + i] = run;
      }
    }
    __syncthreads();
    uint32_t mine[kMaxPer];
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
      const uint32_t p = tid + (uint32_t)i * kMidThreads;
      mine[i] = p < P ? ent[p] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
      const uint32_t p = tid + (uint32_t)i * kMidThreads;
      if (p < P) {
        uint64_t key = ~0ull;
        double v = 0.0;
        if (p < f) mid_product_of(ra, e0 + mine[i], p0, row, p, pbits, key, v);
        skey[p] = key;
        sval[p] = v;
      }
    }
    __syncthreads();
    // Wave w owns pairs w*P/8 .. (w+1)*P/8 - 1, i.e. elements w*P/4 .. (w+1)*P/4 - 1
    // while j <= P/8: those stages need only the wave's own order; the few
    // with larger j are fenced by block barriers.
    {
      const uint32_t per_wave = P / 8, lane = (uint32_t)lane_id(), wv = tid / kWave;
      for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
          const bool wide = j > per_wave;
          if (wide) __syncthreads();
          for (uint32_t i = wv * per_wave + lane; i < (wv + 1) * per_wave; i += kWave) {
            const uint32_t lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
            const uint32_t hi = lo | j;
            const uint64_t a = skey[lo], b = skey[hi];
            if ((a > b) == ((lo & k) == 0)) {
              skey[lo] = b;
              skey[hi] = a;
            }
          }
          if (wide) __syncthreads();
          else wave_lds_sync();
        }
      }
      __syncthreads();
    }
    const uint64_t base = moff[li];
    uint64_t run = 0;
    for (uint32_t c0 = 0; c0 < (uint32_t)f; c0 += kMidThreads) {
      const uint32_t q = c0 + tid;
      const uint64_t col = q < f ? skey[q] >> pbits : 0;
      const bool head = q < f && (q == 0 || (skey[q - 1] >> pbits) != col);
      uint32_t total;
      const uint32_t ex = block_exclusive_scan<uint32_t>(head ? 1u : 0u, wsum, total);
      if (head) {
        double acc = 0.0;
        for (uint32_t t = q; t < (uint32_t)f && (skey[t] >> pbits) == col; ++t) acc += sval[skey[t] & (P - 1)];
        tmp_livs[base + run + ex] = col + ra.np * row;
        tmp_vals[base + run + ex] = acc;
      }
      run += total;
    }
    if (tid == 0) cnt[r] = run;
    __syncthreads();  // every run is summed before the next row is expanded
  }
}

// Moves each staged long row to its place in C (one wave per row; the rows
// are those of the bin lists, `n` apart, with counts c0, c1, c2).
__global__ void row_mid_copy_kernel(const uint32_t* __restrict__ list, const uint32_t* __restrict__ bins, uint32_t n,
                                    uint32_t c0, uint32_t c1, uint32_t c2, const uint64_t* __restrict__ moff,
                                    const uint64_t* __restrict__ coff, const uint64_t* __restrict__ tmp_livs,
                                    const double* __restrict__ tmp_vals, uint64_t* __restrict__ out_livs,
                                    double* __restrict__ out_vals) {
  const int lane = lane_id();
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  const uint32_t total = c0 + c1 + c2;
  for (uint32_t k = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; k < total; k += waves) {
    const uint32_t li = k < c0 ? bins[k] : k < c0 + c1 ? bins[n + (k - c0)] : bins[2 * (uint64_t)n + (k - c0 - c1)];
    const uint64_t src = moff[li];
    const uint32_t r = list[li];
    const uint64_t dst = coff[r], n = coff[r + 1] - dst;
    for (uint64_t q = lane; q < n; q += kWave) {
      out_livs[dst + q] = tmp_livs[src + q];
      out_vals[dst + q] = tmp_vals[src + q];
    }
  }
}

// Product counts of the long rows of the global path (g2) and of the in-LDS
// path (m2), each zero for the other path's rows; the in-LDS rows are also
// listed by size bin (at most kMidWaveMax, 1024 and kMidMax products: bin b's
// list positions at bins + b * n, its count in bin_cnt[b], cleared before).
// Whole waves step together (one list reservation per wave and bin).
constexpr int kMidBins = 3;
__device__ __forceinline__ int mid_bin(uint64_t f) {
  return f <= (uint64_t)kMidWaveMax ? 0 : f <= 1024 ? 1 : f <= (uint64_t)kMidMax ? 2 : -1;
}
__global__ void long_split_kernel(const uint64_t* __restrict__ f2, int64_t n, uint64_t* __restrict__ g2,
                                  uint64_t* __restrict__ m2, uint32_t* __restrict__ bins,
                                  unsigned long long* __restrict__ bin_cnt) {
  const int lane = lane_id();
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < n;
       i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + lane;
    int b = -1;
    if (i < n) {
      const uint64_t f = f2[i];
      b = mid_bin(f);
      g2[i] = b < 0 ? f : 0;
      m2[i] = b < 0 ? 0 : f;
    }
#pragma unroll
    for (int q = 0; q < kMidBins; ++q) {
      const uint64_t m = __ballot(b == q);
      if (!m) continue;
      unsigned long long base = 0;
      if (lane == __builtin_ctzll(m)) base = atomicAdd(&bin_cnt[q], (unsigned long long)__popcll(m));
      base = __shfl(base, __builtin_ctzll(m), kWave);
      if (b == q) bins[(int64_t)q * n + (int64_t)(base + __popcll(m & lanemask_lt()))] = (uint32_t)i;
    }
  }
}

int grid_for(lco_ctx ctx, int64_t n, int threads) {
  const int64_t want = (n + threads - 1) / threads;
  const int64_t cap = (int64_t)ctx->num_cus * 16;
  return (int)(want < 1 ? 1 : (want > cap ? cap : want));
}

}  // namespace

Segments segment_livs(lco_ctx ctx, Scratch& s, const uint64_t* livs, int64_t n, const FastDiv& div) {
  Segments sg;
  sg.count = s.get<uint64_t>(1);
  memset_async(ctx, sg.count, 0, sizeof(uint64_t));
  uint32_t* head = s.get<uint32_t>(n);
  uint32_t* pos = s.get<uint32_t>(n);
  sg.ids = s.get<uint64_t>(n);
  sg.starts = s.get<uint32_t>(n + 1);
  LCO_LAUNCH(ctx, "seg_heads", seg_heads_kernel, grid_for(ctx, n, 256), 256, 0, livs, n, div, head);
  scan_u32(ctx, head, pos, n, (uint32_t*)sg.count);
  LCO_LAUNCH(ctx, "seg_compact", seg_compact_kernel, grid_for(ctx, n, 256), 256, 0, livs, n, div, head, pos, sg.ids,
             sg.starts);
  return sg;
}

lco_tensor row_engine(lco_ctx ctx, const lco_tensor_s* A, const lco_tensor_s* B, uint64_t mp, uint64_t kp,
                      uint64_t np, bool dense, bool acc, int out_order, const uint64_t* out_dims) {
  const int64_t na = A->nnz, nb = B->nnz;
  Scratch s(ctx);
  RowArgs ra;
  ra.a_livs = A->livs;
  ra.a_vals = A->vals;
  ra.nnz_a = na;
  ra.b_livs = B->livs;
  ra.b_vals = B->vals;
  ra.nnz_b = nb;
  ra.kdiv = make_fastdiv(kp);
  ra.kp = kp;
  ra.np = np;
  const FastDiv ndiv = make_fastdiv(np);
  // the tiny and copy row classes pay for their launches only on large products
  const bool classes = na >= kClassMinEntries;
  const bool small = dense && na <= kSetupMaxEntries && nb <= kSetupMaxEntries && kp < kSetupMaxRowPtr;
  // rows of A' taken densely (all m' of them) when few are empty
  const bool dense_rows = !small && mp <= 2 * (uint64_t)na && mp < UINT32_MAX;
  const uint64_t rows_cap = dense_rows ? std::max<uint64_t>(mp, (uint64_t)na) : (uint64_t)na;
  uint32_t* len = s.get<uint32_t>(na);
  uint64_t* poff = s.get<uint64_t>(na + 1);
  uint32_t* bstart = s.get<uint32_t>(na);
  uint32_t* list2 = s.get<uint32_t>(rows_cap);
  uint64_t* f2 = s.get<uint64_t>(rows_cap);
  uint8_t* shape = s.get<uint8_t>(rows_cap);
  ra.bstart = bstart;
  ra.elen = len;
  const bool narrow = np < (1ull << 32);
  // rows per chunk: up to 64, but enough chunks for every resident wave (32 per compute unit)
  auto chunk_rows_for = [&](uint64_t rows) {
    const uint64_t resident = (uint64_t)ctx->num_cus * 32;
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(kChunkRows, rows / resident));
  };
  auto small_grid_for = [&](uint64_t rows, int chunk) {
    const uint64_t nchunks = (rows + chunk - 1) / chunk;
    return (int)std::max<uint64_t>(1, std::min<uint64_t>((nchunks + kRowWaves - 1) / kRowWaves,
                                                         (uint64_t)ctx->num_cus * 16));
  };
#define LCO_ROW_SMALL_N(GRID, NUM, NARROW, ...)                                                                  \
  do {                                                                                                           \
    if (acc)                                                                                                     \
      LCO_LAUNCH(ctx, NUM ? "row_small_num" : "row_small_sym", (row_chunk_kernel<true, NUM, NARROW>), GRID,       \
                 kRowThreads, 0, __VA_ARGS__);                                                                   \
    else                                                                                                         \
      LCO_LAUNCH(ctx, NUM ? "row_small_num" : "row_small_sym", (row_chunk_kernel<false, NUM, NARROW>), GRID,      \
                 kRowThreads, 0, __VA_ARGS__);                                                                   \
  } while (0)
#define LCO_ROW_SMALL(GRID, NUM, ...)                          \
  do {                                                         \
    if (narrow) LCO_ROW_SMALL_N(GRID, NUM, true, __VA_ARGS__); \
    else LCO_ROW_SMALL_N(GRID, NUM, false, __VA_ARGS__);       \
  } while (0)
  const uint64_t* h;
  // Small products: the symbolic pass of the one-wave rows and the scan of the
  // row counts follow the setup over at most nnz_A rows (the row count stays on
  // the device), so that one host synchronisation serves the setup and the
  // output size when there are no long rows.
  uint64_t* cnt = nullptr;
  uint64_t* coff = nullptr;
  bool counted = false;
  uint64_t counted_total = 0;
  if (small) {
    // rows of A', row pointers of B', entry lengths and row classes in one launch
    uint32_t* row_start = s.get<uint32_t>(na + 1);
    uint64_t* row_id = s.get<uint64_t>(na);
    uint64_t* words = s.get<uint64_t>(5);
    uint32_t* bptr = s.get<uint32_t>(kp + 1);
    ra.row_start = row_start;
    ra.row_id = row_id;
    ra.nzr_a = words;
    ra.bptr = bptr;
    cnt = s.get<uint64_t>(na + 1);
    coff = s.get<uint64_t>(na + 1);
    LCO_LAUNCH(ctx, "row_setup_small", row_setup_small_kernel, 1, kSetupThreads, 0, ra, ndiv, classes, row_start,
               row_id, words, bptr, len, bstart, list2, f2, shape, cnt);
    const int spec_chunk = chunk_rows_for((uint64_t)na);
    LCO_ROW_SMALL(small_grid_for((uint64_t)na, spec_chunk), false, ra, (uint32_t)na, spec_chunk,
                  (const uint8_t*)shape, cnt, (const uint64_t*)nullptr, (uint64_t*)nullptr, (double*)nullptr,
                  (const uint64_t*)words);
    scan_u64(ctx, cnt, coff, na, coff + na);
    const uint64_t* rb1[6] = {words, words + 1, words + 2, words + 3, words + 4, coff + na};
    h = readback(ctx, rb1, 6);
    counted = true;
    counted_total = h[5];
  } else {
    // compressed B'
    if (dense) {
      if (kp >= (uint64_t)1 << 34) fail(LCO_E_OOM, "contract: singly-compressed row pointer of more than 2^34 entries");
      uint32_t* bptr = s.get<uint32_t>(kp + 1);
      LCO_LAUNCH(ctx, "dense_ptr", dense_ptr_kernel, grid_for(ctx, nb + 1, 256), 256, 0, B->livs, nb, ndiv, kp,
                 bptr);
      ra.bptr = bptr;
    } else {
      // doubly compressed B': a hash table of its non-empty rows, at most two thirds full
      int logcap = 6;
      while (((uint64_t)1 << logcap) <= (uint64_t)nb + (uint64_t)nb / 2) ++logcap;
      const uint64_t cap = (uint64_t)1 << logcap;
      ulonglong2* tab = s.get<ulonglong2>(cap);
      LCO_LAUNCH(ctx, "dc_clear", dc_clear_kernel, grid_for(ctx, (int64_t)cap, 256), 256, 0, tab, cap);
      if (nb)
        LCO_LAUNCH(ctx, "dc_table", dc_table_kernel, grid_for(ctx, nb, 256), 256, 0, B->livs, nb, ndiv, tab,
                   64 - logcap, cap - 1);
      ra.dc_tab = tab;
      ra.dc_shift = 64 - logcap;
      ra.dc_mask = cap - 1;
    }
    // one block of words: long-row count; some row is tiny; a copy; of the one-wave kernel
    uint64_t* n2_dev = s.get<uint64_t>(4);
    uint64_t* flags_dev = n2_dev + 1;
    // rows of A' (all m' of them when few are empty, else the non-empty ones),
    // and the product count and B' row start of each A' entry
    const uint64_t* nzr_word;
    if (dense_rows) {
      uint32_t* row_start = s.get<uint32_t>(mp + 1);
      uint64_t* count = s.get<uint64_t>(1);
      if (dense)
        LCO_LAUNCH(ctx, "dense_rows_len", dense_rows_len_kernel<true>, grid_for(ctx, na + 1, 256), 256, 0, ra, mp,
                   row_start, count, len, bstart, n2_dev);
      else
        LCO_LAUNCH(ctx, "dense_rows_len", dense_rows_len_kernel<false>, grid_for(ctx, na + 1, 256), 256, 0, ra, mp,
                   row_start, count, len, bstart, n2_dev);
      ra.row_start = row_start;
      ra.row_id = nullptr;
      ra.nzr_a = count;
      nzr_word = count;
    } else {
      Segments arows = segment_livs(ctx, s, A->livs, na, ra.kdiv);
      ra.row_start = arows.starts;
      ra.row_id = arows.ids;
      ra.nzr_a = arows.count;
      nzr_word = arows.count;
      if (dense) LCO_LAUNCH(ctx, "entry_len", entry_len_kernel<true>, grid_for(ctx, na, 256), 256, 0, ra, len, bstart);
      else LCO_LAUNCH(ctx, "entry_len", entry_len_kernel<false>, grid_for(ctx, na, 256), 256, 0, ra, len, bstart);
      memset_async(ctx, n2_dev, 0, 4 * sizeof(uint64_t));
    }
    // row shapes; long rows collected with their product counts
    uint64_t* fl = s.get<uint64_t>(rows_cap);
    LCO_LAUNCH(ctx, "row_classify", row_classify_kernel, grid_for(ctx, (int64_t)rows_cap, kClassifyThreads),
               kClassifyThreads, 0, ra, (int64_t)rows_cap, classes, n2_dev, list2, f2, fl, shape,
               (uint32_t*)flags_dev, (uint32_t*)(flags_dev + 1), (uint32_t*)(flags_dev + 2));
    const uint64_t* rb1[5] = {nzr_word, n2_dev, flags_dev, flags_dev + 1, flags_dev + 2};
    h = readback(ctx, rb1, 5);
  }
  const uint64_t nzr = h[0], n2 = h[1];
  const bool tiny = h[2] != 0, copy = h[3] != 0, wave = h[4] != 0;
  const int tiny_grid = grid_for(ctx, (int64_t)nzr, 256);  // 64 rows per wave and sweep
  const int copy_grid = tiny_grid;  // 64 rows per wave and sweep as well
  uint64_t f2_total = 0, mid_total = 0;
  uint64_t* off2 = nullptr;
  uint64_t* moff = nullptr;
  uint64_t* bin_cnt = nullptr;
  uint32_t* bins = nullptr;
  uint64_t nbin[kMidBins] = {0, 0, 0};
  // long rows of at most kMidMax products are computed in LDS (their keys pack
  // the column and the product index into 63 bits); the rest take the global sort
  const int colbits = bits_for(np - 1);
  const bool mid = colbits + kMidBits <= 63;
  if (n2) {
    // the long-row paths locate products through the entries' product offsets
    scan_u32_u64(ctx, len, poff, na, poff + na);
    ra.poff = poff;
    off2 = s.get<uint64_t>(n2 + 1);
    moff = s.get<uint64_t>(n2 + 1);
    bin_cnt = s.get<uint64_t>(kMidBins);
    memset_async(ctx, bin_cnt, 0, kMidBins * sizeof(uint64_t));
    if (mid) {
      uint64_t* g2 = s.get<uint64_t>(n2);
      uint64_t* m2 = s.get<uint64_t>(n2);
      bins = s.get<uint32_t>((size_t)kMidBins * n2);
      LCO_LAUNCH(ctx, "long_split", long_split_kernel, grid_for(ctx, (int64_t)n2, 256), 256, 0, (const uint64_t*)f2,
                 (int64_t)n2, g2, m2, bins, (unsigned long long*)bin_cnt);
      scan_u64(ctx, g2, off2, (int64_t)n2, off2 + n2);
      scan_u64(ctx, m2, moff, (int64_t)n2, moff + n2);
    } else {
      scan_u64(ctx, f2, off2, (int64_t)n2, off2 + n2);
      memset_async(ctx, moff + n2, 0, sizeof(uint64_t));
    }
    const uint64_t* rb[5] = {off2 + n2, moff + n2, bin_cnt, bin_cnt + 1, bin_cnt + 2};
    const uint64_t* h2 = readback(ctx, rb, 5);
    f2_total = h2[0];
    mid_total = h2[1];
    for (int b = 0; b < kMidBins; ++b) nbin[b] = h2[2 + b];
  }
  // per-row output counts (already cleared and, for the one-wave rows, written on small products)
  if (!counted) {
    cnt = s.get<uint64_t>(nzr + 1);
    coff = s.get<uint64_t>(nzr + 1);
    if (!wave) memset_async(ctx, cnt, 0, (nzr + 1) * sizeof(uint64_t));  // else the one-wave kernel writes every count
  }
  const int chunk_rows = chunk_rows_for(nzr);
  const int small_grid = small_grid_for(nzr, chunk_rows);
  if (wave && !counted)
    LCO_ROW_SMALL(small_grid, false, ra, (uint32_t)nzr, chunk_rows, (const uint8_t*)shape, cnt,
                  (const uint64_t*)nullptr, (uint64_t*)nullptr, (double*)nullptr, (const uint64_t*)nullptr);
  if (tiny)
    LCO_LAUNCH(ctx, "row_tiny_sym", row_tiny_kernel<false>, tiny_grid, 256, 0, ra, (uint32_t)nzr,
               (const uint8_t*)shape, cnt, (const uint64_t*)nullptr, (uint64_t*)nullptr, (double*)nullptr);
  if (copy)
    LCO_LAUNCH(ctx, "row_copy_sym", row_copy_kernel<false>, tiny_grid, 256, 0, ra, (uint32_t)nzr,
               (const uint8_t*)shape, cnt, (const uint64_t*)nullptr, (uint64_t*)nullptr, (double*)nullptr);
  // long rows of the in-LDS path: computed now, staged, moved once placed
  uint64_t* mid_livs = nullptr;
  double* mid_vals = nullptr;
  auto cap_grid = [&](uint64_t want) { return (int)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)ctx->num_cus * 8)); };
  if (mid_total) {
    mid_livs = s.get<uint64_t>(mid_total);
    mid_vals = s.get<double>(mid_total);
    if (nbin[0])
      LCO_LAUNCH(ctx, "row_mid_wave", row_midw_kernel, cap_grid((nbin[0] + 3) / 4), kMidThreads, 0, ra, list2,
                 (const uint32_t*)bins, (uint32_t)nbin[0], (const uint64_t*)f2, (const uint64_t*)moff, cnt, mid_livs,
                 mid_vals);
    if (nbin[1])
      LCO_LAUNCH(ctx, "row_mid_1024", row_mid_kernel<1024>, cap_grid(nbin[1]), kMidThreads, 0, ra, list2,
                 (const uint32_t*)(bins + n2), (uint32_t)nbin[1], (const uint64_t*)f2, (const uint64_t*)moff, cnt,
                 mid_livs, mid_vals);
    if (nbin[2])
      LCO_LAUNCH(ctx, "row_mid_4096", row_mid_kernel<kMidMax>, cap_grid(nbin[2]), kMidThreads, 0, ra, list2,
                 (const uint32_t*)(bins + 2 * n2), (uint32_t)nbin[2], (const uint64_t*)f2, (const uint64_t*)moff, cnt,
                 mid_livs, mid_vals);
  }
  // other long rows: expand, sort by (row rank, column), count distinct
  uint64_t* keys = nullptr;
  double* pvals = nullptr;
  uint64_t colmask = 0;
  const int big_grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(n2, (uint64_t)ctx->num_cus * 8));
  if (f2_total) {
    const int qbits = bits_for(n2 - 1);
    if (colbits + qbits > 64) fail(LCO_E_UNSUPPORTED, "contract: long-row sort key exceeds 64 bits");
    colmask = colbits == 64 ? ~0ull : ((1ull << colbits) - 1);
    uint64_t* ek = s.get<uint64_t>(f2_total);
    double* ev = s.get<double>(f2_total);
    keys = s.get<uint64_t>(f2_total);
    pvals = s.get<double>(f2_total);
    LCO_LAUNCH(ctx, "big_expand", big_expand_kernel, big_grid, kBigThreads, 0, ra, list2, (uint32_t)n2, off2, colbits,
               ek, ev);
    KeyParams kparams;
    radix_sort_pairs(ctx, ek, ev, keys, pvals, (int64_t)f2_total, nullptr, kparams, colbits + qbits, 0);
    LCO_LAUNCH(ctx, "big_reduce_sym", big_reduce_kernel<false>, big_grid, kBigThreads, 0, ra, list2, (uint32_t)n2,
               off2, (const uint64_t*)keys, (const double*)pvals, colmask, cnt, (const uint64_t*)nullptr,
               (uint64_t*)nullptr, (double*)nullptr);
  }
  uint64_t nnz_c = counted_total;
  if (!counted || n2 || tiny || copy) {  // counts written after the first scan: scan again
    scan_u64(ctx, cnt, coff, nzr, coff + nzr);
    const uint64_t* rb2[1] = {coff + nzr};
    nnz_c = readback(ctx, rb2, 1)[0];
  }
  if (nnz_c > UINT32_MAX) fail(LCO_E_UNSUPPORTED, "contract: more than 2^32-1 output entries");
  lco_tensor C = new_tensor(ctx, out_order, out_dims, (int64_t)nnz_c);
  try {
    if (wave)
      LCO_ROW_SMALL(small_grid, true, ra, (uint32_t)nzr, chunk_rows, (const uint8_t*)shape, (uint64_t*)nullptr,
                    (const uint64_t*)coff, C->livs, C->vals, (const uint64_t*)nullptr);
    if (tiny)
      LCO_LAUNCH(ctx, "row_tiny_num", row_tiny_kernel<true>, tiny_grid, 256, 0, ra, (uint32_t)nzr,
                 (const uint8_t*)shape, (uint64_t*)nullptr, (const uint64_t*)coff, C->livs, C->vals);
    if (copy)
      LCO_LAUNCH(ctx, "row_copy_num", row_copy_kernel<true>, copy_grid, 256, 0, ra, (uint32_t)nzr,
                 (const uint8_t*)shape, (uint64_t*)nullptr, (const uint64_t*)coff, C->livs, C->vals);
    if (mid_total)
      LCO_LAUNCH(ctx, "row_mid_copy", row_mid_copy_kernel, cap_grid((nbin[0] + nbin[1] + nbin[2] + 3) / 4), 256, 0,
                 (const uint32_t*)list2, (const uint32_t*)bins, (uint32_t)n2, (uint32_t)nbin[0], (uint32_t)nbin[1],
                 (uint32_t)nbin[2], (const uint64_t*)moff, (const uint64_t*)coff, (const uint64_t*)mid_livs,
                 (const double*)mid_vals, C->livs, C->vals);
    if (f2_total)
      LCO_LAUNCH(ctx, "big_reduce_num", big_reduce_kernel<true>, big_grid, kBigThreads, 0, ra, list2, (uint32_t)n2,
                 off2, (const uint64_t*)keys, (const double*)pvals, colmask, (uint64_t*)nullptr,
                 (const uint64_t*)coff, C->livs, C->vals);
  } catch (...) {
    lco_destroy(C);
    throw;
  }
#undef LCO_ROW_SMALL
#undef LCO_ROW_SMALL_N
  return C;
}

}  // namespace lco
