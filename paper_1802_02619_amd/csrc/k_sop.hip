// Simple outer product, SOP (Section 5.2.5): every rank-1 product of a column
// of A with the matching row of B is written into one list of length f, the
// list is sorted by output LIV (stable, so equal LIVs keep the order of the
// contracted index) and equal LIVs are summed.
//
// A is column-major (LIV = i + m*l), B row-major (LIV = j + n*l).  The
// non-empty columns of A and rows of B are found by segmenting the sorted
// LIVs; a join gives, for each non-empty column l of A with a matching row of
// B, a block of cntA(l)*cntB(l) products; a scan of block sizes places the
// blocks; the expansion is load-balanced over tiles of products.
#include <algorithm>
#include <cstring>

#include "device_common.h"
#include "rows.h"

namespace lco {

namespace {

struct SopArgs {
  const uint64_t* a_livs;
  const double* a_vals;
  const uint64_t* b_livs;
  const double* b_vals;
  uint64_t m, n;
  const uint64_t* acol_id;
  const uint32_t* acol_start;
  const uint64_t* nzc_a;
  const uint64_t* brow_id;
  const uint32_t* brow_start;
  const uint64_t* nzr_b;
  const uint2* bseg;  // per join block: first entry and length of the matching B row
  const uint64_t* boff;
  int simple;  // output LIV = i + m*j
  int nfa, nfb;
  FastDiv fa_div[kMaxOrder];
  uint64_t fa_w[kMaxOrder];
  FastDiv fb_div[kMaxOrder];
  uint64_t fb_w[kMaxOrder];
};

constexpr int kSopThreads = 256;
constexpr int kSopTile = 4096;  // products per tile

__global__ void sop_join_kernel(SopArgs sa, int64_t upper, uint64_t* __restrict__ blk, uint2* __restrict__ bseg) {
  const uint64_t nzc = *sa.nzc_a, nzr = *sa.nzr_b;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < upper; c += (int64_t)gridDim.x * blockDim.x) {
    if ((uint64_t)c >= nzc) break;
    const uint64_t l = sa.acol_id[c];
    uint64_t lo = 0, hi = nzr;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (sa.brow_id[mid] < l) lo = mid + 1;
      else hi = mid;
    }
    uint64_t b = 0;
    uint2 seg = make_uint2(0u, 0u);
    if (lo < nzr && sa.brow_id[lo] == l) {
      const uint64_t ca = sa.acol_start[c + 1] - sa.acol_start[c];
      seg = make_uint2(sa.brow_start[lo], sa.brow_start[lo + 1] - sa.brow_start[lo]);
      b = ca * seg.y;
    }
    blk[c] = b;
    bseg[c] = seg;
  }
}

__device__ __forceinline__ uint64_t relinearise(const FastDiv* div, const uint64_t* w, int nf, uint64_t x) {
  uint64_t key = 0;
  for (int t = 0; t + 1 < nf; ++t) {
    uint64_t c;
    x = fd_divmod(div[t], x, c);
    key += c * w[t];
  }
  if (nf > 0) key += x * w[nf - 1];
  return key;
}

// Products are expanded in tiles of kSopTile consecutive list positions.  Each
// product needs its block c (the last non-empty block starting at or before
// it): every non-empty block that starts inside the tile marks its first
// position with its index relative to the tile's first block, and a running
// maximum over the tile hands every position its block.  (Each wave scans a
// quarter of the tile; the maxima of the quarters before it are added when a
// position is read.)
constexpr int kSopWaves = kSopThreads / kWave;
constexpr int kSopQuarter = kSopTile / kSopWaves;  // positions scanned by one wave
static_assert(kSopWaves == 4, "the running maximum is combined over four quarters");


__global__ __launch_bounds__(kSopThreads) void sop_expand_kernel(SopArgs sa, uint64_t f, uint64_t* __restrict__ keys,
                                                                 double* __restrict__ vals) {
  __shared__ uint32_t s_blk[kSopTile];     // block of each position, relative to c0
  __shared__ uint32_t s_pre[kSopWaves];    // largest block index of the quarters before each quarter
  __shared__ uint64_t s_c[2];
  const uint64_t nzc = *sa.nzc_a;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const uint64_t tiles = (f + kSopTile - 1) / kSopTile;
  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const uint64_t p0 = tile * kSopTile;
    const uint64_t p1 = (p0 + kSopTile < f ? p0 + kSopTile : f) - 1;
    if (threadIdx.x < 2) {
      // last block c with boff[c] <= target
      const uint64_t target = threadIdx.x == 0 ? p0 : p1;
      uint64_t lo = 0, hi = nzc - 1;
      while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (sa.boff[mid] <= target) lo = mid;
        else hi = mid - 1;
      }
      s_c[threadIdx.x] = lo;
    }
    for (int i = threadIdx.x; i < kSopTile; i += kSopThreads) s_blk[i] = 0;
    __syncthreads();
    const uint64_t c0 = s_c[0], c1 = s_c[1];
    // blocks c0+1..c1 start inside the tile (at p0+1..p1); empty ones share the
    // start of the next non-empty block and mark nothing
    for (uint64_t c = c0 + 1 + threadIdx.x; c <= c1; c += kSopThreads) {
      const uint64_t b = sa.boff[c];
      if (b < sa.boff[c + 1]) s_blk[b - p0] = (uint32_t)(c - c0);
    }
    __syncthreads();
    uint32_t carry = 0;
    for (int k = 0; k < kSopQuarter; k += kWave) {
      const int q = w * kSopQuarter + k + lane;
      uint32_t x = s_blk[q];
      x = wave_inclusive_max(x > carry ? x : carry);
      s_blk[q] = x;
      carry = __shfl(x, kWave - 1, kWave);
    }
    if (lane == 0) s_pre[w] = carry;
    __syncthreads();
    const uint32_t pre1 = s_pre[0], pre2 = s_pre[1] > pre1 ? s_pre[1] : pre1, pre3 = s_pre[2] > pre2 ? s_pre[2] : pre2;
    const uint32_t span = (uint32_t)(p1 - p0);
    for (uint32_t q = threadIdx.x; q <= span; q += kSopThreads) {
      const uint32_t qv = q / kSopQuarter;
      const uint32_t pre = qv == 0 ? 0u : (qv == 1 ? pre1 : (qv == 2 ? pre2 : pre3));
      const uint32_t lb = s_blk[q] > pre ? s_blk[q] : pre;
      const uint64_t c = c0 + lb;
      const uint64_t p = p0 + q;
      const uint64_t local = p - sa.boff[c];
      const uint2 seg = sa.bseg[c];
      const uint32_t bstart = seg.x;
      const uint64_t cb = seg.y;
      uint64_t ia, ib;
      if (local < (1ull << 32)) {
        ia = (uint32_t)local / (uint32_t)cb;
        ib = (uint32_t)local - (uint32_t)ia * (uint32_t)cb;
      } else {
        ia = local / cb;
        ib = local - ia * cb;
      }
      const uint32_t ea = sa.acol_start[c] + (uint32_t)ia;
      const uint32_t eb = bstart + (uint32_t)ib;
      const uint64_t l = sa.acol_id[c];
      const uint64_t i = sa.a_livs[ea] - sa.m * l;
      const uint64_t j = sa.b_livs[eb] - sa.n * l;
      uint64_t key;
      if (sa.simple) key = i + sa.m * j;
      else key = relinearise(sa.fa_div, sa.fa_w, sa.nfa, i) + relinearise(sa.fb_div, sa.fb_w, sa.nfb, j);
      keys[p] = key;
      vals[p] = sa.a_vals[ea] * sa.b_vals[eb];
    }
    __syncthreads();
  }
}

__global__ void key_heads_kernel(const uint64_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ head) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// Each run head sums its run left to right starting from 0.0.
__global__ void sum_runs_kernel(const uint64_t* __restrict__ keys, const double* __restrict__ vals, int64_t n,
                                const uint32_t* __restrict__ head, const uint32_t* __restrict__ pos,
                                uint64_t* __restrict__ out_livs, double* __restrict__ out_vals) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!head[i]) continue;
    const uint64_t key = keys[i];
    double acc = 0.0;
    for (int64_t j = i; j < n && keys[j] == key; ++j) acc += vals[j];
    out_livs[pos[i]] = key;
    out_vals[pos[i]] = acc;
  }
}

int grid_for(lco_ctx ctx, int64_t n, int threads) {
  const int64_t want = (n + threads - 1) / threads;
  const int64_t cap = (int64_t)ctx->num_cus * 16;
  return (int)(want < 1 ? 1 : (want > cap ? cap : want));
}

}  // namespace

lco_tensor sop_engine(lco_ctx ctx, const lco_tensor_s* A, const lco_tensor_s* B, const ContractDetail& d) {
  const int64_t na = A->nnz, nb = B->nnz;
  const uint64_t m = d.em, n = d.en;  // A' is m (free and entrywise) by k, B' is k by n (free)
  Scratch s(ctx);
  SopArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.a_livs = A->livs;
  sa.a_vals = A->vals;
  sa.b_livs = B->livs;
  sa.b_vals = B->vals;
  sa.m = m;
  sa.n = n;
  Segments acols = segment_livs(ctx, s, A->livs, na, make_fastdiv(m));
  Segments brows = segment_livs(ctx, s, B->livs, nb, make_fastdiv(n));
  sa.acol_id = acols.ids;
  sa.acol_start = acols.starts;
  sa.nzc_a = acols.count;
  sa.brow_id = brows.ids;
  sa.brow_start = brows.starts;
  sa.nzr_b = brows.count;
  uint64_t* blk = s.get<uint64_t>(na);
  uint2* bseg = s.get<uint2>(na);
  uint64_t* boff = s.get<uint64_t>(na + 1);
  memset_async(ctx, blk, 0, na * sizeof(uint64_t));
  LCO_LAUNCH(ctx, "sop_join", sop_join_kernel, grid_for(ctx, na, 256), 256, 0, sa, na, blk, bseg);
  scan_u64(ctx, blk, boff, na, boff + na);
  sa.bseg = bseg;
  sa.boff = boff;
  const uint64_t* rb[1] = {boff + na};
  const uint64_t f = readback(ctx, rb, 1)[0];
  if (f == 0) return new_tensor(ctx, d.order_c, d.c_dims, 0);
  if (f > UINT32_MAX) fail(LCO_E_UNSUPPORTED, "contract: outer-product list longer than 2^32-1");
  sa.simple = d.sop_simple_key ? 1 : 0;
  sa.nfa = d.n_free_a;
  sa.nfb = d.n_free_b;
  for (int t = 0; t < d.n_free_a; ++t) {
    sa.fa_div[t] = make_fastdiv(d.free_a_dims[t]);
    sa.fa_w[t] = d.free_a_cweight[t];
  }
  for (int t = 0; t < d.n_free_b; ++t) {
    sa.fb_div[t] = make_fastdiv(d.free_b_dims[t]);
    sa.fb_w[t] = d.free_b_cweight[t];
  }
  uint64_t* ek = s.get<uint64_t>(f);
  double* ev = s.get<double>(f);
  const uint64_t tiles = (f + kSopTile - 1) / kSopTile;
  const int eg = (int)std::max<uint64_t>(1, std::min<uint64_t>(tiles, (uint64_t)ctx->num_cus * 8));
  LCO_LAUNCH(ctx, "sop_expand", sop_expand_kernel, eg, kSopThreads, 0, sa, f, ek, ev);
  // sort by output LIV
  unsigned __int128 total = 1;
  for (int r = 0; r < d.order_c; ++r) total *= d.c_dims[r];
  const unsigned __int128 mx = total - 1;
  const int bits = (uint64_t)(mx >> 64) ? 64 : bits_for((uint64_t)mx);
  uint64_t* sk = s.get<uint64_t>(f);
  double* sv = s.get<double>(f);
  KeyParams kp;
  radix_sort_pairs(ctx, ek, ev, sk, sv, (int64_t)f, nullptr, kp, bits, 0);
  uint32_t* head = s.get<uint32_t>(f);
  uint32_t* pos = s.get<uint32_t>(f);
  uint64_t* word = s.get<uint64_t>(1);
  memset_async(ctx, word, 0, sizeof(uint64_t));
  LCO_LAUNCH(ctx, "key_heads", key_heads_kernel, grid_for(ctx, f, 256), 256, 0, sk, (int64_t)f, head);
  scan_u32(ctx, head, pos, (int64_t)f, (uint32_t*)word);
  const uint64_t* rb2[1] = {word};
  const uint64_t nnz_c = readback(ctx, rb2, 1)[0];
  lco_tensor C = new_tensor(ctx, d.order_c, d.c_dims, (int64_t)nnz_c);
  LCO_LAUNCH(ctx, "sum_runs", sum_runs_kernel, grid_for(ctx, f, 256), 256, 0, sk, sv, (int64_t)f, head, pos,
             C->livs, C->vals);
  return C;
}

}  // namespace lco
