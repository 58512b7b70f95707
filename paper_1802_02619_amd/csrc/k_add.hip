// Sparse addition of two LCO tensors held in the same lexicographical order.
//
// Section 2 builds its design tensor as a sum of two products; Section 3.2
// notes that before the two terms can be added one of them must be re-sorted
// into the other's order.  Once both operands are sorted alike, the sum is a
// merge of two strictly increasing LIV lists: an LIV present in both operands
// gives alpha*a + beta*b, an LIV present in one gives that operand's scaled
// value, and the pattern is the union of the two patterns.
//
// GPU form: the merged sequence (na + nb entries, ties ordered a before b) is
// cut into equal tiles by a merge-path search on the diagonals, so every tile
// reads one contiguous range of each operand.  A tile is staged in LDS with
// coalesced loads and merged there, each thread walking eight consecutive
// positions of the merge.  Because ties put a first, an LIV present in both
// operands shows up as a's entry immediately followed by b's: b's copy is
// dropped and its value joins a's.  A first pass counts each tile's outputs; a
// scan gives the tile offsets; the second pass writes the tile's outputs back
// through LDS with coalesced stores.
#include "device_common.h"

namespace lco {

namespace {

constexpr int kAddThreads = 256;
constexpr int kAddItems = 8;
constexpr int kAddTile = kAddThreads * kAddItems;

// Number of entries of a among the first d entries of the merge of a (na
// entries) and b (nb entries), ties ordered a first.
template <class I, class KA, class KB>
__device__ __forceinline__ I merge_path(const KA& akey, I na, const KB& bkey, I nb, I d) {
  I lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const I mid = (lo + hi) >> 1;
    if (akey(mid) <= bkey(d - 1 - mid)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void add_partition_kernel(const uint64_t* __restrict__ a, int64_t na, const uint64_t* __restrict__ b,
                                     int64_t nb, int64_t tiles, int64_t* __restrict__ split) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > tiles) return;
  const int64_t total = na + nb;
  const int64_t d = t * kAddTile < total ? t * kAddTile : total;
  split[t] = merge_path<int64_t>([&](int64_t i) { return a[i]; }, na, [&](int64_t j) { return b[j]; }, nb, d);
}

// One tile of the merge: a[a0, a0 + la) and b[b0, b0 + lb).
struct AddTile {
  int64_t a0, b0;
  int la, lb;
  bool prev_a;  // a[a0 - 1] exists: it may equal b[b0]
  bool next_b;  // b[b0 + lb] exists: it may equal a[a0 + la - 1]
};

__device__ __forceinline__ AddTile tile_of(const int64_t* split, int64_t na, int64_t nb) {
  const int64_t t = blockIdx.x;
  const int64_t total = na + nb;
  const int64_t d0 = t * kAddTile;
  const int64_t d1 = d0 + kAddTile < total ? d0 + kAddTile : total;
  AddTile T;
  T.a0 = split[t];
  const int64_t a1 = split[t + 1];
  T.b0 = d0 - T.a0;
  T.la = (int)(a1 - T.a0);
  T.lb = (int)((d1 - a1) - T.b0);
  T.prev_a = T.a0 > 0;
  T.next_b = T.b0 + T.lb < nb;
  return T;
}

// Stages the tile's keys (and values) in LDS: sk[0] = a[a0 - 1], sk[1 .. 1+la)
// = a's keys, then lb keys of b, then b[b0 + lb]; sv has the same layout.
template <bool VALS>
__device__ __forceinline__ void stage_tile(const AddTile& T, const uint64_t* __restrict__ a,
                                           const double* __restrict__ av, const uint64_t* __restrict__ b,
                                           const double* __restrict__ bv, uint64_t* sk, double* sv) {
  const int n = T.la + T.lb;
  for (int q = threadIdx.x; q < n; q += kAddThreads) {
    if (q < T.la) {
      sk[1 + q] = a[T.a0 + q];
      if (VALS) sv[1 + q] = av[T.a0 + q];
    } else {
      sk[1 + q] = b[T.b0 + (q - T.la)];
      if (VALS) sv[1 + q] = bv[T.b0 + (q - T.la)];
    }
  }
  if (threadIdx.x == 0 && T.prev_a) sk[0] = a[T.a0 - 1];
  if (threadIdx.x == kWave && T.next_b) {
    sk[1 + n] = b[T.b0 + T.lb];
    if (VALS) sv[1 + n] = bv[T.b0 + T.lb];
  }
  __syncthreads();
}

// This thread's share of the tile's merge: positions [diag, end).
struct ThreadRange {
  int diag, end, i, j;  // i, j: entries of a and b before position diag
};

__device__ __forceinline__ ThreadRange thread_range(const AddTile& T, const uint64_t* sa, const uint64_t* sb) {
  const int n = T.la + T.lb;
  ThreadRange r;
  r.diag = (int)threadIdx.x * kAddItems < n ? (int)threadIdx.x * kAddItems : n;
  r.end = r.diag + kAddItems < n ? r.diag + kAddItems : n;
  r.i = merge_path<int>([&](int i) { return sa[i]; }, T.la, [&](int j) { return sb[j]; }, T.lb, r.diag);
  r.j = r.diag - r.i;
  return r;
}

__global__ __launch_bounds__(kAddThreads) void add_count_kernel(const uint64_t* __restrict__ a, int64_t na,
                                                                const uint64_t* __restrict__ b, int64_t nb,
                                                                const int64_t* __restrict__ split,
                                                                uint64_t* __restrict__ cnt) {
  __shared__ uint64_t sk[kAddTile + 2];
  __shared__ uint32_t wsum[kAddThreads / kWave];
  const AddTile T = tile_of(split, na, nb);
  stage_tile<false>(T, a, nullptr, b, nullptr, sk, nullptr);
  const uint64_t* sa = sk + 1;         // sa[-1] is a[a0 - 1]
  const uint64_t* sb = sk + 1 + T.la;  // sb[lb] is b[b0 + lb]
  ThreadRange r = thread_range(T, sa, sb);
  uint32_t c = 0;
  int i = r.i, j = r.j;
#pragma unroll
  for (int k = 0; k < kAddItems; ++k) {
    if (r.diag + k < r.end) {
      if (i < T.la && (j >= T.lb || sa[i] <= sb[j])) {
        ++i;
        ++c;
      } else {
        const bool dup = (i > 0 || T.prev_a) && sa[i - 1] == sb[j];
        c += dup ? 0u : 1u;
        ++j;
      }
    }
  }
  c = wave_reduce_sum(c);
  if (lane_id() == 0) wsum[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t s = 0;
    for (int w = 0; w < kAddThreads / kWave; ++w) s += wsum[w];
    cnt[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kAddThreads) void add_write_kernel(
    const uint64_t* __restrict__ a, const double* __restrict__ av, int64_t na, const uint64_t* __restrict__ b,
    const double* __restrict__ bv, int64_t nb, const int64_t* __restrict__ split, const uint64_t* __restrict__ off,
    double alpha, double beta, uint64_t* __restrict__ out_livs, double* __restrict__ out_vals) {
  __shared__ uint64_t sk[kAddTile + 2];
  __shared__ double sv[kAddTile + 2];
  __shared__ uint32_t wsum[kAddThreads / kWave + 1];
  const AddTile T = tile_of(split, na, nb);
  stage_tile<true>(T, a, av, b, bv, sk, sv);
  const uint64_t* sa = sk + 1;
  const uint64_t* sb = sk + 1 + T.la;
  const double* sva = sv + 1;
  const double* svb = sv + 1 + T.la;
  ThreadRange r = thread_range(T, sa, sb);
  uint64_t ok[kAddItems];
  double ov[kAddItems];
  bool have[kAddItems];
  uint32_t c = 0;
  int i = r.i, j = r.j;
#pragma unroll
  for (int k = 0; k < kAddItems; ++k) {
    have[k] = false;
    ok[k] = 0;
    ov[k] = 0.0;
    if (r.diag + k < r.end) {
      if (i < T.la && (j >= T.lb || sa[i] <= sb[j])) {
        // an entry of a; b's entry with the same LIV, if any, is next in b
        const uint64_t key = sa[i];
        double v = alpha * sva[i];
        if ((j < T.lb || T.next_b) && sb[j] == key) v = v + beta * svb[j];
        ok[k] = key;
        ov[k] = v;
        have[k] = true;
        ++i;
      } else {
        // an entry of b, dropped when a holds the same LIV (then it is a's previous entry)
        const bool dup = (i > 0 || T.prev_a) && sa[i - 1] == sb[j];
        if (!dup) {
          ok[k] = sb[j];
          ov[k] = beta * svb[j];
          have[k] = true;
        }
        ++j;
      }
      c += have[k] ? 1u : 0u;
    }
  }
  uint32_t total;
  uint32_t o = block_exclusive_scan(c, wsum, total);  // ends with a barrier: the staged tile may be overwritten
#pragma unroll
  for (int k = 0; k < kAddItems; ++k) {
    if (have[k]) {
      sk[o] = ok[k];
      sv[o] = ov[k];
      ++o;
    }
  }
  __syncthreads();
  const uint64_t base = off[blockIdx.x];
  for (uint32_t q = threadIdx.x; q < total; q += kAddThreads) {
    out_livs[base + q] = sk[q];
    out_vals[base + q] = sv[q];
  }
}

}  // namespace

lco_tensor add_merge(lco_ctx ctx, double alpha, const lco_tensor_s* a, double beta, const lco_tensor_s* b, int order,
                     const uint64_t* dims) {
  const int64_t na = a->nnz, nb = b->nnz, total = na + nb;
  if (total == 0) return new_tensor(ctx, order, dims, 0);
  if (total > (int64_t)UINT32_MAX) fail(LCO_E_UNSUPPORTED, "add: more than 2^32-1 entries in the two operands");
  const int64_t tiles = (total + kAddTile - 1) / kAddTile;
  Scratch sc(ctx);
  int64_t* split = sc.get<int64_t>(tiles + 1);
  uint64_t* cnt = sc.get<uint64_t>(tiles);
  uint64_t* off = sc.get<uint64_t>(tiles + 1);
  LCO_LAUNCH(ctx, "add_partition", add_partition_kernel, (unsigned)((tiles + 1 + 255) / 256), 256, 0,
             (const uint64_t*)a->livs, na, (const uint64_t*)b->livs, nb, tiles, split);
  LCO_LAUNCH(ctx, "add_count", add_count_kernel, (unsigned)tiles, kAddThreads, 0, (const uint64_t*)a->livs, na,
             (const uint64_t*)b->livs, nb, (const int64_t*)split, cnt);
  scan_u64(ctx, cnt, off, tiles, off + tiles);
  const uint64_t* rb[1] = {off + tiles};
  const uint64_t nnz_c = readback(ctx, rb, 1)[0];
  lco_tensor C = new_tensor(ctx, order, dims, (int64_t)nnz_c);
  try {
    LCO_LAUNCH(ctx, "add_write", add_write_kernel, (unsigned)tiles, kAddThreads, 0, (const uint64_t*)a->livs,
               (const double*)a->vals, na, (const uint64_t*)b->livs, (const double*)b->vals, nb,
               (const int64_t*)split, (const uint64_t*)off, alpha, beta, C->livs, C->vals);
  } catch (...) {
    lco_destroy(C);
    throw;
  }
  return C;
}

}  // namespace lco
