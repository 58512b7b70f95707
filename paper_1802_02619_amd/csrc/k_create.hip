// Construction of LCO tensors (Section 3.1): coordinates -> LIVs, validation,
// full-key sort, and summation of duplicate LIVs.
#include "device_common.h"

namespace lco {

namespace {

struct DimsParam {
  int order;
  uint64_t dims[kMaxOrder];
};

// LIV = c0 + n0*(c1 + n1*(c2 + ...)); flags out-of-range coordinates in *err.
__global__ void coords_to_liv_kernel(const uint64_t* __restrict__ coords, int64_t n, DimsParam dp,
                                     uint64_t* __restrict__ livs, uint32_t* __restrict__ err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t* c = coords + i * dp.order;
    uint64_t liv = 0;
    bool bad = false;
    for (int r = dp.order - 1; r >= 0; --r) {
      const uint64_t x = c[r];
      bad |= x >= dp.dims[r];
      liv = liv * dp.dims[r] + x;
    }
    if (bad) atomicOr(err, 1u);
    livs[i] = liv;
  }
}

// LIVs supplied directly: copy and flag values >= max_liv+1 (err bit 1) and,
// when `need_sorted`, any non-increasing neighbour pair (err bit 2).
__global__ void check_livs_kernel(const uint64_t* __restrict__ in, int64_t n, uint64_t max_liv, int need_sorted,
                                  uint32_t* __restrict__ err) {
  uint32_t e = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t x = in[i];
    if (x > max_liv) e |= 1u;
    if (need_sorted && i > 0 && in[i - 1] >= x) e |= 2u;
  }
  if (e) atomicOr(err, e);
}

// head[i] = 1 where a new LIV starts in sorted order.
__global__ void mark_heads_kernel(const uint64_t* __restrict__ livs, int64_t n, uint32_t* __restrict__ head) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (i == 0 || livs[i] != livs[i - 1]) ? 1u : 0u;
}

// Each run head sums its run left to right (the stable sort kept input order),
// starting from the first value, and writes to its compacted position.
__global__ void reduce_runs_kernel(const uint64_t* __restrict__ livs, const double* __restrict__ vals, int64_t n,
                                   const uint32_t* __restrict__ head, const uint32_t* __restrict__ pos,
                                   uint64_t* __restrict__ out_livs, double* __restrict__ out_vals) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!head[i]) continue;
    const uint64_t key = livs[i];
    double acc = vals[i];
    for (int64_t j = i + 1; j < n && livs[j] == key; ++j) acc += vals[j];
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

// Builds the storage of `t` (allocated by the caller for `n` entries).  Returns
// the number of distinct entries and throws on invalid input.  On return with
// fewer entries than n the caller shrinks the tensor.
int64_t create_storage(lco_ctx ctx, lco_tensor t, const uint64_t* d_idx, const double* d_vals, int64_t n,
                       uint32_t flags, int full_bits, uint64_t max_liv, uint64_t** out_livs, double** out_vals,
                       void** out_base, size_t* out_bytes) {
  Scratch s(ctx);
  uint64_t* words = s.get<uint64_t>(2);  // [0]: error flags, [1]: distinct count
  memset_async(ctx, words, 0, 2 * sizeof(uint64_t));
  uint32_t* err = (uint32_t*)words;
  const bool coords = flags & LCO_COORDS;
  const bool sorted = flags & LCO_SORTED;
  uint64_t* livs = s.get<uint64_t>(n);
  if (coords) {
    DimsParam dp;
    dp.order = t->order;
    for (int r = 0; r < t->order; ++r) dp.dims[r] = t->dims[r];
    LCO_LAUNCH(ctx, "coords_to_liv", coords_to_liv_kernel, grid_for(ctx, n, 256), 256, 0, d_idx, n, dp, livs, err);
    if (sorted)
      LCO_LAUNCH(ctx, "check_livs", check_livs_kernel, grid_for(ctx, n, 256), 256, 0, livs, n, max_liv, 1, err);
  } else {
    LCO_LAUNCH(ctx, "check_livs", check_livs_kernel, grid_for(ctx, n, 256), 256, 0, d_idx, n, max_liv,
               sorted ? 1 : 0, err);
  }
  const uint64_t* src_livs = coords ? livs : d_idx;
  // sort (stable, full key) unless the input claims to be sorted
  uint64_t* sl = t->livs;
  double* sv = t->vals;
  if (!sorted) {
    KeyParams kp;
    radix_sort_pairs(ctx, src_livs, d_vals, sl, sv, n, nullptr, kp, full_bits, 0);
  } else {
    copy_d2d(ctx, sl, src_livs, n * sizeof(uint64_t));
    copy_d2d(ctx, sv, d_vals, n * sizeof(double));
  }
  // distinct count
  uint32_t* head = s.get<uint32_t>(n);
  uint32_t* pos = s.get<uint32_t>(n);
  LCO_LAUNCH(ctx, "mark_heads", mark_heads_kernel, grid_for(ctx, n, 256), 256, 0, sl, n, head);
  scan_u32(ctx, head, pos, n, (uint32_t*)(words + 1));
  const uint64_t* rb[2] = {words, words + 1};
  const uint64_t* r = readback(ctx, rb, 2);
  const uint64_t e = r[0] & 0xffffffffull;
  const int64_t distinct = (int64_t)(r[1] & 0xffffffffull);
  if (e & 1u) fail(LCO_E_ARG, coords ? "create: coordinate out of range" : "create: LIV out of range");
  if (e & 2u) fail(LCO_E_UNSORTED, "create: LCO_SORTED input is not strictly increasing");
  if (distinct == n) return n;
  if (!(flags & LCO_SUM_DUPLICATES)) fail(LCO_E_DUPLICATE, "create: repeated coordinate");
  // compact into a new allocation of the exact size
  const size_t bytes = (size_t)distinct * 16;
  char* base = (char*)dev_alloc(ctx, bytes);
  uint64_t* ol = (uint64_t*)base;
  double* ov = (double*)(base + (size_t)distinct * 8);
  LCO_LAUNCH(ctx, "reduce_runs", reduce_runs_kernel, grid_for(ctx, n, 256), 256, 0, sl, sv, n, head, pos, ol, ov);
  *out_livs = ol;
  *out_vals = ov;
  *out_base = base;
  *out_bytes = bytes;
  return distinct;
}

}  // namespace lco
