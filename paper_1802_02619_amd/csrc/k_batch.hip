// Batched contraction: many independent products run as one sequence of
// launches.  Every instance that the per-call path would run through the
// one-wave-per-row engine (row- or column-wise, singly compressed B', every
// row of A' with at most 64 products and entries) is processed together: each
// phase -- row pointers of B', rows of A', products per entry, row shapes, the
// symbolic count, the numeric product -- is a single launch over the
// concatenated entries and rows of all instances, and the whole batch needs
// two host synchronisations (the batch's row count, then its output size).
// Rows are computed by the same device code as the per-call path, so each
// result is bit-identical to the per-call result.  Instances outside that case
// (doubly compressed, outer product, long rows) run through the per-call path.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "row_core.h"

namespace lco {

namespace {

struct BInst {
  const uint64_t* a_livs;
  const double* a_vals;
  const uint64_t* b_livs;
  const double* b_vals;
  int64_t nnz_a, nnz_b;
  int64_t eoff;  // first global A' entry
  int64_t boff;  // first global B' slot (nnz_b + 1 slots per instance)
  int64_t koff;  // first row pointer (k' + 1 per instance)
  uint64_t kp, np;
  FastDiv kdiv, ndiv;
};

// index i with off[i] <= g < off[i + 1]
__device__ __forceinline__ int find_inst(const int64_t* __restrict__ off, int count, int64_t g) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Row pointers of every instance's B' (k' + 1 slots each, from x.koff).  Whole
// waves step together, so that fill_slots can hand a long run of empty rows
// (clustered rows of B') to the whole wave.
__global__ void bt_dense_ptr_kernel(const BInst* __restrict__ in, const int64_t* __restrict__ boff, int count,
                                    int64_t total, uint32_t* __restrict__ bptr) {
  const int lane = lane_id();
  for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; g0 < total;
       g0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = g0 + lane;
    const bool valid = g < total;
    uint64_t lo = 0, hi = 0;
    uint32_t e32 = 0;
    if (valid) {
      const int i = find_inst(boff, count, g);
      const BInst& x = in[i];
      const int64_t e = g - x.boff;  // 0..nnz_b
      lo = (uint64_t)x.koff + (e == 0 ? 0 : fd_div(x.ndiv, x.b_livs[e - 1]) + 1);
      hi = (uint64_t)x.koff + (e == x.nnz_b ? x.kp : fd_div(x.ndiv, x.b_livs[e])) + 1;
      e32 = (uint32_t)e;
    }
    fill_slots(bptr, valid, lo, hi, e32);
  }
}

__global__ void bt_heads_kernel(const BInst* __restrict__ in, const int64_t* __restrict__ eoff, int count,
                                int64_t total, uint32_t* __restrict__ head) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int i = find_inst(eoff, count, g);
    const BInst& x = in[i];
    const int64_t e = g - x.eoff;
    head[g] = (e == 0 || fd_div(x.kdiv, x.a_livs[e]) != fd_div(x.kdiv, x.a_livs[e - 1])) ? 1u : 0u;
  }
}

__global__ void bt_compact_kernel(const BInst* __restrict__ in, const int64_t* __restrict__ eoff, int count,
                                  int64_t total, const uint32_t* __restrict__ head, const uint32_t* __restrict__ pos,
                                  uint32_t* __restrict__ rs, uint64_t* __restrict__ rid, uint32_t* __restrict__ rinst) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    if (head[g]) {
      const int i = find_inst(eoff, count, g);
      const BInst& x = in[i];
      rs[pos[g]] = (uint32_t)g;
      rid[pos[g]] = fd_div(x.kdiv, x.a_livs[g - x.eoff]);
      rinst[pos[g]] = (uint32_t)i;
    }
    if (g == total - 1) rs[pos[g] + head[g]] = (uint32_t)total;
  }
}

__global__ void bt_entry_len_kernel(const BInst* __restrict__ in, const int64_t* __restrict__ eoff, int count,
                                    int64_t total, const uint32_t* __restrict__ bptr, uint64_t* __restrict__ len,
                                    uint32_t* __restrict__ bstart) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int i = find_inst(eoff, count, g);
    const BInst& x = in[i];
    uint64_t j;
    fd_divmod(x.kdiv, x.a_livs[g - x.eoff], j);
    const uint32_t s = bptr[x.koff + j];
    len[g] = bptr[x.koff + j + 1] - s;
    bstart[g] = s;
  }
}

// Row shapes; rows that the one-wave engine cannot take send their instance to
// the per-call path.
__global__ void bt_classify_kernel(const uint32_t* __restrict__ rs, const uint32_t* __restrict__ rinst,
                                   const uint64_t* __restrict__ poff, const uint64_t* __restrict__ nrows,
                                   int64_t upper, uint8_t* __restrict__ shape, uint32_t* __restrict__ fallback) {
  const uint64_t R = *nrows;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < upper; r += (int64_t)gridDim.x * blockDim.x) {
    if ((uint64_t)r >= R) break;
    const uint32_t e0 = rs[r], e1 = rs[r + 1];
    const uint64_t f = poff[e1] - poff[e0];
    uint8_t sh = kShapeSkip;
    if (f > 0 && small_row(f, e1 - e0)) {
      uint64_t mx = 0;
      for (uint32_t e = e0; e < e1; ++e) {
        const uint64_t l = poff[e + 1] - poff[e];
        mx = l > mx ? l : mx;
      }
      uint32_t lw = 0;
      while ((1ull << lw) < mx) ++lw;
      sh = ((uint64_t)(e1 - e0) << lw) <= (uint64_t)kWave ? (uint8_t)lw : kShapeSearch;
    } else if (f > 0) {
      atomicOr(&fallback[rinst[r]], 1u);
    }
    shape[r] = sh;
  }
}

// The batched rows in chunks of consecutive rows per wave, with the chunk's row
// metadata and a window of 64 consecutive entries loaded coalesced (the rows'
// products are then gathered by lane shuffles, as in the per-call engine).  A
// window holds entries of one instance only; a row of another instance, or
// entries outside the window, move it.  As in the per-call engine, the B'
// loads of the next row are issued before the current row is reduced.
// NARROW: every instance has columns below 2^32 (else each row checks).
template <bool ACC, bool NUMERIC, bool NARROW>
__global__ __launch_bounds__(kRowThreads, NUMERIC ? 6 : 8) void bt_chunk_kernel(
    const BInst* __restrict__ in, const uint32_t* __restrict__ rs, const uint64_t* __restrict__ rid,
    const uint32_t* __restrict__ rinst, const uint8_t* __restrict__ shape, const uint32_t* __restrict__ fallback,
    const uint64_t* __restrict__ poff, const uint32_t* __restrict__ bstart, uint32_t nrows, int chunk_rows,
    uint64_t* __restrict__ cnt, const uint64_t* __restrict__ coff, uint64_t* __restrict__ out_livs,
    double* __restrict__ out_vals) {
  __shared__ RowLds<NUMERIC> s_lds[kRowWaves];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const uint64_t nchunks = ((uint64_t)nrows + chunk_rows - 1) / chunk_rows;
  const RowSpan span = xcd_row_span(nchunks, w);
  if constexpr (ACC && NUMERIC) tab_clear(s_lds[w], lane);
  for (uint64_t c = span.first; c < span.end; c += span.step) {
    const uint64_t r0 = c * chunk_rows;
    const int rows = (int)((uint64_t)nrows - r0 < (uint64_t)chunk_rows ? (uint64_t)nrows - r0 : (uint64_t)chunk_rows);
    uint32_t m_s0 = 0, m_s1 = 0, m_sh = kShapeSkip, m_in = 0;
    uint64_t m_id = 0, m_off = 0;
    if (lane < rows) {
      const uint64_t r = r0 + lane;
      m_s0 = rs[r];
      m_s1 = rs[r + 1];
      m_id = rid[r];
      m_in = rinst[r];
      m_sh = fallback[m_in] ? kShapeSkip : shape[r];
      if (NUMERIC) m_off = coff[r];
    }
    uint32_t my_cnt = 0;
    // entry window [w0, w0 + 64) of instance w_inst (none before the first row;
    // entry indexes are 32-bit, so the tests are scalar compares)
    uint32_t w0 = 0;
    uint32_t w_inst = 0xFFFFFFFFu;
    uint32_t x_len = 0, x_bs = 0;
    uint64_t x_jn = 0;
    double x_av = 0.0;
    uint64_t todo = __ballot(lane < rows && m_sh != kShapeSkip);
    RowProduct<NUMERIC> next;
    int t_next = 0;
    auto stage = [&](int i) {
      const uint8_t sh = (uint8_t)readlane_u32(m_sh, i);
      const uint32_t e0 = readlane_u32(m_s0, i), e1 = readlane_u32(m_s1, i);
      const uint32_t xi = readlane_u32(m_in, i);
      const BInst& x = in[xi];
      t_next = (int)(e1 - e0);  // at most 64 for the rows of this kernel
      if (xi != w_inst || e0 - w0 > (uint32_t)(kWave - t_next)) {
        w0 = e0;
        w_inst = xi;
        const int64_t g = (int64_t)w0 + lane;
        if (g < x.eoff + x.nnz_a) {
          x_len = (uint32_t)(poff[g + 1] - poff[g]);
          x_bs = bstart[g];
          uint64_t j;
          fd_divmod(x.kdiv, x.a_livs[g - x.eoff], j);
          x_jn = j * x.np;
          if (NUMERIC) x_av = x.a_vals[g - x.eoff];
        }
      }
      window_products<NUMERIC>(x.b_livs, x.b_vals, e0, t_next, sh, lane, (int64_t)w0, x_len, x_bs, x_jn, x_av,
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
      const uint64_t np = in[readlane_u32(m_in, i)].np;
      if (todo) stage(__builtin_ctzll(todo));
      RowOut o;
      const uint32_t d =
          row_reduce<ACC, NUMERIC>(valid, ent, col, v, t, NARROW || np < (1ull << 32), lane, s_lds[w], o);
      if (!NUMERIC) {
        if (lane == i) my_cnt = d;
      } else if (o.own) {
        // scalar row base, 32-bit lane offset (the rank is below 64)
        const uint64_t r_off = readlane_u64(m_off, i);
        const uint32_t boff = o.rank * 8u;
        *reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(out_livs + r_off) + boff) =
            o.col + np * readlane_u64(m_id, i);
        *reinterpret_cast<double*>(reinterpret_cast<char*>(out_vals + r_off) + boff) = o.val;
      }
    }
    if (!NUMERIC && lane < rows) cnt[r0 + lane] = my_cnt;
  }
}

// First output position of each instance (its first row's offset) and the flags.
__global__ void bt_ranges_kernel(const BInst* __restrict__ in, int count, const uint32_t* __restrict__ rpos,
                                 const uint64_t* __restrict__ coff, const uint32_t* __restrict__ fallback,
                                 uint64_t* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    out[2 * i] = coff[rpos[in[i].eoff]];
    out[2 * i + 1] = fallback[i];
  }
}

__global__ void gather_vals_kernel(const double* __restrict__ src, const uint64_t* __restrict__ idx, int64_t n,
                                   double* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[idx[i]];
}

__global__ void iota_kernel(uint64_t* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint64_t)i;
}

int grid_for(lco_ctx ctx, int64_t n, int threads) {
  const int64_t want = (n + threads - 1) / threads;
  const int64_t cap = (int64_t)ctx->num_cus * 16;
  return (int)(want < 1 ? 1 : (want > cap ? cap : want));
}

}  // namespace

// Runs one group of jobs that share the accumulator choice; fills outs[job.index]
// for every job it completes and returns the indices that must take the per-call path.
void gather_values(lco_ctx ctx, const double* src, const uint64_t* idx, int64_t n, double* dst) {
  if (n > 0) LCO_LAUNCH(ctx, "gather_vals", gather_vals_kernel, grid_for(ctx, n, 256), 256, 0, src, idx, n, dst);
}

void fill_iota(lco_ctx ctx, uint64_t* out, int64_t n) {
  if (n > 0) LCO_LAUNCH(ctx, "iota", iota_kernel, grid_for(ctx, n, 256), 256, 0, out, n);
}

void* KeptBuffers::raw(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  void* p = dev_alloc(ctx, bytes);
  bufs.push_back({p, bytes});
  return p;
}

void KeptBuffers::release() {
  for (auto& b : bufs) dev_free(ctx, b.first, b.second);
  bufs.clear();
}

int batch_chunk_rows(lco_ctx ctx, uint64_t rows) {
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(kWave, rows / ((uint64_t)ctx->num_cus * 32)));
}

int batch_grid(lco_ctx ctx, uint64_t rows, int chunk_rows, int blocks_per_cu) {
  const uint64_t chunks = (rows + chunk_rows - 1) / chunk_rows;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>((chunks + kRowWaves - 1) / kRowWaves,
                                                       (uint64_t)ctx->num_cus * blocks_per_cu));
}

#define LCO_BT_LAUNCH(NAME, ACC, NUM, ...)                                                               \
  do {                                                                                                     \
    if (narrow) LCO_LAUNCH(ctx, NAME, (bt_chunk_kernel<ACC, NUM, true>), __VA_ARGS__);                   \
    else LCO_LAUNCH(ctx, NAME, (bt_chunk_kernel<ACC, NUM, false>), __VA_ARGS__);                         \
  } while (0)

void batch_numeric(lco_ctx ctx, const BatchLaunch& L) {
  const BInst* in = static_cast<const BInst*>(L.inst);
  const bool narrow = L.narrow;
  if (L.acc)
    LCO_BT_LAUNCH("bt_small_num", true, true, L.grid, kRowThreads, 0, in, L.rs, L.rid, L.rinst, L.shape, L.fallback,
                  L.poff, L.bstart, L.rows, L.chunk_rows, (uint64_t*)nullptr, L.coff, L.out_livs, L.out_vals);
  else
    LCO_BT_LAUNCH("bt_small_num", false, true, L.grid, kRowThreads, 0, in, L.rs, L.rid, L.rinst, L.shape, L.fallback,
                  L.poff, L.bstart, L.rows, L.chunk_rows, (uint64_t*)nullptr, L.coff, L.out_livs, L.out_vals);
}

std::vector<int> batch_group(lco_ctx ctx, const std::vector<BatchJob>& jobs, bool acc, lco_tensor* outs,
                             KeptBuffers* keep, BatchLaunch* launch) {
  const int count = (int)jobs.size();
  std::vector<BInst> host(count);
  std::vector<int64_t> eoff(count + 1), boff(count + 1);
  int64_t E = 0, BS = 0, K = 0;
  bool narrow = true;  // every instance has columns below 2^32
  for (int i = 0; i < count; ++i) {
    const BatchJob& j = jobs[i];
    BInst& x = host[i];
    x.a_livs = j.A->livs;
    x.a_vals = j.A->vals;
    x.b_livs = j.B->livs;
    x.b_vals = j.B->vals;
    x.nnz_a = j.A->nnz;
    x.nnz_b = j.B->nnz;
    x.eoff = eoff[i] = E;
    x.boff = boff[i] = BS;
    x.koff = K;
    x.kp = j.kp;
    x.np = j.np;
    narrow = narrow && j.np < ((uint64_t)1 << 32);
    x.kdiv = make_fastdiv(j.kp);
    x.ndiv = make_fastdiv(j.np);
    E += x.nnz_a;
    BS += x.nnz_b + 1;
    if (j.kp >= (uint64_t)1 << 34) fail(LCO_E_OOM, "batch: singly-compressed row pointer of more than 2^34 entries");
    K += (int64_t)j.kp + 1;
  }
  eoff[count] = E;
  boff[count] = BS;
  if (E > (int64_t)UINT32_MAX) fail(LCO_E_UNSUPPORTED, "batch: more than 2^32-1 entries");
  Scratch s(ctx);
  auto kept = [&](auto* tag, size_t n) { using T = std::remove_pointer_t<decltype(tag)>; return keep ? keep->get<T>(n) : s.get<T>(n); };
  BInst* d_in = kept((BInst*)nullptr, count);
  int64_t* d_eoff = s.get<int64_t>(count + 1);
  int64_t* d_boff = s.get<int64_t>(count + 1);
  LCO_HIP(hipMemcpyAsync(d_in, host.data(), sizeof(BInst) * count, hipMemcpyHostToDevice, ctx->stream));
  LCO_HIP(hipMemcpyAsync(d_eoff, eoff.data(), sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice, ctx->stream));
  LCO_HIP(hipMemcpyAsync(d_boff, boff.data(), sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice, ctx->stream));
  uint32_t* bptr = s.get<uint32_t>(K);
  LCO_LAUNCH(ctx, "bt_dense_ptr", bt_dense_ptr_kernel, grid_for(ctx, BS, 256), 256, 0, d_in, d_boff, count, BS, bptr);
  // rows of A' over all instances (an instance's first entry always starts a row)
  uint32_t* head = s.get<uint32_t>(E);
  uint32_t* rpos = s.get<uint32_t>(E);
  uint64_t* words = s.get<uint64_t>(2);
  memset_async(ctx, words, 0, 2 * sizeof(uint64_t));
  LCO_LAUNCH(ctx, "bt_heads", bt_heads_kernel, grid_for(ctx, E, 256), 256, 0, d_in, d_eoff, count, E, head);
  scan_u32(ctx, head, rpos, E, (uint32_t*)words);
  uint32_t* rs = kept((uint32_t*)nullptr, E + 1);
  uint64_t* rid = kept((uint64_t*)nullptr, E);
  uint32_t* rinst = kept((uint32_t*)nullptr, E);
  LCO_LAUNCH(ctx, "bt_compact", bt_compact_kernel, grid_for(ctx, E, 256), 256, 0, d_in, d_eoff, count, E, head, rpos,
             rs, rid, rinst);
  uint64_t* len = s.get<uint64_t>(E);
  uint64_t* poff = kept((uint64_t*)nullptr, E + 1);
  uint32_t* bstart = kept((uint32_t*)nullptr, E);
  LCO_LAUNCH(ctx, "bt_entry_len", bt_entry_len_kernel, grid_for(ctx, E, 256), 256, 0, d_in, d_eoff, count, E, bptr,
             len, bstart);
  scan_u64(ctx, len, poff, E, poff + E);
  uint8_t* shape = kept((uint8_t*)nullptr, E);
  uint32_t* fallback = kept((uint32_t*)nullptr, count);
  memset_async(ctx, fallback, 0, sizeof(uint32_t) * count);
  LCO_LAUNCH(ctx, "bt_classify", bt_classify_kernel, grid_for(ctx, E, 256), 256, 0, rs, rinst, poff, words, E, shape,
             fallback);
  const uint64_t* rb[1] = {words};
  const uint64_t R = readback(ctx, rb, 1)[0] & 0xffffffffull;
  uint64_t* cnt = s.get<uint64_t>(R + 1);
  uint64_t* coff = kept((uint64_t*)nullptr, R + 1);
  memset_async(ctx, cnt, 0, sizeof(uint64_t) * (R + 1));
  const int chunk_rows = batch_chunk_rows(ctx, R);
  const int grid = batch_grid(ctx, R, chunk_rows, 16);
  if (acc)
    LCO_BT_LAUNCH("bt_small_sym", true, false, grid, kRowThreads, 0, d_in, rs, rid, rinst, shape, fallback, poff,
                  bstart, (uint32_t)R, chunk_rows, cnt, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                  (double*)nullptr);
  else
    LCO_BT_LAUNCH("bt_small_sym", false, false, grid, kRowThreads, 0, d_in, rs, rid, rinst, shape, fallback, poff,
                  bstart, (uint32_t)R, chunk_rows, cnt, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                  (double*)nullptr);
  scan_u64(ctx, cnt, coff, R, coff + R);
  uint64_t* ranges = s.get<uint64_t>(2 * count);
  LCO_LAUNCH(ctx, "bt_ranges", bt_ranges_kernel, grid_for(ctx, count, 256), 256, 0, d_in, count, rpos, coff, fallback,
             ranges);
  // one synchronisation: the output size of every instance
  std::vector<uint64_t> hr(2 * count + 1);
  LCO_HIP(hipMemcpyAsync(hr.data(), ranges, sizeof(uint64_t) * 2 * count, hipMemcpyDeviceToHost, ctx->stream));
  LCO_HIP(hipMemcpyAsync(hr.data() + 2 * count, coff + R, sizeof(uint64_t), hipMemcpyDeviceToHost, ctx->stream));
  sync(ctx);
  const uint64_t total = hr[2 * count];
  if (total > UINT32_MAX) fail(LCO_E_UNSUPPORTED, "batch: more than 2^32-1 output entries");
  // one pool holds every batched output: all LIVs, then all values
  Pool* pool = new_pool(ctx, total * 16);
  uint64_t* pl = (uint64_t*)pool->base;
  double* pv = (double*)((char*)pool->base + total * 8);
  std::vector<int> redo;
  try {
    BatchLaunch L;
    L.acc = acc;
    L.narrow = narrow;
    L.grid = grid;
    L.chunk_rows = chunk_rows;
    L.rows = (uint32_t)R;
    L.inst = d_in;
    L.rs = rs;
    L.rid = rid;
    L.rinst = rinst;
    L.shape = shape;
    L.fallback = fallback;
    L.poff = poff;
    L.bstart = bstart;
    L.coff = coff;
    L.out_livs = pl;
    L.out_vals = pv;
    batch_numeric(ctx, L);
    if (launch) *launch = L;
    for (int i = 0; i < count; ++i) {
      if (hr[2 * i + 1]) {
        redo.push_back(jobs[i].index);
        continue;
      }
      const uint64_t a = hr[2 * i], b = i + 1 < count ? hr[2 * (i + 1)] : total;
      outs[jobs[i].index] = pool_tensor(ctx, pool, jobs[i].order_c, jobs[i].natural_dims, pl + a, pv + a,
                                        (int64_t)(b - a));
    }
  } catch (...) {
    release_pool(pool);
    throw;
  }
  release_pool(pool);  // the tensors hold the remaining references
  return redo;
}

#undef LCO_BT_LAUNCH

}  // namespace lco
