// C-ABI entry points: contexts, tensors, construction and permutation, plus the
// runtime plumbing (errors, allocator bridge, scratch arena, per-kernel timing).
#include <cmath>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>

#include "lco_internal.h"

namespace lco {

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

void clear_error() { g_last_error.clear(); }

lco_status set_error_msg(lco_status s, const char* msg) {
  g_last_error = msg ? msg : "";
  return s;
}

lco_status set_error(const Error& e) { return set_error_msg(e.code, e.what()); }

void fail(lco_status code, const std::string& msg) { throw Error(code, msg); }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? LCO_E_OOM : LCO_E_HIP,
         std::string(what) + ": " + hipGetErrorString(e));
  }
}

// ---------------------------------------------------------------- timing
int Timer::idx(const char* n) {
  auto it = name_idx.find(n);
  if (it != name_idx.end()) return it->second;
  const int i = (int)names.size();
  names.push_back(n);
  name_idx[n] = i;
  launches.push_back(0);
  total_ms.push_back(0.0);
  return i;
}

hipEvent_t Timer::get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  LCO_HIP(hipEventCreate(&e));
  return e;
}

void Timer::collect() {
  for (const Rec& r : pending) {
    LCO_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    LCO_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    launches[r.name] += 1;
    total_ms[r.name] += ms;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
}

void Timer::reset() {
  collect();
  std::fill(launches.begin(), launches.end(), 0);
  std::fill(total_ms.begin(), total_ms.end(), 0.0);
}

Timer::~Timer() {
  for (const Rec& r : pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

LaunchScope::LaunchScope(lco_ctx c, const char* n) : ctx(c), name(-1) {
  if (!ctx->timer.on) return;
  if (!ctx->timer.only.empty() && ctx->timer.only != n) return;
  name = ctx->timer.idx(n);
  hipEvent_t a = ctx->timer.get_event();
  LCO_HIP(hipEventRecord(a, ctx->stream));
  b = ctx->timer.get_event();
  ctx->timer.pending.push_back({name, a, b});
}

LaunchScope::~LaunchScope() {
  if (name < 0) return;
  (void)hipEventRecord(b, ctx->stream);
}

// ---------------------------------------------------------------- memory
namespace {
constexpr size_t kCacheCap = (size_t)32 << 30;  // bytes of released blocks a context keeps at most

size_t block_size(size_t bytes) {
  if (bytes < ((size_t)1 << 20)) {
    size_t b = 4096;
    while (b < bytes) b <<= 1;
    return b;
  }
  const size_t g = (size_t)2 << 20;
  return (bytes + g - 1) / g * g;
}

// Returns cached blocks to the device, largest first, until at most `keep`
// bytes stay cached (the stream is drained first: a block may have been
// released while work that uses it is still queued).
void trim_blocks(lco_ctx ctx, size_t keep) {
  BlockCache& c = ctx->blocks;
  std::vector<void*> out;
  {
    std::lock_guard<std::mutex> lk(c.mu);
    while (c.cached > keep && !c.free.empty()) {
      auto it = std::prev(c.free.end());
      c.cached -= it->first;
      out.push_back(it->second);
      c.size.erase(it->second);
      c.free.erase(it);
    }
  }
  if (out.empty()) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (void* p : out) (void)hipFree(p);
}
}  // namespace

void* dev_alloc(lco_ctx ctx, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (ctx->alloc) {
    p = ctx->alloc(ctx->user, bytes, (void*)ctx->stream);
    if (!p) fail(LCO_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
  }
  const size_t want = block_size(bytes);
  BlockCache& c = ctx->blocks;
  {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.free.lower_bound(want);
    if (it != c.free.end() && it->first <= want + want / 4) {
      p = it->second;
      c.cached -= it->first;
      c.free.erase(it);
      return p;
    }
  }
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim_blocks(ctx, 0);  // give every cached block back and try once more
    e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(LCO_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
  }
  std::lock_guard<std::mutex> lk(c.mu);
  c.size[p] = want;
  return p;
}

void dev_free(lco_ctx ctx, void* p, size_t bytes) {
  if (!p) return;
  if (ctx->free_fn) {
    ctx->free_fn(ctx->user, p, bytes, (void*)ctx->stream);
    return;
  }
  BlockCache& c = ctx->blocks;
  bool over = false;
  {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.size.find(p);
    if (it == c.size.end()) return;  // not a block of this context
    c.free.emplace(it->second, p);
    c.cached += it->second;
    over = c.cached > kCacheCap;
  }
  if (over) trim_blocks(ctx, kCacheCap / 2);
}

Scratch::Scratch(lco_ctx ctx) : ctx_(ctx) {
  Arena& a = ctx->arena;
  mark_chunk_ = a.chunks.empty() ? 0 : a.chunks.size() - 1;
  mark_used_ = a.used;
  mark_in_use_ = a.in_use;
  ctx->scratch_depth++;
}

void* Scratch::raw(size_t bytes) {
  Arena& a = ctx_->arena;
  bytes = (bytes + 255) & ~(size_t)255;
  if (a.fixed) {
    if (a.used + bytes > a.fixed_cap) fail(LCO_E_OOM, "scratch: the operation needs more than the fixed workspace");
    char* p = a.fixed + a.used;
    a.used += bytes;
    a.in_use += bytes;
    a.high_water = std::max(a.high_water, a.in_use);
    return p;
  }
  if (a.chunks.empty() || a.used + bytes > a.chunks.back().cap) {
    size_t cap = std::max<size_t>(bytes, (size_t)32 << 20);
    if (!a.chunks.empty()) cap = std::max(cap, a.chunks.back().cap * 2);
    cap = std::max(cap, a.high_water);
    char* p = (char*)dev_alloc(ctx_, cap);
    a.chunks.push_back({p, cap});
    a.used = 0;
  }
  char* p = a.chunks.back().p + a.used;
  a.used += bytes;
  a.in_use += bytes;
  a.high_water = std::max(a.high_water, a.in_use);
  return p;
}

Scratch::~Scratch() {
  Arena& a = ctx_->arena;
  ctx_->scratch_depth--;
  if (a.fixed) {
    a.used = ctx_->scratch_depth == 0 ? 0 : mark_used_;
    a.in_use = ctx_->scratch_depth == 0 ? 0 : mark_in_use_;
    return;
  }
  if (ctx_->scratch_depth == 0) {
    if (a.chunks.size() > 1) {
      // the op outgrew the main chunk: release everything (stream-ordered); the
      // next op allocates one chunk of the high-water size
      const size_t hw = a.high_water;
      for (auto& c : a.chunks) dev_free(ctx_, c.p, c.cap);
      a.chunks.clear();
      a.high_water = hw;
    }
    a.used = 0;
    a.in_use = 0;
  } else if (!a.chunks.empty() && a.chunks.size() - 1 == mark_chunk_) {
    a.used = mark_used_;
    a.in_use = mark_in_use_;
  } else {
    a.in_use = mark_in_use_;
  }
}

FixedScratch::FixedScratch(lco_ctx ctx, void* base, size_t bytes) : ctx_(ctx) {
  if (ctx->scratch_depth != 0) fail(LCO_E_ARG, "fixed workspace inside another operation");
  saved_ = std::move(ctx->arena);
  ctx->arena = Arena{};
  ctx->arena.fixed = static_cast<char*>(base);
  ctx->arena.fixed_cap = bytes;
}

FixedScratch::~FixedScratch() { ctx_->arena = std::move(saved_); }

void memset_async(lco_ctx ctx, void* p, int v, size_t bytes) {
  if (bytes) LCO_HIP(hipMemsetAsync(p, v, bytes, ctx->stream));
}

void copy_d2d(lco_ctx ctx, void* dst, const void* src, size_t bytes) {
  if (bytes) LCO_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
}

static void check_device_error(lco_ctx ctx, uint32_t word) {
  if (word) {
    LCO_HIP(hipMemsetAsync(ctx->dev_err, 0, sizeof(uint32_t), ctx->stream));
    fail(LCO_E_HIP, "a kernel exceeded its bounded wait for another workgroup (results discarded)");
  }
}

namespace {
constexpr int kErrWord = 61;   // pinned word receiving the device error word
constexpr int kFlagWord = 62;  // pinned word receiving the readback sequence number

struct ReadbackArgs {
  const uint64_t* words[kReadbackWords];
  int count;
};

// Gathers the words and the device error word into the pinned buffer, then
// publishes `seq` in its flag word with a system-scope release, so that the
// host can wait for the flag rather than for the whole stream.
__global__ void readback_kernel(ReadbackArgs a, const uint32_t* __restrict__ err, uint64_t* out, uint64_t seq) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < a.count; ++i) out[i] = *a.words[i];
  out[kErrWord] = *err;
  __hip_atomic_store(&out[kFlagWord], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
}  // namespace

const uint64_t* readback(lco_ctx ctx, const uint64_t* const* dev_words, int count) {
  if (count < 0 || count > kReadbackWords) fail(LCO_E_ARG, "readback: too many words");
  ReadbackArgs a{};
  for (int i = 0; i < count; ++i) a.words[i] = dev_words[i];
  a.count = count;
  const uint64_t seq = ++ctx->readback_seq;
  LCO_LAUNCH(ctx, "readback", readback_kernel, 1, 64, 0, a, (const uint32_t*)ctx->dev_err, ctx->pinned_dev, seq);
  // Spin on the flag (it lands a few microseconds after the kernel runs); after
  // 20 ms, wait for the stream instead, which also reports a failed kernel.
  volatile uint64_t* flag = ctx->pinned + kFlagWord;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t it = 1; *flag != seq; ++it) {
    if ((it & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) {
      LCO_HIP(hipStreamSynchronize(ctx->stream));
      if (*flag != seq) fail(LCO_E_HIP, "readback: the device did not publish the requested words");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  check_device_error(ctx, (uint32_t)ctx->pinned[kErrWord]);
  return ctx->pinned;
}

void sync(lco_ctx ctx) {
  LCO_HIP(hipMemcpyAsync((uint32_t*)(ctx->pinned + 63), ctx->dev_err, sizeof(uint32_t), hipMemcpyDeviceToHost,
                         ctx->stream));
  LCO_HIP(hipStreamSynchronize(ctx->stream));
  check_device_error(ctx, *(uint32_t*)(ctx->pinned + 63));
}

lco_tensor new_tensor(lco_ctx ctx, int order, const uint64_t* dims, int64_t nnz) {
  lco_tensor t = new lco_tensor_s;
  t->ctx = ctx;
  t->order = order;
  for (int r = 0; r < order; ++r) t->dims[r] = dims[r];
  t->nnz = nnz;
  if (nnz > 0) {
    t->bytes = (size_t)nnz * 16;
    try {
      t->base = dev_alloc(ctx, t->bytes);
    } catch (...) {
      delete t;
      throw;
    }
    t->livs = (uint64_t*)t->base;
    t->vals = (double*)((char*)t->base + (size_t)nnz * 8);
  }
  return t;
}

Pool* new_pool(lco_ctx ctx, size_t bytes) {
  Pool* p = new Pool;
  p->ctx = ctx;
  p->bytes = bytes;
  p->refs = 1;
  try {
    p->base = dev_alloc(ctx, bytes);
  } catch (...) {
    delete p;
    throw;
  }
  return p;
}

void release_pool(Pool* p) {
  if (!p) return;
  if (--p->refs == 0) {
    dev_free(p->ctx, p->base, p->bytes);
    delete p;
  }
}

lco_tensor pool_tensor(lco_ctx ctx, Pool* p, int order, const uint64_t* dims, uint64_t* livs, double* vals,
                       int64_t nnz) {
  lco_tensor t = new lco_tensor_s;
  t->ctx = ctx;
  t->order = order;
  for (int r = 0; r < order; ++r) t->dims[r] = dims[r];
  t->nnz = nnz;
  if (nnz > 0) {
    t->pool = p;
    p->refs++;
    t->livs = livs;
    t->vals = vals;
  }
  return t;
}

static void free_tensor(lco_tensor t) {
  if (!t) return;
  if (t->pool) release_pool(t->pool);
  else if (t->base) dev_free(t->ctx, t->base, t->bytes);
  delete t;
}

int64_t create_storage(lco_ctx ctx, lco_tensor t, const uint64_t* d_idx, const double* d_vals, int64_t n,
                       uint32_t flags, int full_bits, uint64_t max_liv, uint64_t** out_livs, double** out_vals,
                       void** out_base, size_t* out_bytes);

lco_tensor contract_run(lco_ctx ctx, const lco_tensor_s* a, const lco_tensor_s* b, const ContractDetail& d);

}  // namespace lco

using namespace lco;

#define LCO_TRY try {
#define LCO_CATCH                                                   \
  }                                                                 \
  catch (const Error& e) {                                          \
    return set_error(e);                                            \
  }                                                                 \
  catch (const std::bad_alloc&) {                                   \
    return set_error_msg(LCO_E_OOM, "host allocation failed");      \
  }                                                                 \
  catch (const std::exception& e) {                                 \
    return set_error_msg(LCO_E_HIP, e.what());                      \
  }

extern "C" {

const char* lco_version(void) { return "lco-mi355x 0.1 (gfx950)"; }

const char* lco_status_str(lco_status s) {
  switch (s) {
    case LCO_OK: return "ok";
    case LCO_E_ARG: return "bad argument";
    case LCO_E_OVERFLOW: return "index overflow";
    case LCO_E_SHAPE: return "shape mismatch";
    case LCO_E_UNSORTED: return "unsorted input";
    case LCO_E_DUPLICATE: return "duplicate entry";
    case LCO_E_OOM: return "out of memory";
    case LCO_E_UNSUPPORTED: return "unsupported";
    case LCO_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* lco_last_error(void) { return g_last_error.c_str(); }

lco_status lco_ctx_create(int device, void* hip_stream, lco_alloc_fn alloc, lco_free_fn free_fn, void* user,
                          lco_ctx* out) {
  LCO_TRY
  if (!out) fail(LCO_E_ARG, "lco_ctx_create: out is NULL");
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) fail(LCO_E_ARG, "lco_ctx_create: give both alloc and free or neither");
  int count = 0;
  LCO_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) fail(LCO_E_ARG, "lco_ctx_create: no such device");
  LCO_HIP(hipSetDevice(device));
  noalloc_init_device(device);
  lco_ctx c = new lco_ctx_s;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->alloc = alloc;
  c->free_fn = free_fn;
  c->user = user;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->num_cus = cus;
  hipError_t e = hipHostMalloc((void**)&c->pinned, 64 * sizeof(uint64_t), hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&c->pinned_dev, c->pinned, 0);
  if (e != hipSuccess) {
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
    hip_check(e, "hipHostMalloc");
  }
  std::memset(c->pinned, 0, 64 * sizeof(uint64_t));
  try {
    c->dev_err = (uint32_t*)dev_alloc(c, 256);
    LCO_HIP(hipMemsetAsync(c->dev_err, 0, 256, c->stream));
  } catch (...) {
    (void)hipHostFree(c->pinned);
    delete c;
    throw;
  }
  *out = c;
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_ctx_destroy(lco_ctx ctx) {
  if (!ctx) return LCO_OK;
  LCO_TRY
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& c : ctx->arena.chunks) dev_free(ctx, c.p, c.cap);
  ctx->arena.chunks.clear();
  if (ctx->dev_err) dev_free(ctx, ctx->dev_err, 256);
  (void)hipStreamSynchronize(ctx->stream);
  trim_blocks(ctx, 0);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_ctx_set_stream(lco_ctx ctx, void* hip_stream) {
  if (!ctx) return set_error_msg(LCO_E_ARG, "lco_ctx_set_stream: ctx is NULL");
  // released blocks are reused in stream order: drain the old stream first
  if ((hipStream_t)hip_stream != ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ctx->stream = (hipStream_t)hip_stream;
  return LCO_OK;
}

lco_status lco_ctx_synchronize(lco_ctx ctx) {
  if (!ctx) return set_error_msg(LCO_E_ARG, "lco_ctx_synchronize: ctx is NULL");
  LCO_TRY
  LCO_HIP(hipSetDevice(ctx->device));
  // a readback of no words: its kernel runs once everything queued before it
  // has finished and publishes the device error word; the host spins on its
  // flag (falling back to a stream synchronisation after 20 ms), which wakes
  // sooner than a sleeping stream synchronisation
  (void)readback(ctx, nullptr, 0);
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_timing_enable(lco_ctx ctx, int on) {
  if (!ctx) return set_error_msg(LCO_E_ARG, "lco_timing_enable: ctx is NULL");
  ctx->timer.on = on != 0;
  return LCO_OK;
}

lco_status lco_timing_only(lco_ctx ctx, const char* kernel) {
  if (!ctx) return set_error_msg(LCO_E_ARG, "lco_timing_only: ctx is NULL");
  LCO_TRY
  ctx->timer.only = kernel ? kernel : "";
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_timing_reset(lco_ctx ctx) {
  if (!ctx) return set_error_msg(LCO_E_ARG, "lco_timing_reset: ctx is NULL");
  LCO_TRY
  ctx->timer.reset();
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_timing_query(lco_ctx ctx, const char* kernel, int64_t* launches, double* total_ms) {
  if (!ctx || !kernel || !launches || !total_ms) return set_error_msg(LCO_E_ARG, "lco_timing_query: bad argument");
  LCO_TRY
  ctx->timer.collect();
  *launches = 0;
  *total_ms = 0.0;
  auto it = ctx->timer.name_idx.find(kernel);
  if (it != ctx->timer.name_idx.end()) {
    *launches = ctx->timer.launches[it->second];
    *total_ms = ctx->timer.total_ms[it->second];
  }
  return LCO_OK;
  LCO_CATCH
}

const char* lco_timing_kernel_name(lco_ctx ctx, int i) {
  if (!ctx || i < 0 || i >= (int)ctx->timer.names.size()) return nullptr;
  return ctx->timer.names[i].c_str();
}

lco_status lco_create(lco_ctx ctx, int order, const uint64_t* dims, int64_t nnz, const uint64_t* d_idx,
                      const double* d_vals, uint32_t flags, lco_tensor* out) {
  LCO_TRY
  if (!out) fail(LCO_E_ARG, "lco_create: out is NULL");
  *out = nullptr;
  if (!ctx) fail(LCO_E_ARG, "lco_create: ctx is NULL");
  if (order < 0 || order > LCO_MAX_ORDER) fail(LCO_E_ARG, "lco_create: order out of range");
  if (order > 0 && !dims) fail(LCO_E_ARG, "lco_create: dims is NULL");
  if (nnz < 0) fail(LCO_E_ARG, "lco_create: negative nnz");
  if (nnz > 0 && (!d_idx || !d_vals)) fail(LCO_E_ARG, "lco_create: data pointers are NULL");
  if (flags & ~(LCO_SORTED | LCO_COORDS | LCO_SUM_DUPLICATES)) fail(LCO_E_ARG, "lco_create: unknown flags");
  unsigned __int128 total = 1;
  for (int r = 0; r < order; ++r) {
    if (dims[r] == 0) fail(LCO_E_ARG, "lco_create: zero dimension");
    total *= dims[r];
    if (total > ((unsigned __int128)1 << 64)) fail(LCO_E_OVERFLOW, "lco_create: product of dimensions exceeds 2^64");
  }
  if (nnz > (int64_t)UINT32_MAX) fail(LCO_E_UNSUPPORTED, "lco_create: more than 2^32-1 entries");
  if (order == 0 && nnz > 1 && !(flags & LCO_SUM_DUPLICATES))
    fail(LCO_E_DUPLICATE, "lco_create: an order-0 tensor holds at most one entry");
  LCO_HIP(hipSetDevice(ctx->device));
  const uint64_t max_liv = (uint64_t)(total - 1);
  int full_bits = 0;
  {
    const unsigned __int128 mx = total - 1;
    const uint64_t hi = (uint64_t)(mx >> 64), lo = (uint64_t)mx;
    full_bits = hi ? 64 + bits_for(hi) : bits_for(lo);
  }
  lco_tensor t = new_tensor(ctx, order, dims, nnz);
  if (nnz > 0) {
    try {
      uint64_t* nl = nullptr;
      double* nv = nullptr;
      void* nb = nullptr;
      size_t nbytes = 0;
      const int64_t distinct =
          create_storage(ctx, t, d_idx, d_vals, nnz, flags, full_bits, max_liv, &nl, &nv, &nb, &nbytes);
      if (distinct != nnz) {
        dev_free(ctx, t->base, t->bytes);
        t->base = nb;
        t->bytes = nbytes;
        t->livs = nl;
        t->vals = nv;
        t->nnz = distinct;
      }
    } catch (...) {
      free_tensor(t);
      throw;
    }
  }
  *out = t;
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_destroy(lco_tensor t) {
  LCO_TRY
  if (t) {
    (void)hipSetDevice(t->ctx->device);
    free_tensor(t);
  }
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_read(lco_tensor t, uint64_t* livs, double* vals) {
  LCO_TRY
  if (!t) fail(LCO_E_ARG, "lco_read: tensor is NULL");
  LCO_HIP(hipSetDevice(t->ctx->device));
  LCO_HIP(hipStreamSynchronize(t->ctx->stream));
  const size_t bytes = (size_t)t->nnz * 8;
  if (bytes && livs) LCO_HIP(hipMemcpy(livs, t->livs, bytes, hipMemcpyDeviceToHost));
  if (bytes && vals) LCO_HIP(hipMemcpy(vals, t->vals, bytes, hipMemcpyDeviceToHost));
  return LCO_OK;
  LCO_CATCH
}

int64_t lco_nnz(lco_tensor t) { return t ? t->nnz : -1; }
int lco_order(lco_tensor t) { return t ? t->order : -1; }
const uint64_t* lco_dims(lco_tensor t) { return t ? t->dims : nullptr; }
const uint64_t* lco_livs(lco_tensor t) { return t ? t->livs : nullptr; }
const double* lco_vals(lco_tensor t) { return t ? t->vals : nullptr; }

lco_status lco_permute(lco_ctx ctx, lco_tensor in, const int* perm, lco_tensor* out) {
  LCO_TRY
  if (!out) fail(LCO_E_ARG, "lco_permute: out is NULL");
  *out = nullptr;
  if (!ctx || !in) fail(LCO_E_ARG, "lco_permute: ctx or tensor is NULL");
  if (in->ctx->device != ctx->device) fail(LCO_E_ARG, "lco_permute: tensor lives on another device");
  RpDetail plan = plan_permute(in->order, in->dims, perm, in->nnz, default_digit_cap());
  LCO_HIP(hipSetDevice(ctx->device));
  lco_tensor t = new_tensor(ctx, in->order, plan.new_dims, in->nnz);
  try {
    permute_storage(ctx, in, plan, t->livs, t->vals);
  } catch (...) {
    free_tensor(t);
    throw;
  }
  *out = t;
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_contract(lco_ctx ctx, lco_tensor a, const int* a_labels, lco_tensor b, const int* b_labels,
                        int c_order, const int* c_labels, uint32_t flags, lco_tensor* out) {
  LCO_TRY
  if (!out) fail(LCO_E_ARG, "lco_contract: out is NULL");
  *out = nullptr;
  if (!ctx || !a || !b) fail(LCO_E_ARG, "lco_contract: ctx or tensor is NULL");
  if (a->ctx->device != ctx->device || b->ctx->device != ctx->device)
    fail(LCO_E_ARG, "lco_contract: tensor lives on another device");
  ContractDetail d = plan_contract(a->order, a->dims, a_labels, a->nnz, b->order, b->dims, b_labels, b->nnz,
                                   c_order, c_labels, flags, &ctx->sel);
  LCO_HIP(hipSetDevice(ctx->device));
  *out = contract_run(ctx, a, b, d);
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_ctx_set_crossovers(lco_ctx ctx, double doubly_compressed, double no_accumulator,
                                  double outer_product) {
  LCO_TRY
  if (!ctx) fail(LCO_E_ARG, "lco_ctx_set_crossovers: ctx is NULL");
  for (double x : {doubly_compressed, no_accumulator, outer_product})
    if (!(x >= 3.0) || std::isinf(x)) fail(LCO_E_ARG, "lco_ctx_set_crossovers: crossovers must be finite and >= 3");
  ctx->sel.cross[0] = doubly_compressed;
  ctx->sel.cross[1] = no_accumulator;
  ctx->sel.cross[2] = outer_product;
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_ctx_set_index_algorithm(lco_ctx ctx, int algo) {
  LCO_TRY
  if (!ctx) fail(LCO_E_ARG, "lco_ctx_set_index_algorithm: ctx is NULL");
  if (algo != LCO_ALG_SOP && algo != LCO_ALG_DCSC && algo != LCO_ALG_DCSR)
    fail(LCO_E_ARG, "lco_ctx_set_index_algorithm: algo must be SOP, DCSC or DCSR");
  ctx->sel.index_dc = algo != LCO_ALG_SOP;
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_ctx_get_index_algorithm(lco_ctx ctx, int* algo) {
  LCO_TRY
  if (!ctx || !algo) fail(LCO_E_ARG, "lco_ctx_get_index_algorithm: bad argument");
  *algo = ctx->sel.index_dc ? LCO_ALG_DCSC : LCO_ALG_SOP;
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_ctx_get_crossovers(lco_ctx ctx, double* doubly_compressed, double* no_accumulator,
                                  double* outer_product) {
  LCO_TRY
  if (!ctx || !doubly_compressed || !no_accumulator || !outer_product)
    fail(LCO_E_ARG, "lco_ctx_get_crossovers: bad argument");
  *doubly_compressed = ctx->sel.cross[0];
  *no_accumulator = ctx->sel.cross[1];
  *outer_product = ctx->sel.cross[2];
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_add(lco_ctx ctx, double alpha, lco_tensor a, const int* a_labels, double beta, lco_tensor b,
                   const int* b_labels, const int* c_labels, lco_tensor* out) {
  LCO_TRY
  if (!out) fail(LCO_E_ARG, "lco_add: out is NULL");
  *out = nullptr;
  if (!ctx || !a || !b) fail(LCO_E_ARG, "lco_add: ctx or tensor is NULL");
  if (a->ctx->device != ctx->device || b->ctx->device != ctx->device)
    fail(LCO_E_ARG, "lco_add: tensor lives on another device");
  AddDetail d = plan_add(a->order, a->dims, a_labels, b->order, b->dims, b_labels, c_labels);
  LCO_HIP(hipSetDevice(ctx->device));
  *out = add_run(ctx, alpha, a, beta, b, d);
  return LCO_OK;
  LCO_CATCH
}

lco_status lco_plan_info(lco_ctx ctx, lco_tensor a, const int* a_labels, lco_tensor b, const int* b_labels,
                         int c_order, const int* c_labels, uint32_t flags, lco_plan* out) {
  LCO_TRY
  if (!out || !ctx || !a || !b) fail(LCO_E_ARG, "lco_plan_info: bad argument");
  ContractDetail d = plan_contract(a->order, a->dims, a_labels, a->nnz, b->order, b->dims, b_labels, b->nnz,
                                   c_order, c_labels, flags, &ctx->sel);
  *out = d.pub;
  return LCO_OK;
  LCO_CATCH
}

}  // extern "C"
