// Internal declarations shared by the host orchestration and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <stdexcept>
#include <unordered_map>
#include <string>
#include <vector>

#include "../../include/lco.h"
#include "fastdiv.h"

namespace lco {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  lco_status code;
  Error(lco_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(lco_status code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define LCO_HIP(x) ::lco::hip_check((x), #x)

// ------------------------------------------------------------------ timing
struct Timer {
  bool on = false;
  std::string only;  // when not empty: time launches of this kernel only
  struct Rec { int name; hipEvent_t a, b; };
  std::vector<std::string> names;
  std::map<std::string, int> name_idx;
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::vector<int64_t> launches;
  std::vector<double> total_ms;
  int idx(const char* n);
  hipEvent_t get_event();
  void collect();  // synchronises pending events and accumulates
  void reset();
  ~Timer();
};

// ------------------------------------------------------------------ context
struct Arena {
  struct Chunk { char* p; size_t cap; };
  std::vector<Chunk> chunks;  // chunks[0] is the main chunk
  size_t used = 0;            // bytes used in the current (last) chunk
  size_t high_water = 0;      // total bytes in use at the peak of the current op
  size_t in_use = 0;
  // A fixed workspace (not null): scratch is carved from it and never
  // allocated; a request beyond fixed_cap fails with LCO_E_OOM.
  char* fixed = nullptr;
  size_t fixed_cap = 0;
};

// ------------------------------------------------------------------ device blocks
// Device memory a context allocated itself (no allocator callbacks) and has
// released, kept for reuse.  Every block is used in the order of the
// context's stream, so a released block can serve the next allocation on that
// stream at once.  Requests are rounded up (powers of two below 1 MiB,
// multiples of 2 MiB above); a request takes the smallest cached block of its
// rounded size up to a quarter more.  Beyond kCacheCap bytes cached, the
// largest blocks are returned to the device.
struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, void*> free;       // cached blocks by size
  std::unordered_map<void*, size_t> size;  // size of every block this cache allocated
  size_t cached = 0;                       // bytes held in `free`
};

// ------------------------------------------------------------------ selector
// Hyper-sparsity up to which the doubly-compressed, no-accumulator and
// index-cell algorithms give way to CSC/CSR, and the index-sparse x
// index-sparse cell's algorithm: SOP (the paper's table) or the doubly
// compressed accumulator algorithms.
struct Selector {
  double cross[3] = {LCO_MI355X_DC_CROSSOVER, LCO_MI355X_NA_CROSSOVER, LCO_MI355X_INDEX_CROSSOVER};
  bool index_dc = LCO_MI355X_INDEX_ALGORITHM != LCO_ALG_SOP;
};

}  // namespace lco

struct lco_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  lco_alloc_fn alloc = nullptr;
  lco_free_fn free_fn = nullptr;
  void* user = nullptr;
  int num_cus = 256;
  size_t max_lds = 65536;
  lco::Arena arena;
  lco::BlockCache blocks;  // released device blocks (when the library allocates itself)
  int scratch_depth = 0;
  uint64_t* pinned = nullptr;  // host-pinned readback buffer (64 words, device-coherent)
  uint64_t* pinned_dev = nullptr;  // the same buffer as the device addresses it
  uint64_t readback_seq = 0;       // last sequence number published in the buffer's flag word
  lco::Timer timer;
  uint32_t* dev_err = nullptr; // device word: set by a kernel that gave up a bounded wait
  int64_t batch_stats[3] = {0, 0, 0};  // last batch on this context: instances batched, run per call, of the
                                     // batched those in the persistent engine
  // batched-engine autotuner: (size bucket, selected branch) -> (branch, 64-row chunks per work item)
  std::map<int, std::pair<int, int>> tune;
  // the selector's settings (default: those measured on MI355X)
  lco::Selector sel;
};

namespace lco {
// Device memory shared by several tensors (the outputs of a batch); freed when
// the last tensor referring to it is destroyed.
struct Pool {
  lco_ctx ctx = nullptr;
  void* base = nullptr;
  size_t bytes = 0;
  int refs = 0;
};
}  // namespace lco

struct lco_tensor_s {
  lco::Pool* pool = nullptr;  // non-null: livs/vals point into a shared pool
  lco_ctx ctx = nullptr;
  int order = 0;
  uint64_t dims[LCO_MAX_ORDER] = {};
  int64_t nnz = 0;
  uint64_t* livs = nullptr;  // device
  double* vals = nullptr;    // device
  void* base = nullptr;      // single allocation holding livs then vals
  size_t bytes = 0;
};

namespace lco {

// device memory through the context's allocator
void* dev_alloc(lco_ctx ctx, size_t bytes);
void dev_free(lco_ctx ctx, void* p, size_t bytes);

// An LCO tensor whose storage is allocated (not yet filled).
lco_tensor new_tensor(lco_ctx ctx, int order, const uint64_t* dims, int64_t nnz);
// Shared pools: a new pool holds one reference; each pool tensor adds one.
Pool* new_pool(lco_ctx ctx, size_t bytes);
void release_pool(Pool* p);
lco_tensor pool_tensor(lco_ctx ctx, Pool* p, int order, const uint64_t* dims, uint64_t* livs, double* vals,
                       int64_t nnz);

// Per-operation scratch space carved from the context's arena (256-byte aligned).
// Scopes nest; memory is reclaimed when the outermost scope of an op ends.
class Scratch {
 public:
  explicit Scratch(lco_ctx ctx);
  ~Scratch();
  void* raw(size_t bytes);
  template <class T> T* get(size_t count) { return static_cast<T*>(raw(count * sizeof(T) + 1)); }
 private:
  lco_ctx ctx_;
  size_t mark_chunk_, mark_used_, mark_in_use_;
};

// The context's scratch taken from a fixed device workspace for the lifetime of
// this object (the previous arena is put back afterwards).
class FixedScratch {
 public:
  FixedScratch(lco_ctx ctx, void* base, size_t bytes);
  ~FixedScratch();
 private:
  lco_ctx ctx_;
  Arena saved_;
};

// Called once per context creation with the context's device current: sets up
// the device's fixed workspace of the no-allocation entry points.
void noalloc_init_device(int device);

// small host<->device helpers on the context stream
void memset_async(lco_ctx ctx, void* p, int v, size_t bytes);
void copy_d2d(lco_ctx ctx, void* dst, const void* src, size_t bytes);
// Copies `count` (at most kReadbackWords) 64-bit device words to the pinned
// buffer once every operation queued before has finished; returns the buffer.
constexpr int kReadbackWords = 8;
const uint64_t* readback(lco_ctx ctx, const uint64_t* const* dev_words, int count);
void sync(lco_ctx ctx);

// timing scope around one kernel launch
struct LaunchScope {
  lco_ctx ctx; int name; hipEvent_t b = nullptr;
  LaunchScope(lco_ctx c, const char* n);
  ~LaunchScope();
};

#define LCO_LAUNCH(ctx, name, kernel, grid, block, shmem, ...)                                   \
  do {                                                                                           \
    ::lco::LaunchScope _ls((ctx), (name));                                                       \
    hipLaunchKernelGGL((kernel), dim3(grid), dim3(block), (shmem), (ctx)->stream, __VA_ARGS__);  \
    ::lco::hip_check(hipGetLastError(), name);                                                   \
  } while (0)

inline int bits_for(uint64_t max_value) {  // bits needed to represent max_value (0 -> 0)
  return max_value ? 64 - __builtin_clzll(max_value) : 0;
}

// ------------------------------------------------------------------ planning
struct RpDetail {
  lco_rp_plan pub;
  int order;
  uint64_t new_dims[LCO_MAX_ORDER];
  uint64_t new_weight_of_input_mode[LCO_MAX_ORDER];  // W'_{perm^-1[q]}
  int sort_bits;                                     // bits sorted by the chosen method
  double avg_segment = 0;                            // non-zeros per possible segment (segmented method)
};
RpDetail plan_permute(int order, const uint64_t* dims, const int* perm, int64_t nnz, int digit_cap);

struct ContractDetail {
  lco_plan pub;
  bool empty = false;          // an operand has no non-zeros
  // operand layouts: output mode r of the rearranged operand is input mode perm[r]
  int perm_a[LCO_MAX_ORDER], perm_b[LCO_MAX_ORDER];
  int order_a, order_b, order_c;
  // natural product layout -> c_labels: output mode r is natural mode perm_c[r]
  int perm_c[LCO_MAX_ORDER];
  uint64_t natural_dims[LCO_MAX_ORDER];
  uint64_t c_dims[LCO_MAX_ORDER];
  // SOP output key: modes of the rearranged A (free part) and B (free part)
  int n_free_a, n_free_b, n_contracted;
  uint64_t free_a_dims[LCO_MAX_ORDER], free_b_dims[LCO_MAX_ORDER];
  uint64_t free_a_cweight[LCO_MAX_ORDER], free_b_cweight[LCO_MAX_ORDER];  // weight in the C LIV
  bool sop_simple_key = false;  // C LIV == i + m * j
  // Entrywise modes (in a, b and the output): the product is block diagonal.
  // The operand on the engine's row side (dup = 1: a, 2: b) is re-sorted by its
  // block-diagonal matricised LIV, in which each entrywise mode appears with its
  // rows and with its columns: the LIV is sum_q coord_q * dup_weight[q], below
  // 2^dup_bits; the other operand is permuted as usual (perm_a / perm_b).
  int n_entrywise = 0;
  int dup = 0;
  uint64_t dup_weight[LCO_MAX_ORDER];
  uint64_t dup_dims[2];  // (contracted x E, rows x E) of the re-sorted operand
  int dup_bits = 0;
  // sizes handed to the engine: rows of its left operand, contracted, columns
  // of its right operand (entrywise modes counted on the left only)
  uint64_t em, ek, en;
};
// `sel`: the selector's crossovers and index-cell algorithm (NULL: the paper's table as is)
ContractDetail plan_contract(int oa, const uint64_t* da, const int* la, int64_t na, int ob, const uint64_t* db,
                             const int* lb, int64_t nb, int oc, const int* lc, uint32_t flags,
                             const Selector* sel = nullptr);
// Addition of two tensors over the same labelled modes: each operand is brought
// into the output's mode order (output mode r is operand mode perm[r]).
struct AddDetail {
  int order = 0;
  uint64_t c_dims[LCO_MAX_ORDER] = {};
  int perm_a[LCO_MAX_ORDER] = {}, perm_b[LCO_MAX_ORDER] = {};
  bool permute_a = false, permute_b = false;
};
AddDetail plan_add(int oa, const uint64_t* da, const int* la, int ob, const uint64_t* db, const int* lb,
                   const int* lc);

// ------------------------------------------------------------------ kernels (launchers)
constexpr int kMaxOrder = LCO_MAX_ORDER;

// Parameters for recomputing LIVs in a new lexicographical order (the LIV shuffle).
struct ShuffleParams {
  int order = 0;
  FastDiv dim[kMaxOrder];        // old dimensions, least significant first
  uint64_t new_weight[kMaxOrder];  // weight of old mode q in the new LIV
  // When every dimension is a power of two the shuffle only moves bit fields:
  // old mode q is bits [in_shift[q], in_shift[q] + log2 dim) of the old LIV and
  // lands at bit out_shift[q] of the new one.
  int all_pow2 = 0;
  uint32_t in_shift[kMaxOrder] = {}, out_shift[kMaxOrder] = {};
  uint64_t in_mask[kMaxOrder] = {};
};
ShuffleParams make_shuffle(int order, const uint64_t* dims, const uint64_t* new_weight_of_input_mode);

// Key of an element for the radix passes: key = (x / key_div) - key_base.
struct KeyParams {
  FastDiv key_div;
  uint64_t key_base = 0;
};

// exclusive scans; `total` (device, may be null) receives the sum
void scan_u32(lco_ctx ctx, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total);
void scan_u64(lco_ctx ctx, const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total);
// 64-bit prefix sums of 32-bit values.
void scan_u32_u64(lco_ctx ctx, const uint32_t* in, uint64_t* out, int64_t n, uint64_t* total);

// Stable LSD radix sort of (livs, vals) pairs by bits [0, bits) of the element key.
// If `shuffle` is non-null, the input LIVs are first recomputed (pass 1 reads old
// LIVs and writes new ones).  Output goes to (out_livs, out_vals); input is untouched.
void radix_sort_pairs(lco_ctx ctx, const uint64_t* in_livs, const double* in_vals, uint64_t* out_livs,
                      double* out_vals, int64_t n, const ShuffleParams* shuffle, const KeyParams& key, int bits,
                      int digit_cap);
// LIV shuffle without reordering (identity order or single-valued key).
void shuffle_copy(lco_ctx ctx, const uint64_t* in_livs, const double* in_vals, uint64_t* out_livs,
                  double* out_vals, int64_t n, const ShuffleParams* shuffle);
// Segmented permutation: returns false (and does nothing) if a segment exceeds the tile capacity.
// With `small_first`, segments are first assumed to hold at most 32 entries each
// and are ranked directly; a longer segment sends the whole permutation to the
// tile sort.  With `half_first`, the tile sort first tries half-size tiles
// (4096 entries) and falls back to full ones (8192) when a tile overflows.
bool segmented_permute(lco_ctx ctx, const uint64_t* in_livs, const double* in_vals, uint64_t* out_livs,
                       double* out_vals, int64_t n, const ShuffleParams& shuffle, const FastDiv& seg_div,
                       const FastDiv& key_div, uint64_t key_range, bool small_first, bool half_first);
int default_digit_cap();

// permutation of a tensor's storage according to a plan
void permute_storage(lco_ctx ctx, const lco_tensor_s* in, const RpDetail& plan, uint64_t* out_livs,
                     double* out_vals);
// a new tensor holding `in` permuted (output mode r is input mode perm[r])
lco_tensor permuted(lco_ctx ctx, const lco_tensor_s* in, const int* perm);
// c = alpha*a + beta*b of two sorted tensors in the same mode order (the merge
// of their LIV lists); returns a new tensor with dimensions `dims`
lco_tensor add_merge(lco_ctx ctx, double alpha, const lco_tensor_s* a, double beta, const lco_tensor_s* b, int order,
                     const uint64_t* dims);
// lco_add after planning: permutes the operands that need it, then merges
lco_tensor add_run(lco_ctx ctx, double alpha, const lco_tensor_s* a, double beta, const lco_tensor_s* b,
                   const AddDetail& d);

}  // namespace lco
