// Shared declarations of the multiplication kernels (row-wise engine and outer product).
#pragma once

#include <vector>

#include "lco_internal.h"

namespace lco {

// Non-empty groups of a sorted LIV array, group id = LIV / div (device arrays
// sized for the worst case; the group count lives on the device).
struct Segments {
  uint64_t* ids = nullptr;     // group ids, ascending
  uint32_t* starts = nullptr;  // first entry of each group, plus a terminal entry
  uint64_t* count = nullptr;   // device word: number of groups
};
Segments segment_livs(lco_ctx ctx, Scratch& s, const uint64_t* livs, int64_t n, const FastDiv& div);

// Arguments of the row-wise product kernels (see k_rows.hip for the layout).
struct RowArgs {
  const uint64_t* a_livs = nullptr;
  const double* a_vals = nullptr;
  int64_t nnz_a = 0;
  const uint64_t* b_livs = nullptr;
  const double* b_vals = nullptr;
  int64_t nnz_b = 0;
  FastDiv kdiv;          // k': row of A' = LIV / k'
  uint64_t kp = 1, np = 1;
  const uint32_t* bptr = nullptr;        // singly compressed B': k'+1 row starts
  const ulonglong2* dc_tab = nullptr;    // doubly compressed B': hash table of its non-empty rows,
  uint64_t dc_mask = 0;                  //   slots {row id, start | length << 32}, dc_mask + 1 of them,
  int dc_shift = 64;                     //   home slot dc_home(id, dc_shift), linear probing
  const uint32_t* row_start = nullptr;   // non-empty rows of A': starts (plus terminal)
  const uint64_t* row_id = nullptr;      //   and ids (nullptr: row r of the list is row r of A')
  const uint64_t* nzr_a = nullptr;       //   device count
  const uint32_t* elen = nullptr;        // products per A' entry (nnz_a; a B' row length, below 2^32)
  const uint64_t* poff = nullptr;        // exclusive prefix of products per A' entry (nnz_a + 1)
  const uint32_t* bstart = nullptr;      // first B' entry of the row each A' entry selects
};

// Doubly compressed B' table: the id of an empty slot (row ids are below k' <= 2^64 - 1)
// and a row id's home slot (Fibonacci hashing: the top bits of id * 2^64/phi).
constexpr uint64_t kDcEmpty = ~0ull;
__device__ __forceinline__ uint64_t dc_home(uint64_t id, int shift) { return (id * 0x9E3779B97F4A7C15ull) >> shift; }

// Row of A' at position r of the row list.
__device__ __forceinline__ uint64_t row_of(const RowArgs& ra, uint64_t r) { return ra.row_id ? ra.row_id[r] : r; }

// C' = A' * B' row by row; `dense` selects singly (CSR) or doubly (DCSR)
// compressed B', `acc` the sparse accumulator (CSR, DCSR) or none (CSRNA).
lco_tensor row_engine(lco_ctx ctx, const lco_tensor_s* A, const lco_tensor_s* B, uint64_t mp, uint64_t kp,
                      uint64_t np, bool dense, bool acc, int out_order, const uint64_t* out_dims);

// One instance of a batch, in the row-engine roles (A' row-major, B' singly compressed).
struct BatchJob {
  int index;              // position in the caller's batch
  const lco_tensor_s* A;  // A'
  const lco_tensor_s* B;  // B'
  uint64_t kp, np;
  int order_c;
  uint64_t natural_dims[LCO_MAX_ORDER];
};
// Rows in flight per workgroup of the one-wave-per-row kernels (one wave each).
constexpr int kRowWaves = 4;

// A batch runs in chunks of at most this many A' entries in total.
constexpr int64_t kBatchChunkEntries = int64_t(1) << 26;

// Device buffers that outlive one call (those of a batch plan), released together.
struct KeptBuffers {
  lco_ctx ctx = nullptr;
  std::vector<std::pair<void*, size_t>> bufs;
  void* raw(size_t bytes);
  template <class T> T* get(size_t count) { return static_cast<T*>(raw(count * sizeof(T) + 1)); }
  void release();
};

// Everything the numeric pass of one batch group reads and writes.
struct BatchLaunch {
  bool acc = true;
  bool narrow = false;  // every instance has columns below 2^32
  int grid = 1;
  int chunk_rows = 1;  // consecutive rows per wave visit
  uint32_t rows = 0;
  const void* inst = nullptr;  // device array of per-instance descriptors
  const uint32_t* rs = nullptr;
  const uint64_t* rid = nullptr;
  const uint32_t* rinst = nullptr;
  const uint8_t* shape = nullptr;
  const uint32_t* fallback = nullptr;
  const uint64_t* poff = nullptr;
  const uint32_t* bstart = nullptr;
  const uint64_t* coff = nullptr;
  uint64_t* out_livs = nullptr;
  double* out_vals = nullptr;
};
// dst[i] = src[idx[i]] for i < n, and out[i] = i (value-permutation helpers of batch plans).
void gather_values(lco_ctx ctx, const double* src, const uint64_t* idx, int64_t n, double* dst);
void fill_iota(lco_ctx ctx, uint64_t* out, int64_t n);
// Rows per wave chunk and the grid of the batched row kernels for `rows` rows.
int batch_chunk_rows(lco_ctx ctx, uint64_t rows);
int batch_grid(lco_ctx ctx, uint64_t rows, int chunk_rows, int blocks_per_cu);
// The numeric pass: every batched row recomputed from the operands' current values.
void batch_numeric(lco_ctx ctx, const BatchLaunch& L);

// Runs the jobs (all with or all without accumulator) as one batch; writes
// outs[job.index] for each completed job and returns the indices that need the
// per-call path.  With `keep`, the buffers the numeric pass reads stay
// allocated in `keep` and `*launch` describes that pass, so it can be re-run.
std::vector<int> batch_group(lco_ctx ctx, const std::vector<BatchJob>& jobs, bool acc, lco_tensor* outs,
                             KeptBuffers* keep = nullptr, BatchLaunch* launch = nullptr);

// ---------------------------------------------------------------- persistent batched engine (k_persist.hip)

// Rows of A' per instance up to which an instance runs in the persistent engine
// (each instance's chunk counts are scanned by one wave), and A' entries: the
// engine is for many small and medium products; a larger one keeps the GPU
// busy alone, and its setup phases run faster as separate launches.
constexpr uint64_t kPersistMaxRows = uint64_t(1) << 20;
constexpr int64_t kPersistMaxEntries = int64_t(1) << 21;

// One instance of a persistent batch, in the row-engine roles.
struct PJob {
  int index;              // position in the caller's batch
  const lco_tensor_s* A;  // A' (rows of the product)
  const lco_tensor_s* B;  // B'
  uint64_t mp, kp, np;    // rows of A', contracted size, columns of B'
  bool acc;               // accumulator (CSR/CSC) or none (CSRNA/CSCNA)
  int group;              // 64-row chunks per work item
  int bucket;             // size bucket (autotuner key)
  int order_c;
  uint64_t natural_dims[LCO_MAX_ORDER];
};
// Rows of A' listed densely (few empty rows), sizes within the engine's limits.
bool persist_eligible(uint64_t mp, uint64_t kp, int64_t nnz_a, int64_t nnz_b);

// The device state of a persistent batch: descriptors, work-item tables and
// the per-entry, per-row and per-chunk arrays of every instance (from `s`, or
// kept in `keep` when the batch is re-run).  Launches enqueue on the context's
// stream.
class PersistBatch {
 public:
  PersistBatch(lco_ctx ctx, const std::vector<PJob>& jobs, Scratch* s, KeptBuffers* keep);
  ~PersistBatch();
  PersistBatch(const PersistBatch&) = delete;
  PersistBatch& operator=(const PersistBatch&) = delete;
  // Instances whose numeric phase the following launches run (all, after
  // construction; phases 0-4 always cover every instance), and the work items
  // of every phase from the current chunks-per-item choices.
  void set_items(const std::vector<bool>& active);
  // Branch and chunks per item of instance i; take effect after upload_params() and set_items().
  void set_params(int i, bool acc, int group);
  void upload_params();
  // One reset and one persistent launch running phases [first, last] (0: setup ... 4: output
  // offsets; 5: numeric into the pool of `capacity` entries at out_livs / out_vals).
  void launch(int first, int last, uint64_t* out_livs, double* out_vals, uint64_t capacity);
  // After a launch of phases 0-4: each instance's output size and pool offset, and
  // whether it must take the per-call path (one host synchronisation).
  void read_sizes();
  const std::vector<uint64_t>& sizes() const { return sizes_; }
  const std::vector<uint64_t>& offsets() const { return offsets_; }
  const std::vector<uint32_t>& fallback() const { return fallback_; }
  uint64_t total() const { return total_; }
  int grid() const;

 private:
  struct Dev;
  lco_ctx ctx_;
  Dev* dev_;
  std::vector<uint32_t> pre_;
  std::vector<uint64_t> sizes_, offsets_;
  std::vector<uint32_t> fallback_;
  uint64_t total_ = 0;
};

// Simple outer product (Section 5.2.5) of A (column-major) and B (row-major).
lco_tensor sop_engine(lco_ctx ctx, const lco_tensor_s* A, const lco_tensor_s* B, const ContractDetail& d);

}  // namespace lco
