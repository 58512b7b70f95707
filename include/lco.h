/*
 * lco.h -- C-ABI of the MI355X (gfx950) library for sparse tensors in the
 * linearised-coordinate (LCO) format: construction, mode permutation by radix
 * permutation, and contraction by the multiplication poly-algorithm.
 *
 * The operations follow Harrison & Joseph, "High Performance Rearrangement and
 * Multiplication Routines for Sparse Tensor Arithmetic":
 *   - LCO tensor (Section 3.1): a list of linearised index values (LIVs), one
 *     unsigned 64-bit integer per non-zero, strictly increasing, with a parallel
 *     list of FP64 values.  Default lexicographical order: the first mode is the
 *     least significant, LIV = c0 + n0*(c1 + n1*(c2 + ...)).
 *   - Permutation (Section 4): re-sorting already-sorted data into another
 *     lexicographical order, done here by radix permutation (RP).
 *   - Contraction (Sections 2 and 5): Einstein-notation products of two
 *     tensors, executed as matricise -> convert to a multiplication datatype
 *     and multiply -> map back, with the algorithm chosen from the paper's
 *     table of sparsity combinations (Section 5.2, Table "Multiplication
 *     possibilities based on sparse characteristics of operands").
 *   - Addition (Sections 2 and 3.2): the sum of two tensors over the same
 *     labelled modes, as a permutation of the operand not yet in the output's
 *     order followed by a merge of the two sorted lists.
 *
 * Conventions shared by every entry point
 *   - Every function returns an lco_status; no exception crosses the ABI.  On
 *     error no output handle is produced (the out-pointer is set to NULL),
 *     scratch memory is released, and lco_last_error() describes the cause.
 *     Argument errors are detected on the host before any device work.
 *   - "device" pointers address HIP device memory of the context's device;
 *     "host" pointers address ordinary host memory.
 *   - All device work is enqueued on the context's stream.  Entry points that
 *     must learn a data-dependent size (lco_create, lco_contract, lco_add) wait
 *     on the host for the stream's work up to that point (a device-written
 *     flag in pinned memory) before they allocate their output; the kernels
 *     that fill it may still be running when they return.  lco_permute does
 *     not wait.
 *   - Tensors are owned by the caller and released with lco_destroy, which must
 *     happen before the context that made them is destroyed.  Inputs are never
 *     modified.  An input may come from any context on the same device; work
 *     that produced it on another stream must be complete (or ordered before
 *     the call by the caller).
 *   - LIVs are unsigned: the product of a tensor's dimensions may be anything up
 *     to and including 2^64 (the paper limits itself to signed 63-bit LIVs).
 *   - At most LCO_MAX_ORDER modes per tensor; at most 2^32-1 non-zeros per
 *     tensor and per intermediate product list.
 */
#ifndef LCO_H
#define LCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LCO_MAX_ORDER 16

typedef enum {
  LCO_OK = 0,
  LCO_E_ARG = 1,         /* malformed argument: NULL pointer, bad permutation, bad labels, coordinate out of range */
  LCO_E_OVERFLOW = 2,    /* product of dimensions exceeds 2^64 */
  LCO_E_SHAPE = 3,       /* contracted modes of different dimension */
  LCO_E_UNSORTED = 4,    /* LCO_SORTED input whose LIVs are not strictly increasing */
  LCO_E_DUPLICATE = 5,   /* repeated coordinate without LCO_SUM_DUPLICATES */
  LCO_E_OOM = 6,         /* the allocator returned NULL */
  LCO_E_UNSUPPORTED = 7, /* valid request outside what this library implements (see each call) */
  LCO_E_HIP = 8          /* a HIP runtime call failed */
} lco_status;

typedef struct lco_ctx_s* lco_ctx;
typedef struct lco_tensor_s* lco_tensor;

/* Device allocator callbacks.  alloc returns device memory of at least `bytes`
 * bytes usable in stream order on `stream` (NULL on failure); free releases it
 * in stream order.  `user` is passed through unchanged. */
typedef void* (*lco_alloc_fn)(void* user, size_t bytes, void* stream);
typedef void (*lco_free_fn)(void* user, void* ptr, size_t bytes, void* stream);

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  If alloc/free are NULL the library
 * allocates with hipMalloc and keeps the blocks its tensors and scratch
 * release for reuse in the order of the context's stream (at most 32 GiB
 * cached; lco_ctx_destroy returns them).  Tensors of a context are destroyed
 * before it.  *out receives the handle. */
lco_status lco_ctx_create(int device, void* hip_stream, lco_alloc_fn alloc, lco_free_fn free_fn, void* user,
                          lco_ctx* out);
/* Destroy a context (waits for its stream first). */
lco_status lco_ctx_destroy(lco_ctx ctx);
/* Redirect subsequent work of the context to another stream of the same device
 * (waits for the old stream first). */
lco_status lco_ctx_set_stream(lco_ctx ctx, void* hip_stream);
/* Block until all work enqueued by the context has finished: the host spins
 * for up to 20 ms, then waits in a stream synchronisation.  Reports an error
 * that a kernel recorded (LCO_E_HIP otherwise). */
lco_status lco_ctx_synchronize(lco_ctx ctx);

/* Crossovers of the selector.  The paper's table (Section 5.2) picks a cell
 * and an orientation from the operands' hyper-sparsity classes (ratio of a
 * matricised dimension to the non-zeros above 3).  Sections 5.2.3-5.2.5
 * measure where each specialised algorithm actually starts to win against CSC
 * (about 10 for DCSC, 3 for CSCNA, 6 for SOP on the paper's CPU).  A
 * context's selector keeps the table's classes, cell and orientation and
 * refines the cell's choice with three crossovers: a chosen DCSC/DCSR gives
 * way to CSC/CSR (same orientation) while the operand's relevant
 * hyper-sparsity (A's columns, B's rows) is at most `doubly_compressed`;
 * CSCNA/CSRNA to CSC/CSR while A's rows / B's columns are at most
 * `no_accumulator`; the index-sparse x index-sparse cell's algorithm to CSC or
 * CSR (fewest rearrangements, then n > m) while the smallest of the four
 * ratios is at most `outer_product`.  Above that, that cell runs SOP (the
 * paper's table) or DCSC/DCSR in the same orientation (see
 * lco_ctx_set_index_algorithm).  Crossovers of 3 and SOP in the index cell are
 * the paper's table unchanged.  A new context starts with the values measured
 * on MI355X (LCO_MI355X_*).  Every algorithm sums each output in the same
 * order, so only the speed changes.  Applies to lco_contract, lco_plan_info,
 * batches, batch plans and servers made on this context.  Errors: LCO_E_ARG
 * (NULL, or a value below 3 or not finite). */
lco_status lco_ctx_set_crossovers(lco_ctx ctx, double doubly_compressed, double no_accumulator,
                                  double outer_product);
lco_status lco_ctx_get_crossovers(lco_ctx ctx, double* doubly_compressed, double* no_accumulator,
                                  double* outer_product);
/* The algorithm of the index-sparse x index-sparse cell above the
 * `outer_product` crossover: LCO_ALG_SOP (the paper's table, Section 5.2.5) or
 * the doubly compressed accumulator algorithms (LCO_ALG_DCSC or LCO_ALG_DCSR;
 * either selects the pair, oriented as above).  The getter reports
 * LCO_ALG_SOP or LCO_ALG_DCSC.  Errors: LCO_E_ARG (NULL, another algorithm). */
lco_status lco_ctx_set_index_algorithm(lco_ctx ctx, int algo);
lco_status lco_ctx_get_index_algorithm(lco_ctx ctx, int* algo);
/* The selector measured on MI355X with the paper's R-TENSOR sweeps (the
 * benchmark's calibration leg): DCSC overtakes CSC above a column-sparsity of
 * about 10 (the two are within a few percent between 6 and 25); CSCNA and CSC
 * take the same time at every row-sparsity (the accumulator is a per-row LDS
 * table here, not a dense array of the row count), so NA keeps the paper's 3;
 * in the index-sparse cell DCSC beats SOP above an index-sparsity of about 19
 * and CSC above about 30 (within a few percent of CSC from 5 to 100), and on
 * the 2^16-per-mode Kronecker pair runs in 7.4 ms against SOP's 14.8 ms. */
#define LCO_MI355X_DC_CROSSOVER 10.0
#define LCO_MI355X_NA_CROSSOVER 3.0
#define LCO_MI355X_INDEX_CROSSOVER 30.0
#define LCO_MI355X_INDEX_ALGORITHM LCO_ALG_DCSC

/* Per-kernel timing with HIP events recorded on the context's stream around
 * every launch of the library's kernels (off by default; costs two events per
 * launch).  lco_timing_query sums over all launches of kernels whose name
 * equals `kernel` since the last reset: *launches, *total_ms.  Timing of a
 * launch is collected lazily at query time. */
lco_status lco_timing_enable(lco_ctx ctx, int on);
/* Restricts timing to launches of the kernel named `kernel` (copied; NULL or
 * "" times every kernel again).  Each timed launch adds two event records to
 * the stream, which costs a few microseconds of device time per launch, so a
 * caller that needs one kernel's duration times only that one.  Errors:
 * LCO_E_ARG when ctx is NULL. */
lco_status lco_timing_only(lco_ctx ctx, const char* kernel);
lco_status lco_timing_reset(lco_ctx ctx);
lco_status lco_timing_query(lco_ctx ctx, const char* kernel, int64_t* launches, double* total_ms);
/* Name of the i-th distinct kernel seen by the timer (NULL past the end). */
const char* lco_timing_kernel_name(lco_ctx ctx, int i);

/* ------------------------------------------------------------------ tensors */

#define LCO_SORTED 0x1u          /* d_idx holds LIVs, claimed strictly increasing (verified: LCO_E_UNSORTED) */
#define LCO_COORDS 0x2u          /* d_idx holds nnz*order coordinates, entry-major (entry i: d_idx[i*order + r]) */
#define LCO_SUM_DUPLICATES 0x4u  /* repeated coordinates are summed, in input order; else LCO_E_DUPLICATE */

/* Build an LCO tensor (Section 3.1) of order `order` (0..LCO_MAX_ORDER) and
 * dimensions `dims` (host, `order` entries, each >= 1, product <= 2^64) from
 * `nnz` entries.  `d_idx` (device) holds either LIVs in the default order
 * (default) or coordinates (LCO_COORDS); `d_vals` (device) holds nnz FP64
 * values.  Unsorted input is sorted (stable LSD radix sort on the full LIV);
 * explicit zeros are kept.  The tensor copies the data (the caller keeps
 * ownership of d_idx/d_vals).  Errors: LCO_E_ARG (coordinate or LIV out of
 * range, bad order), LCO_E_OVERFLOW, LCO_E_UNSORTED, LCO_E_DUPLICATE, LCO_E_OOM. */
lco_status lco_create(lco_ctx ctx, int order, const uint64_t* dims, int64_t nnz, const uint64_t* d_idx,
                      const double* d_vals, uint32_t flags, lco_tensor* out);

/* Release a tensor's device memory (stream-ordered) and its handle. */
lco_status lco_destroy(lco_tensor t);

/* Copy a tensor's nnz LIVs and values into host arrays `livs` / `vals` (each
 * with room for lco_nnz(t) entries; either may be NULL to skip it).  Blocking:
 * waits for the tensor's context stream, then copies. */
lco_status lco_read(lco_tensor t, uint64_t* livs, double* vals);

int64_t lco_nnz(lco_tensor t);
int lco_order(lco_tensor t);
/* Host array of `order` dimensions, owned by the tensor. */
const uint64_t* lco_dims(lco_tensor t);
/* Device arrays of nnz LIVs / values, owned by the tensor (NULL when nnz == 0). */
const uint64_t* lco_livs(lco_tensor t);
const double* lco_vals(lco_tensor t);

/* -------------------------------------------------------------- permutation */

/* Radix permutation (Section 4.1).  Output mode r is input mode perm[r]
 * (host array of `order` distinct indices); the output has dimensions
 * dims[perm[r]] and is sorted in its default order -- identical to re-sorting
 * the input into the lexicographical order that makes input mode perm[r] the
 * r-th least significant.  Only the digit groups the permutation disturbs are
 * sorted (stable LSD passes over the truncated key between the shared leading
 * resting modes and the trailing resting modes).  Values are copied
 * bit-exactly.  No host synchronisation except on the segmented path (a
 * common leading resting mode), which reads back the largest segment size.
 * Errors: LCO_E_ARG (not a permutation), LCO_E_OOM. */
lco_status lco_permute(lco_ctx ctx, lco_tensor in, const int* perm, lco_tensor* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * lco_permute that writes into caller-owned device arrays and takes every
 * temporary buffer from a fixed workspace of LCO_NOALLOC_SCRATCH_BYTES inside
 * the library (one per device, set up by lco_ctx_create on that device and
 * held until the process ends).  out_livs / out_vals: device arrays of
 * in->nnz entries each (unused when nnz is 0) that receive the permuted
 * tensor in its default order; out_dims: host array of `order` entries that
 * receives dims[perm[r]].  The result equals lco_permute's bit for bit.  Calls
 * that overlap on one device (several streams or threads) race on the shared
 * workspace; the workspace keeps the last call's contents, and every call
 * clears what it needs.  Errors: those of lco_permute, and
 * LCO_E_UNSUPPORTED when nnz exceeds LCO_NOALLOC_MAX_NNZ. */
#define LCO_NOALLOC_MAX_NNZ (1 << 20)
#define LCO_NOALLOC_SCRATCH_BYTES (24u << 20)
lco_status lco_permute_noalloc(lco_ctx ctx, lco_tensor in, const int* perm, uint64_t* out_livs, double* out_vals,
                               uint64_t* out_dims);

/* -------------------------------------------------------------- contraction */

/* Sparsity classes of a matricised operand (Section 5.1): a dimension is
 * "hyper-sparse" when it exceeds three times the number of non-zeros
 * (Sections 5.2.3-5.2.5 use the ratio dimension/nnz > 3). */
typedef enum { LCO_SPARSE = 0, LCO_ROW_SPARSE = 1, LCO_COL_SPARSE = 2, LCO_INDEX_SPARSE = 3 } lco_sparsity;

/* Multiplication algorithms (Section 5.2); the value is also the "force"
 * field of lco_contract's flags. */
typedef enum {
  LCO_ALG_AUTO = 0,
  LCO_ALG_CSC = 1,   /* column-by-column with accumulator, A compressed by columns */
  LCO_ALG_CSR = 2,   /* row-by-row with accumulator, B compressed by rows */
  LCO_ALG_DCSC = 3,  /* as CSC with A doubly compressed (only non-empty columns) */
  LCO_ALG_DCSR = 4,  /* as CSR with B doubly compressed (only non-empty rows) */
  LCO_ALG_CSCNA = 5, /* column-by-column, no accumulator: products sorted and summed */
  LCO_ALG_CSRNA = 6, /* row-by-row, no accumulator */
  LCO_ALG_SOP = 7    /* simple outer product: all rank-1 products sorted and summed */
} lco_algo;

#define LCO_FORCE_MASK 0xFu  /* flags & LCO_FORCE_MASK = lco_algo to force (0 = choose by the table) */

typedef struct {
  uint64_t m, k, n;                 /* A is m x k, B is k x n after matricisation */
  int64_t nnz_a, nnz_b;
  int a_class, b_class;             /* lco_sparsity of A and B */
  int algo;                         /* lco_algo that runs */
  int permute_a, permute_b;         /* 1 if that operand is rearranged before multiplying */
  int permute_c;                    /* 1 if the product is rearranged into c_labels order */
  int num_contracted;               /* number of contracted labels */
  int num_entrywise;                /* number of entrywise labels (in a, b and the output) */
} lco_plan;

/* Einstein-notation product (Section 2; Section 5.2's three steps).
 * `a_labels` / `b_labels` (host) name the modes of a and b; `c_labels` (host,
 * c_order entries, 0 <= c_order) name the output modes in output order.  A
 * label in both inputs and not in the output is contracted; a label in exactly
 * one input and in the output is free; a label in both inputs and in the output
 * is entrywise: entries are multiplied only where they agree on it, and it is
 * not summed (batched products such as c_hik = a_hij b_hjk; the product is then
 * block diagonal, and the operand on the engine's row side is re-sorted into
 * that form).  Each output entry sums its products in ascending order of the
 * contracted index (contracted modes linearised in the order they occur in a),
 * starting from 0.0; every structural non-zero is kept.
 * flags & LCO_FORCE_MASK forces an lco_algo instead of the table's choice.
 * Synchronises the stream once per data-dependent size (output nnz; product
 * count for the outer-product and long-row paths).
 * Errors: LCO_E_ARG (labels malformed, label repeated within an operand or in
 * the output), LCO_E_SHAPE (contracted or entrywise modes of different
 * dimensions), LCO_E_OVERFLOW (output dimension product > 2^64),
 * LCO_E_UNSUPPORTED (a free label absent from the output, a matricised side of
 * 2^64 or more, or a block-diagonal operand form beyond 2^64), LCO_E_OOM. */
lco_status lco_contract(lco_ctx ctx, lco_tensor a, const int* a_labels, lco_tensor b, const int* b_labels,
                        int c_order, const int* c_labels, uint32_t flags, lco_tensor* out);

/* ----------------------------------------------------------------- addition */

/* Sparse addition (Section 2: the design tensor there is a sum of two products;
 * Section 3.2: before two terms can be added, one must be re-sorted into the
 * other's lexicographical order).  c = alpha*a + beta*b, where a and b have the
 * same order and `a_labels`, `b_labels` and `c_labels` (host, that many entries
 * each) name the same set of distinct labels; modes with the same label must
 * have the same dimension.  Output mode r is the mode labelled c_labels[r]; the
 * output is sorted in its default order.  An operand whose label order differs
 * from c_labels is first permuted (as by lco_permute); the two sorted lists are
 * then merged.  An LIV present in both operands gets alpha*a + beta*b (two
 * rounded products, then one rounded sum); an LIV present in one operand gets
 * that operand's value times its coefficient.  The pattern is the union of the
 * two patterns, whatever the values (a - a keeps every position, at 0.0).
 * Synchronises once to learn the output size.  Errors: LCO_E_ARG (NULL
 * argument, different orders, repeated labels, label lists naming different
 * sets), LCO_E_SHAPE (same label, different dimensions), LCO_E_UNSUPPORTED
 * (more than 2^32-1 entries in the two operands together), LCO_E_OOM. */
lco_status lco_add(lco_ctx ctx, double alpha, lco_tensor a, const int* a_labels, double beta, lco_tensor b,
                   const int* b_labels, const int* c_labels, lco_tensor* out);

/* One product of a batch (the arguments of lco_contract). */
typedef struct {
  lco_tensor a;
  const int* a_labels;
  lco_tensor b;
  const int* b_labels;
  int c_order;
  const int* c_labels;
  uint32_t flags;
} lco_contract_desc;

/* Batched products: outs[i] receives the product of descs[i], bit-identical to
 * what lco_contract returns for the same arguments (Section 5.2's three steps,
 * applied per instance).  Instances whose plan is CSR/CSC/CSRNA/CSCNA (after
 * any operand rearrangement) and that have no entrywise label are batched.
 * Those whose rows of A' are listed densely (at most 2 nnz(A') + 64 rows and at
 * most 2^20 of them, at most 2^21 A' entries, k' < 2^34) run in the persistent
 * engine when there are at least 32 of them (fewer run in the chunked engine
 * below): one launch of a persistent grid computes every instance's multiplication datatype, symbolic
 * counts and output offsets from a device work queue, one host synchronisation
 * reads the output sizes, and a second persistent launch writes every
 * instance's product.  The other batched instances run in the chunked engine:
 * chunks of at most 2^26 A' entries, one launch per phase over all the
 * instances of a chunk.  Outputs of batched instances share
 * device allocations that are released with the last of their tensors.  An
 * instance with a row of more than 64 products or entries, and every
 * instance that is not batched (doubly compressed, outer product, entrywise),
 * runs through the per-call path.  Errors are those of lco_contract; on error
 * no output handle survives. */
lco_status lco_contract_batch(lco_ctx ctx, int count, const lco_contract_desc* descs, lco_tensor* outs);
/* How many instances of the last lco_contract_batch call ran batched / per
 * call, and how many of the batched ones ran in the persistent engine
 * (`persistent` may be NULL). */
lco_status lco_batch_stats(lco_ctx ctx, int64_t* batched, int64_t* per_call, int64_t* persistent);

/* Planned batches.  lco_batch_plan_create does the shape-dependent host work
 * of a batch once -- operand and output rearrangements (kept as value
 * gathers), the output sizes and one device allocation holding every output --
 * and computes the outputs.  lco_batch_plan_execute then recomputes the whole
 * batch from the operands' current values: the value gathers and ONE launch of
 * the persistent engine, which rebuilds every instance's multiplication
 * datatype, counts its rows, places them and writes the products (the same
 * offsets every time), with no allocation and no host synchronisation, so it
 * can be captured in a HIP graph; lco_batch_plan_graph_launch captures it once
 * into a graph owned by the plan and replays that graph.  The operands' LIVs
 * (sparsity patterns) must not change after planning; their values may.
 *
 * While planning, an autotuner picks for every size bucket (A' non-zeros
 * within a factor of 4) the row-engine branch (accumulator or sort-based, both
 * of which sum every output in the same order, so the result does not depend
 * on the choice) and the number of 64-row chunks per work item of the
 * persistent engine, by timing the candidates on the bucket's own instances;
 * choices are kept in the context and reused by later plans and by
 * lco_contract_batch.
 *
 * Only instances that the persistent engine runs completely (row-wise or
 * column-wise singly compressed products without entrywise labels, rows of A'
 * listed densely, within its size limits above, every row with at most 64
 * products and entries) can be planned; others give LCO_E_UNSUPPORTED.  The outputs belong to the plan
 * (lco_batch_plan_output returns borrowed handles, valid until
 * lco_batch_plan_destroy). */
typedef struct lco_batch_plan_s* lco_batch_plan;
lco_status lco_batch_plan_create(lco_ctx ctx, int count, const lco_contract_desc* descs, lco_batch_plan* out);
/* Borrowed handle of the i-th output (NULL if i is out of range). */
lco_tensor lco_batch_plan_output(lco_batch_plan p, int i);
lco_status lco_batch_plan_execute(lco_ctx ctx, lco_batch_plan p);
lco_status lco_batch_plan_graph_launch(lco_ctx ctx, lco_batch_plan p);
/* The i-th size bucket of the plan: the bucket (floor(log2(nnz of A'))/2), its
 * instances, the chosen branch (LCO_ALG_CSR = accumulator, LCO_ALG_CSRNA =
 * sort-based), 64-row chunks per work item, and the measured time of the
 * bucket's numeric phase with that choice (0 when it came from an earlier
 * plan).  LCO_E_ARG past the last bucket. */
lco_status lco_batch_plan_launch_info(lco_batch_plan p, int i, int* bucket, int* instances, int* algo,
                                      int* group, double* ms);
lco_status lco_batch_plan_destroy(lco_batch_plan p);

/* ------------------------------------------------------------------ serving
 *
 * A request server for contractions (continuous batching).  Requests are
 * submitted as they arrive; `workers` threads each own a HIP stream (default
 * priority) and a context that keeps its released device blocks for reuse.  A
 * worker that becomes free takes every pending request that fits -- in arrival
 * order, up to `max_batch`, while the sum of their estimated device footprints
 * stays within `hbm_budget` bytes -- and runs them as one lco_contract_batch;
 * requests that arrive meanwhile wait for the next free worker, so batches of
 * different workers overlap on the device.  Requests whose plan is not a
 * row-engine product (doubly compressed, outer product) or whose operands hold
 * more than `solo_nnz` non-zeros are run in a batch of their own.  With
 * `plain` set every request runs alone through lco_contract (the serial
 * baseline when workers == 1).  Results are bit-identical to lco_contract on
 * the same operands whatever the batch they ran in.
 *
 * Operands may belong to any context on the server's device; the caller
 * guarantees that they are complete (their context synchronised) when
 * submitted and that they live until the request completes.  Result tensors
 * belong to the caller (lco_destroy, before lco_server_destroy); their LIVs and
 * values are read with lco_read. */
typedef struct lco_server_s* lco_server;

typedef struct {
  int workers;          /* >= 1 */
  int max_batch;        /* >= 1 */
  int plain;            /* 0 or 1 */
  int64_t solo_nnz;     /* operands with more non-zeros (nnz_a + nnz_b) run alone; <= 0: never */
  uint64_t hbm_budget;  /* bytes; a request above the whole budget runs when nothing else is in flight */
} lco_server_config;

typedef struct {
  int64_t ticket;       /* from lco_server_submit */
  lco_status status;    /* the request's own result */
  lco_tensor out;       /* the product (NULL on error) */
  double latency_ms;    /* submission -> result complete on the device */
  double queue_ms;      /* submission -> its batch started */
  int batch_size;       /* requests in the batch it ran in */
} lco_server_result;

lco_status lco_server_create(int device, const lco_server_config* cfg, lco_server* out);
/* Enqueue a product (arguments as lco_contract; label arrays are copied).
 * *ticket receives the request's number (0, 1, 2, ... in submission order). */
lco_status lco_server_submit(lco_server s, const lco_contract_desc* desc, int64_t* ticket);
/* Non-blocking: moves up to `cap` completed requests into results[] and sets
 * *count to how many. */
lco_status lco_server_poll(lco_server s, lco_server_result* results, int cap, int* count);
/* Block until every submitted request has completed (they stay pollable). */
lco_status lco_server_drain(lco_server s);
/* Drain, join the workers, release results never polled, destroy the server. */
lco_status lco_server_destroy(lco_server s);

/* The plan lco_contract would run for these operands, without running it. */
lco_status lco_plan_info(lco_ctx ctx, lco_tensor a, const int* a_labels, lco_tensor b, const int* b_labels,
                         int c_order, const int* c_labels, uint32_t flags, lco_plan* out);

/* ------------------------------------------------- host-only planning logic */

/* Classify an m x k matricised operand with nnz non-zeros (Section 5.2: row-
 * sparse iff rows/nnz > 3, column-sparse iff cols/nnz > 3, index-sparse iff both). */
lco_status lco_classify(uint64_t rows, uint64_t cols, int64_t nnz, int* cls);

/* The cell of the paper's multiplication table for operand classes
 * (a_class, b_class): *first and *second receive the algorithm(s) named in the
 * cell (equal when the cell names one; CSC-family first when it names two). */
lco_status lco_select(int a_class, int b_class, int* first, int* second);

/* The same plan as lco_plan_info from shapes alone (host arrays; no device). */
lco_status lco_plan_contract(int a_order, const uint64_t* a_dims, const int* a_labels, int64_t a_nnz, int b_order,
                             const uint64_t* b_dims, const int* b_labels, int64_t b_nnz, int c_order,
                             const int* c_labels, uint32_t flags, lco_plan* out);

/* Radix-permutation plan (Section 4.1): classification of the modes into
 * rearrangement and resting indices and the truncated key that must be sorted. */
typedef struct {
  int identity;            /* 1: the permutation leaves every LIV order unchanged (plain copy + LIV shuffle) */
  int prefix;              /* leading (most significant) modes shared by the old and new orders: segments */
  int suffix;              /* trailing (least significant) new-order modes left out of the key */
  uint32_t rearrangement;  /* bit q set iff input mode q is a rearrangement index */
  int key_bits;            /* bits of the truncated key (the modes between prefix and suffix) */
  int seg_bits;            /* bits of the segment id (prefix modes) */
  int full_bits;           /* bits of the whole LIV range */
  int method;              /* 0 copy, 1 single-tile LDS sort, 2 global LSD on the key, 3 segmented LDS sort,
                              4 global LSD on segment and key */
  int passes;              /* radix passes of the chosen method */
  int digit_bits;          /* bits per radix pass */
  uint64_t key_div;        /* new-LIV divisor removing the suffix modes */
  uint64_t key_range;      /* number of distinct key values (product of the keyed dimensions) */
  uint64_t seg_div;        /* old-LIV divisor whose quotient is the segment id */
} lco_rp_plan;

lco_status lco_plan_permute(int order, const uint64_t* dims, const int* perm, int64_t nnz, lco_rp_plan* out);

/* Host run of the library's invariant-divisor division (Granlund & Montgomery,
 * 1994, "Division by invariant integers using multiplication", Fig. 4.1) used
 * by the kernels for LIV decoding: quot[i] = num[i] / d, rem[i] = num[i] % d. */
lco_status lco_fastdiv_host(uint64_t d, int64_t count, const uint64_t* num, uint64_t* quot, uint64_t* rem);

/* --------------------------------------------------------------- diagnostics */

const char* lco_status_str(lco_status s);
/* Message of the last error raised on the calling thread ("" if none). */
const char* lco_last_error(void);
/* Library version string. */
const char* lco_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LCO_H */
