// Contraction orchestration, following the three steps of Section 5.2:
// (1) map each LCO operand to a matrix, permuting it only if its lexicographical
// order does not already give the layout the chosen algorithm needs;
// (2) build the multiplication datatype and multiply (row engine or SOP);
// (3) map the product back: permute it into the output label order if needed.
#include <algorithm>

#include "rows.h"

namespace lco {

namespace {

struct Owned {  // a temporary tensor released on scope exit
  lco_tensor t = nullptr;
  ~Owned() {
    if (t) lco_destroy(t);
  }
};

}  // namespace

lco_tensor permuted(lco_ctx ctx, const lco_tensor_s* in, const int* perm) {
  RpDetail plan = plan_permute(in->order, in->dims, perm, in->nnz, default_digit_cap());
  lco_tensor t = new_tensor(ctx, in->order, plan.new_dims, in->nnz);
  try {
    permute_storage(ctx, in, plan, t->livs, t->vals);
  } catch (...) {
    lco_destroy(t);
    throw;
  }
  return t;
}

// An operand re-sorted into its block-diagonal matricised form (entrywise modes
// counted with its rows and with its columns): the LIV shuffle takes arbitrary
// weights, and the sort runs over the whole new LIV.  The result is a plain
// array of (LIV, value) pairs handed to the engines (its "dims" are the two
// matricised sides).
lco_tensor block_diagonal(lco_ctx ctx, const lco_tensor_s* in, const ContractDetail& d) {
  lco_tensor t = new_tensor(ctx, 2, d.dup_dims, in->nnz);
  try {
    if (in->nnz) {
      const ShuffleParams sp = make_shuffle(in->order, in->dims, d.dup_weight);
      KeyParams kp;
      radix_sort_pairs(ctx, in->livs, in->vals, t->livs, t->vals, in->nnz, &sp, kp, d.dup_bits,
                       default_digit_cap());
    }
  } catch (...) {
    lco_destroy(t);
    throw;
  }
  return t;
}

lco_tensor contract_run(lco_ctx ctx, const lco_tensor_s* a, const lco_tensor_s* b, const ContractDetail& d) {
  if (d.empty) return new_tensor(ctx, d.order_c, d.c_dims, 0);
  Owned ta, tb;
  const lco_tensor_s* A = a;
  const lco_tensor_s* B = b;
  if (d.dup == 1) A = ta.t = block_diagonal(ctx, a, d);
  else if (d.pub.permute_a) A = ta.t = permuted(ctx, a, d.perm_a);
  if (d.dup == 2) B = tb.t = block_diagonal(ctx, b, d);
  else if (d.pub.permute_b) B = tb.t = permuted(ctx, b, d.perm_b);
  Owned natural;
  switch (d.pub.algo) {
    case LCO_ALG_CSR:
    case LCO_ALG_DCSR:
    case LCO_ALG_CSRNA:
      natural.t = row_engine(ctx, A, B, d.em, d.ek, d.en, d.pub.algo != LCO_ALG_DCSR, d.pub.algo != LCO_ALG_CSRNA,
                             d.order_c, d.natural_dims);
      break;
    case LCO_ALG_CSC:
    case LCO_ALG_DCSC:
    case LCO_ALG_CSCNA:
      // column by column: C^T = B^T A^T row by row over the same arrays
      natural.t = row_engine(ctx, B, A, d.em, d.ek, d.en, d.pub.algo != LCO_ALG_DCSC, d.pub.algo != LCO_ALG_CSCNA,
                             d.order_c, d.natural_dims);
      break;
    case LCO_ALG_SOP:
      natural.t = sop_engine(ctx, A, B, d);
      break;
    default:
      fail(LCO_E_ARG, "contract: unknown algorithm");
  }
  if (d.pub.permute_c) return permuted(ctx, natural.t, d.perm_c);
  lco_tensor out = natural.t;
  natural.t = nullptr;
  return out;
}

// Addition: operands whose mode order differs from the output's are permuted
// first (Section 3.2: one term is re-sorted into the other's order), then the
// two sorted lists are merged.
lco_tensor add_run(lco_ctx ctx, double alpha, const lco_tensor_s* a, double beta, const lco_tensor_s* b,
                   const AddDetail& d) {
  Owned ta, tb;
  const lco_tensor_s* A = a;
  const lco_tensor_s* B = b;
  if (d.permute_a && a->nnz) A = ta.t = permuted(ctx, a, d.perm_a);
  if (d.permute_b && b->nnz) B = tb.t = permuted(ctx, b, d.perm_b);
  return add_merge(ctx, alpha, A, beta, B, d.order, d.c_dims);
}

}  // namespace lco

// ---------------------------------------------------------------- batched C-ABI

namespace lco {
lco_status set_error(const Error& e);
lco_status set_error_msg(lco_status s, const char* msg);
}  // namespace lco

using namespace lco;

namespace lco {

// Chunks per work item of the persistent engine when no tuned value is known.
constexpr int kDefaultGroup = 4;
// Instances from which a batch runs in the persistent engine: its phases
// (each with a grid-wide wait) cost about half a millisecond, which a handful
// of products does not amortise; smaller batches (a server's batches of a few
// requests among them) run in the chunked engine, one launch per phase.
constexpr size_t kPersistMinInstances = 32;

// The persistent engine's choice for one instance: the tuned branch and chunks
// per item of its size bucket, else the selector's branch.
void persist_params(lco_ctx ctx, PJob& j, bool selector_acc) {
  j.acc = selector_acc;
  j.group = kDefaultGroup;
  j.bucket = bits_for((uint64_t)j.A->nnz) / 2;
  auto it = ctx->tune.find(j.bucket * 2 + (selector_acc ? 1 : 0));
  if (it != ctx->tune.end()) {
    j.acc = it->second.first != 0;
    j.group = it->second.second;
  }
}

// Runs jobs through the persistent engine: one launch sizes every output (setup,
// symbolic count, scans), one host synchronisation reads the sizes, and one
// launch writes every output into a shared pool.  Fills outs[job.index] and
// returns the indices that need the per-call path.
std::vector<int> persist_group(lco_ctx ctx, const std::vector<PJob>& jobs, lco_tensor* outs) {
  std::vector<int> redo;
  if (jobs.empty()) return redo;
  Scratch s(ctx);
  PersistBatch pb(ctx, jobs, &s, nullptr);
  pb.launch(0, 4, nullptr, nullptr, 0);
  pb.read_sizes();
  const uint64_t total = pb.total();
  if (total > ((uint64_t)1 << 40)) fail(LCO_E_OOM, "batch: output pool beyond 2^40 entries");
  Pool* pool = total ? new_pool(ctx, total * 16) : nullptr;
  uint64_t* pl = pool ? (uint64_t*)pool->base : nullptr;
  double* pv = pool ? (double*)((char*)pool->base + total * 8) : nullptr;
  try {
    if (total) pb.launch(5, 5, pl, pv, total);
    for (size_t i = 0; i < jobs.size(); ++i) {
      const PJob& j = jobs[i];
      if (pb.fallback()[i]) {
        redo.push_back(j.index);
        continue;
      }
      const uint64_t off = pb.offsets()[i], n = pb.sizes()[i];
      outs[j.index] = n ? pool_tensor(ctx, pool, j.order_c, j.natural_dims, pl + off, pv + off, (int64_t)n)
                        : new_tensor(ctx, j.order_c, j.natural_dims, 0);
    }
  } catch (...) {
    if (pool) release_pool(pool);
    throw;
  }
  if (pool) release_pool(pool);  // the tensors hold the remaining references
  return redo;
}

}  // namespace lco

extern "C" lco_status lco_contract_batch(lco_ctx ctx, int count, const lco_contract_desc* descs, lco_tensor* outs) {
  if (!ctx || count < 0 || (count && (!descs || !outs))) return set_error_msg(LCO_E_ARG, "lco_contract_batch: bad argument");
  for (int i = 0; i < count; ++i) outs[i] = nullptr;
  std::vector<lco_tensor> temps;
  try {
    std::vector<ContractDetail> plans(count);
    for (int i = 0; i < count; ++i) {
      const lco_contract_desc& x = descs[i];
      if (!x.a || !x.b) fail(LCO_E_ARG, "lco_contract_batch: tensor is NULL");
      if (x.a->ctx->device != ctx->device || x.b->ctx->device != ctx->device)
        fail(LCO_E_ARG, "lco_contract_batch: tensor lives on another device");
      plans[i] = plan_contract(x.a->order, x.a->dims, x.a_labels, x.a->nnz, x.b->order, x.b->dims, x.b_labels,
                               x.b->nnz, x.c_order, x.c_labels, x.flags, &ctx->sel);
    }
    LCO_HIP(hipSetDevice(ctx->device));
    std::vector<BatchJob> acc_jobs, na_jobs;
    std::vector<PJob> pjobs;
    std::vector<int> percall, batched;
    for (int i = 0; i < count; ++i) {
      const ContractDetail& d = plans[i];
      if (d.empty) {
        outs[i] = new_tensor(ctx, d.order_c, d.c_dims, 0);
        continue;
      }
      const int algo = d.pub.algo;
      const bool rowwise = algo == LCO_ALG_CSR || algo == LCO_ALG_CSRNA;
      const bool colwise = algo == LCO_ALG_CSC || algo == LCO_ALG_CSCNA;
      if ((!rowwise && !colwise) || d.n_entrywise) {
        percall.push_back(i);
        continue;
      }
      const lco_tensor_s* A = descs[i].a;
      const lco_tensor_s* B = descs[i].b;
      if (d.pub.permute_a) {
        temps.push_back(permuted(ctx, A, d.perm_a));
        A = temps.back();
      }
      if (d.pub.permute_b) {
        temps.push_back(permuted(ctx, B, d.perm_b));
        B = temps.back();
      }
      const bool acc = algo == LCO_ALG_CSR || algo == LCO_ALG_CSC;
      const lco_tensor_s* Ap = rowwise ? A : B;
      const lco_tensor_s* Bp = rowwise ? B : A;
      if (persist_eligible(d.em, d.ek, Ap->nnz, Bp->nnz)) {
        PJob j{};
        j.index = i;
        j.A = Ap;
        j.B = Bp;
        j.mp = d.em;
        j.kp = d.ek;
        j.np = d.en;
        j.order_c = d.order_c;
        for (int r = 0; r < d.order_c; ++r) j.natural_dims[r] = d.natural_dims[r];
        persist_params(ctx, j, acc);
        pjobs.push_back(j);
      } else {
        BatchJob j;
        j.index = i;
        j.A = Ap;
        j.B = Bp;
        j.kp = d.pub.k;
        j.np = rowwise ? d.pub.n : d.pub.m;
        j.order_c = d.order_c;
        for (int r = 0; r < d.order_c; ++r) j.natural_dims[r] = d.natural_dims[r];
        (acc ? acc_jobs : na_jobs).push_back(j);
      }
      batched.push_back(i);
    }
    if (!pjobs.empty() && pjobs.size() < kPersistMinInstances) {
      // too few for the persistent engine: the chunked engine takes them
      for (const PJob& p : pjobs) {
        BatchJob j;
        j.index = p.index;
        j.A = p.A;
        j.B = p.B;
        j.kp = p.kp;
        j.np = p.np;
        j.order_c = p.order_c;
        for (int r = 0; r < p.order_c; ++r) j.natural_dims[r] = p.natural_dims[r];
        (p.acc ? acc_jobs : na_jobs).push_back(j);
      }
      pjobs.clear();
    }
    std::vector<int> redo = persist_group(ctx, pjobs, outs);
    // the rest (rows of A' listed sparsely) in chunks of bounded total entries
    auto run_chunks = [&](const std::vector<BatchJob>& jobs, bool acc) {
      size_t i = 0;
      while (i < jobs.size()) {
        std::vector<BatchJob> chunk;
        int64_t entries = 0;
        while (i < jobs.size() && (chunk.empty() || entries + jobs[i].A->nnz <= kBatchChunkEntries)) {
          entries += jobs[i].A->nnz;
          chunk.push_back(jobs[i++]);
        }
        std::vector<int> r = batch_group(ctx, chunk, acc, outs);
        redo.insert(redo.end(), r.begin(), r.end());
      }
    };
    run_chunks(acc_jobs, true);
    run_chunks(na_jobs, false);
    for (int i : batched) {
      if (!outs[i] || !plans[i].pub.permute_c) continue;
      lco_tensor natural = outs[i];
      outs[i] = permuted(ctx, natural, plans[i].perm_c);
      lco_destroy(natural);
    }
    percall.insert(percall.end(), redo.begin(), redo.end());
    for (int i : percall) outs[i] = contract_run(ctx, descs[i].a, descs[i].b, plans[i]);
    for (lco_tensor t : temps) lco_destroy(t);
    ctx->batch_stats[0] = (int64_t)batched.size() - (int64_t)redo.size();
    ctx->batch_stats[1] = (int64_t)percall.size();
    ctx->batch_stats[2] = (int64_t)pjobs.size();
    return LCO_OK;
  } catch (const Error& e) {
    for (lco_tensor t : temps) lco_destroy(t);
    for (int i = 0; i < count; ++i) {
      if (outs[i]) lco_destroy(outs[i]);
      outs[i] = nullptr;
    }
    return set_error(e);
  } catch (const std::exception& e) {
    for (lco_tensor t : temps) lco_destroy(t);
    for (int i = 0; i < count; ++i) {
      if (outs[i]) lco_destroy(outs[i]);
      outs[i] = nullptr;
    }
    return set_error_msg(LCO_E_HIP, e.what());
  }
}

extern "C" lco_status lco_batch_stats(lco_ctx ctx, int64_t* batched, int64_t* per_call, int64_t* persistent) {
  if (!ctx || !batched || !per_call) return set_error_msg(LCO_E_ARG, "lco_batch_stats: bad argument");
  *batched = ctx->batch_stats[0];
  *per_call = ctx->batch_stats[1];
  if (persistent) *persistent = ctx->batch_stats[2];
  return LCO_OK;
}
