// Planned batches: the shape-dependent work of a batch of contractions done
// once (operand rearrangements, output sizes, the output pool), then the whole
// batch -- multiplication datatypes, symbolic counts, offsets and numeric
// products of every instance -- re-run as one persistent launch, which a HIP
// graph can capture.  An autotuner picks the row-engine branch and the work
// item size of each size bucket.
#include <algorithm>
#include <map>

#include "rows.h"

namespace lco {
lco_status set_error(const Error& e);
lco_status set_error_msg(lco_status s, const char* msg);
void persist_params(lco_ctx ctx, PJob& j, bool selector_acc);
}  // namespace lco

using namespace lco;

namespace {

struct Gather {
  const double* src;
  const uint64_t* idx;
  int64_t n;
  double* dst;
};

struct BucketInfo {
  int bucket = 0, instances = 0, algo = LCO_ALG_CSR, group = 0;
  double ms = 0.0;
};

}  // namespace

struct lco_batch_plan_s {
  lco_ctx ctx = nullptr;
  std::vector<lco_tensor> outs;   // the outputs (owned)
  std::vector<lco_tensor> owned;  // rearranged operands and outputs in the natural product order
  KeptBuffers keep;
  std::vector<Gather> pre, post;  // value gathers before and after the persistent launch
  PersistBatch* pb = nullptr;
  Pool* pool = nullptr;
  uint64_t total = 0;
  std::vector<BucketInfo> info;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

uint64_t* pool_livs(lco_batch_plan P) { return P->pool ? (uint64_t*)P->pool->base : nullptr; }
double* pool_vals(lco_batch_plan P) {
  return P->pool ? (double*)((char*)P->pool->base + P->total * 8) : nullptr;
}

// `in` rearranged by `plan`, with the gather that refreshes its values: returns the
// rearranged tensor (LIVs final) and appends dst[i] = src[idx[i]] to `gathers`.
lco_tensor permuted_with_gather(lco_batch_plan P, const lco_tensor_s* in, const RpDetail& plan,
                                std::vector<Gather>& gathers) {
  lco_ctx ctx = P->ctx;
  const int64_t n = in->nnz;
  uint64_t* iota = P->keep.get<uint64_t>(n);
  uint64_t* idx = P->keep.get<uint64_t>(n);
  fill_iota(ctx, iota, n);
  lco_tensor_s src = *in;  // the same LIVs, with positions as the payload
  src.vals = reinterpret_cast<double*>(iota);
  lco_tensor t = new_tensor(ctx, in->order, plan.new_dims, n);
  P->owned.push_back(t);
  permute_storage(ctx, &src, plan, t->livs, reinterpret_cast<double*>(idx));
  gathers.push_back({in->vals, idx, n, t->vals});
  gather_values(ctx, in->vals, idx, n, t->vals);
  return t;
}

// The whole batch from the operands' current values: value gathers of the
// rearranged operands, one persistent launch (every phase of every instance),
// value gathers of the rearranged outputs.
void run_all(lco_ctx ctx, lco_batch_plan P) {
  for (const Gather& g : P->pre) gather_values(ctx, g.src, g.idx, g.n, g.dst);
  if (P->pb) P->pb->launch(0, 5, pool_livs(P), pool_vals(P), P->total);
  for (const Gather& g : P->post) gather_values(ctx, g.src, g.idx, g.n, g.dst);
}

double time_numeric(lco_ctx ctx, lco_batch_plan P) {
  hipEvent_t a, b;
  LCO_HIP(hipEventCreate(&a));
  LCO_HIP(hipEventCreate(&b));
  P->pb->launch(5, 5, pool_livs(P), pool_vals(P), P->total);  // warm
  LCO_HIP(hipEventRecord(a, ctx->stream));
  P->pb->launch(5, 5, pool_livs(P), pool_vals(P), P->total);
  LCO_HIP(hipEventRecord(b, ctx->stream));
  LCO_HIP(hipEventSynchronize(b));
  float ms = 0.f;
  LCO_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

// Autotuner: for each size bucket without a choice in the context, the branch
// (accumulator or sort-based) and the 64-row chunks per work item, timed on
// the numeric phase of the bucket's own instances.  Every candidate computes
// the same values, so the outputs stay valid.
void tune_buckets(lco_ctx ctx, lco_batch_plan P, std::vector<PJob>& jobs, const std::vector<bool>& sel_acc) {
  std::map<int, std::vector<int>> buckets;
  for (size_t i = 0; i < jobs.size(); ++i) buckets[jobs[i].bucket].push_back((int)i);
  const bool timer_was_on = ctx->timer.on;
  ctx->timer.on = false;
  for (auto& kv : buckets) {
    const std::vector<int>& idx = kv.second;
    BucketInfo bi;
    bi.bucket = kv.first;
    bi.instances = (int)idx.size();
    const int key = kv.first * 2 + (sel_acc[idx[0]] ? 1 : 0);
    bool mixed = false;  // instances of one bucket whose selected branches differ keep their own choices
    for (int i : idx) mixed = mixed || sel_acc[i] != sel_acc[idx[0]];
    auto it = ctx->tune.find(key);
    if (it == ctx->tune.end() && !mixed) {
      std::vector<bool> active(jobs.size(), false);
      for (int i : idx) active[i] = true;
      double best = 1e30;
      int best_acc = 1, best_group = 1;
      for (int acc = 1; acc >= 0; --acc) {
        for (int group : {1, 4, 16}) {
          for (int i : idx) P->pb->set_params(i, acc != 0, group);
          P->pb->upload_params();
          P->pb->set_items(active);
          const double ms = time_numeric(ctx, P);
          if (ms < best) {
            best = ms;
            best_acc = acc;
            best_group = group;
          }
        }
      }
      ctx->tune[key] = {best_acc, best_group};
      bi.ms = best;
    }
    for (int i : idx) {
      persist_params(ctx, jobs[i], sel_acc[i]);
      P->pb->set_params(i, jobs[i].acc, jobs[i].group);
    }
    bi.algo = jobs[idx[0]].acc ? LCO_ALG_CSR : LCO_ALG_CSRNA;
    bi.group = jobs[idx[0]].group;
    P->info.push_back(bi);
  }
  ctx->timer.on = timer_was_on;
  P->pb->upload_params();
  P->pb->set_items(std::vector<bool>(jobs.size(), true));
}

void destroy_plan(lco_batch_plan P) {
  if (!P) return;
  if (P->ctx) (void)hipStreamSynchronize(P->ctx->stream);
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  for (lco_tensor t : P->outs)
    if (t) lco_destroy(t);
  for (lco_tensor t : P->owned) lco_destroy(t);
  if (P->pool) release_pool(P->pool);
  delete P->pb;
  P->keep.release();
  delete P;
}

}  // namespace

extern "C" {

lco_status lco_batch_plan_create(lco_ctx ctx, int count, const lco_contract_desc* descs, lco_batch_plan* out) {
  if (!out) return set_error_msg(LCO_E_ARG, "lco_batch_plan_create: out is NULL");
  *out = nullptr;
  if (!ctx || count < 0 || (count && !descs)) return set_error_msg(LCO_E_ARG, "lco_batch_plan_create: bad argument");
  lco_batch_plan P = new lco_batch_plan_s;
  P->ctx = ctx;
  P->keep.ctx = ctx;
  P->outs.assign(count, nullptr);
  try {
    LCO_HIP(hipSetDevice(ctx->device));
    std::vector<ContractDetail> plans(count);
    for (int i = 0; i < count; ++i) {
      const lco_contract_desc& x = descs[i];
      if (!x.a || !x.b) fail(LCO_E_ARG, "lco_batch_plan_create: tensor is NULL");
      if (x.a->ctx->device != ctx->device || x.b->ctx->device != ctx->device)
        fail(LCO_E_ARG, "lco_batch_plan_create: tensor lives on another device");
      plans[i] = plan_contract(x.a->order, x.a->dims, x.a_labels, x.a->nnz, x.b->order, x.b->dims, x.b_labels,
                               x.b->nnz, x.c_order, x.c_labels, x.flags, &ctx->sel);
      const int algo = plans[i].pub.algo;
      if (!plans[i].empty && ((algo != LCO_ALG_CSR && algo != LCO_ALG_CSC && algo != LCO_ALG_CSRNA &&
                               algo != LCO_ALG_CSCNA) || plans[i].n_entrywise))
        fail(LCO_E_UNSUPPORTED, "lco_batch_plan_create: instance " + std::to_string(i) +
                                    " is not a singly compressed row or column product without entrywise modes");
    }
    // operands in the layout each product needs (one rearranged copy per tensor and order)
    std::map<std::pair<const void*, std::vector<int>>, lco_tensor> rearranged;
    auto operand = [&](const lco_tensor_s* t, bool needs, const int* perm) -> const lco_tensor_s* {
      if (!needs) return t;
      std::vector<int> key(perm, perm + t->order);
      auto it = rearranged.find({t, key});
      if (it != rearranged.end()) return it->second;
      const RpDetail rp = plan_permute(t->order, t->dims, perm, t->nnz, default_digit_cap());
      lco_tensor r = permuted_with_gather(P, t, rp, P->pre);
      rearranged[{t, key}] = r;
      return r;
    };
    std::vector<PJob> jobs;
    std::vector<bool> sel_acc;
    for (int i = 0; i < count; ++i) {
      const ContractDetail& d = plans[i];
      if (d.empty) {
        P->outs[i] = new_tensor(ctx, d.order_c, d.c_dims, 0);
        continue;
      }
      const int algo = d.pub.algo;
      const bool rowwise = algo == LCO_ALG_CSR || algo == LCO_ALG_CSRNA;
      const lco_tensor_s* A = operand(descs[i].a, d.pub.permute_a, d.perm_a);
      const lco_tensor_s* B = operand(descs[i].b, d.pub.permute_b, d.perm_b);
      PJob j{};
      j.index = i;
      j.A = rowwise ? A : B;
      j.B = rowwise ? B : A;
      j.mp = d.em;
      j.kp = d.ek;
      j.np = d.en;
      j.order_c = d.order_c;
      for (int r = 0; r < d.order_c; ++r) j.natural_dims[r] = d.natural_dims[r];
      if (!persist_eligible(j.mp, j.kp, j.A->nnz, j.B->nnz))
        fail(LCO_E_UNSUPPORTED, "lco_batch_plan_create: instance " + std::to_string(i) +
                                    " has mostly empty rows of A' or exceeds the batched engine's sizes");
      const bool acc = algo == LCO_ALG_CSR || algo == LCO_ALG_CSC;
      persist_params(ctx, j, acc);
      jobs.push_back(j);
      sel_acc.push_back(acc);
    }
    std::vector<lco_tensor> natural(count, nullptr);
    if (!jobs.empty()) {
      P->pb = new PersistBatch(ctx, jobs, nullptr, &P->keep);
      P->pb->launch(0, 4, nullptr, nullptr, 0);
      P->pb->read_sizes();
      for (size_t i = 0; i < jobs.size(); ++i)
        if (P->pb->fallback()[i])
          fail(LCO_E_UNSUPPORTED, "lco_batch_plan_create: instance " + std::to_string(jobs[i].index) +
                                      " has a row with more than 64 products or entries");
      P->total = P->pb->total();
      if (P->total) {
        P->pool = new_pool(ctx, P->total * 16);
        P->pb->launch(5, 5, pool_livs(P), pool_vals(P), P->total);
      }
      for (size_t i = 0; i < jobs.size(); ++i) {
        const PJob& j = jobs[i];
        const uint64_t off = P->pb->offsets()[i], n = P->pb->sizes()[i];
        natural[j.index] = n ? pool_tensor(ctx, P->pool, j.order_c, j.natural_dims, pool_livs(P) + off,
                                           pool_vals(P) + off, (int64_t)n)
                             : new_tensor(ctx, j.order_c, j.natural_dims, 0);
        P->owned.push_back(natural[j.index]);
      }
      tune_buckets(ctx, P, jobs, sel_acc);
    }
    // outputs in the order of c_labels
    for (int i = 0; i < count; ++i) {
      const ContractDetail& d = plans[i];
      if (d.empty) continue;
      lco_tensor nat = natural[i];
      if (!d.pub.permute_c) {
        // hand the natural output over to the caller-visible list
        P->owned.erase(std::find(P->owned.begin(), P->owned.end(), nat));
        P->outs[i] = nat;
        continue;
      }
      const RpDetail rp = plan_permute(nat->order, nat->dims, d.perm_c, nat->nnz, default_digit_cap());
      lco_tensor fin = permuted_with_gather(P, nat, rp, P->post);
      P->owned.erase(std::find(P->owned.begin(), P->owned.end(), fin));
      P->outs[i] = fin;
    }
    sync(ctx);
    *out = P;
    return LCO_OK;
  } catch (const Error& e) {
    destroy_plan(P);
    return set_error(e);
  } catch (const std::exception& e) {
    destroy_plan(P);
    return set_error_msg(LCO_E_HIP, e.what());
  }
}

lco_tensor lco_batch_plan_output(lco_batch_plan p, int i) {
  if (!p || i < 0 || i >= (int)p->outs.size()) return nullptr;
  return p->outs[i];
}

lco_status lco_batch_plan_execute(lco_ctx ctx, lco_batch_plan p) {
  if (!ctx || !p || p->ctx->device != ctx->device) return set_error_msg(LCO_E_ARG, "lco_batch_plan_execute: bad argument");
  try {
    LCO_HIP(hipSetDevice(ctx->device));
    run_all(ctx, p);
    return LCO_OK;
  } catch (const Error& e) {
    return set_error(e);
  }
}

lco_status lco_batch_plan_graph_launch(lco_ctx ctx, lco_batch_plan p) {
  if (!ctx || !p || p->ctx->device != ctx->device)
    return set_error_msg(LCO_E_ARG, "lco_batch_plan_graph_launch: bad argument");
  try {
    LCO_HIP(hipSetDevice(ctx->device));
    if (!p->exec) {
      // capture the batch once, on a stream of the plan's own
      if (!p->cap) LCO_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
      hipStream_t saved = ctx->stream;
      const bool timer_was_on = ctx->timer.on;
      ctx->stream = p->cap;
      ctx->timer.on = false;
      hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        try {
          run_all(ctx, p);
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(p->cap, &g);
          if (g) (void)hipGraphDestroy(g);
          ctx->stream = saved;
          ctx->timer.on = timer_was_on;
          throw;
        }
        e = hipStreamEndCapture(p->cap, &p->graph);
      }
      ctx->stream = saved;
      ctx->timer.on = timer_was_on;
      hip_check(e, "capture of the batch plan");
      LCO_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    }
    LCO_HIP(hipGraphLaunch(p->exec, ctx->stream));
    return LCO_OK;
  } catch (const Error& e) {
    return set_error(e);
  }
}

lco_status lco_batch_plan_launch_info(lco_batch_plan p, int i, int* bucket, int* instances, int* algo, int* group,
                                      double* ms) {
  if (!p || i < 0 || i >= (int)p->info.size() || !bucket || !instances || !algo || !group || !ms)
    return set_error_msg(LCO_E_ARG, "lco_batch_plan_launch_info: bad argument");
  const BucketInfo& x = p->info[i];
  *bucket = x.bucket;
  *instances = x.instances;
  *algo = x.algo;
  *group = x.group;
  *ms = x.ms;
  return LCO_OK;
}

lco_status lco_batch_plan_destroy(lco_batch_plan p) {
  destroy_plan(p);
  return LCO_OK;
}

}  // extern "C"
