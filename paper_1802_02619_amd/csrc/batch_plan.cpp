// Planned batches: the shape-dependent work of a batch of contractions done
// once, the numeric work re-run (and graph-captured) on demand, with an
// autotuner for the row-engine branch and launch width of each size bucket.
#include <algorithm>
#include <map>

#include "rows.h"

namespace lco {
lco_status set_error(const Error& e);
lco_status set_error_msg(lco_status s, const char* msg);
}  // namespace lco

using namespace lco;

namespace {

struct Gather {
  const double* src;
  const uint64_t* idx;
  int64_t n;
  double* dst;
};

struct LaunchInfo {
  int bucket = 0, instances = 0, algo = LCO_ALG_CSR, blocks_per_cu = 0;
  double ms = 0.0;
};

}  // namespace

struct lco_batch_plan_s {
  lco_ctx ctx = nullptr;
  std::vector<lco_tensor> outs;   // the outputs (owned)
  std::vector<lco_tensor> owned;  // rearranged operands and outputs in the natural product order
  KeptBuffers keep;
  std::vector<Gather> pre, post;  // value gathers before and after the numeric launches
  std::vector<BatchLaunch> launches;
  std::vector<LaunchInfo> info;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

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

void run_numeric(lco_ctx ctx, lco_batch_plan P) {
  for (const Gather& g : P->pre) gather_values(ctx, g.src, g.idx, g.n, g.dst);
  for (const BatchLaunch& L : P->launches) batch_numeric(ctx, L);
  for (const Gather& g : P->post) gather_values(ctx, g.src, g.idx, g.n, g.dst);
}

double time_launch(lco_ctx ctx, const BatchLaunch& L) {
  hipEvent_t a, b;
  LCO_HIP(hipEventCreate(&a));
  LCO_HIP(hipEventCreate(&b));
  batch_numeric(ctx, L);  // warm
  LCO_HIP(hipEventRecord(a, ctx->stream));
  batch_numeric(ctx, L);
  LCO_HIP(hipEventRecord(b, ctx->stream));
  LCO_HIP(hipEventSynchronize(b));
  float ms = 0.f;
  LCO_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

// Autotuner: the branch and blocks per compute unit of one launch, timed on the launch itself.
void tune_launch(lco_ctx ctx, BatchLaunch& L, int bucket, LaunchInfo& info) {
  const int key = bucket * 2 + (L.acc ? 1 : 0);
  auto it = ctx->tune.find(key);
  if (it != ctx->tune.end()) {
    L.acc = it->second.first != 0;
    L.grid = batch_grid(ctx, L.rows, L.chunk_rows, it->second.second);
    info.ms = 0.0;
  } else {
    const bool timer_was_on = ctx->timer.on;
    ctx->timer.on = false;
    double best = 1e30;
    int best_acc = L.acc, best_bpc = 0;
    for (int acc = 1; acc >= 0; --acc) {
      for (int bpc : {4, 8, 16}) {
        BatchLaunch c = L;
        c.acc = acc != 0;
        c.grid = batch_grid(ctx, L.rows, L.chunk_rows, bpc);
        const double ms = time_launch(ctx, c);
        if (ms < best) {
          best = ms;
          best_acc = acc;
          best_bpc = bpc;
        }
      }
    }
    ctx->timer.on = timer_was_on;
    ctx->tune[key] = {best_acc, best_bpc};
    L.acc = best_acc != 0;
    L.grid = batch_grid(ctx, L.rows, L.chunk_rows, best_bpc);
    info.ms = best;
  }
  info.algo = L.acc ? LCO_ALG_CSR : LCO_ALG_CSRNA;
  info.blocks_per_cu = ctx->tune[key].second;
  // the outputs hold this launch's results (every candidate computes the same values)
  batch_numeric(ctx, L);
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
                               x.b->nnz, x.c_order, x.c_labels, x.flags, ctx->cross);
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
    // jobs grouped by (branch, size bucket)
    std::map<std::pair<int, int>, std::vector<BatchJob>> groups;
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
      BatchJob j;
      j.index = i;
      j.A = rowwise ? A : B;
      j.B = rowwise ? B : A;
      j.kp = d.pub.k;
      j.np = rowwise ? d.pub.n : d.pub.m;
      j.order_c = d.order_c;
      for (int r = 0; r < d.order_c; ++r) j.natural_dims[r] = d.natural_dims[r];
      const bool acc = algo == LCO_ALG_CSR || algo == LCO_ALG_CSC;
      const int bucket = bits_for((uint64_t)j.A->nnz) / 2;
      groups[{bucket, acc ? 1 : 0}].push_back(j);
    }
    std::vector<lco_tensor> natural(count, nullptr);
    for (auto& kv : groups) {
      const std::vector<BatchJob>& jobs = kv.second;
      size_t i = 0;
      while (i < jobs.size()) {
        std::vector<BatchJob> chunk;
        int64_t entries = 0;
        while (i < jobs.size() && (chunk.empty() || entries + jobs[i].A->nnz <= kBatchChunkEntries)) {
          entries += jobs[i].A->nnz;
          chunk.push_back(jobs[i++]);
        }
        BatchLaunch L;
        const std::vector<int> redo = batch_group(ctx, chunk, kv.first.second != 0, natural.data(), &P->keep, &L);
        for (const BatchJob& j : chunk)
          if (natural[j.index]) P->owned.push_back(natural[j.index]);
        if (!redo.empty())
          fail(LCO_E_UNSUPPORTED, "lco_batch_plan_create: instance " + std::to_string(redo[0]) +
                                      " has a row with more than 64 products");
        LaunchInfo info;
        info.bucket = kv.first.first;
        info.instances = (int)chunk.size();
        tune_launch(ctx, L, kv.first.first, info);
        P->launches.push_back(L);
        P->info.push_back(info);
      }
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
    run_numeric(ctx, p);
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
      // capture the numeric launches once, on a stream of the plan's own
      if (!p->cap) LCO_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
      hipStream_t saved = ctx->stream;
      const bool timer_was_on = ctx->timer.on;
      ctx->stream = p->cap;
      ctx->timer.on = false;
      hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        try {
          run_numeric(ctx, p);
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

lco_status lco_batch_plan_launch_info(lco_batch_plan p, int i, int* bucket, int* instances, int* algo,
                                      int* blocks_per_cu, double* ms) {
  if (!p || i < 0 || i >= (int)p->info.size() || !bucket || !instances || !algo || !blocks_per_cu || !ms)
    return set_error_msg(LCO_E_ARG, "lco_batch_plan_launch_info: bad argument");
  const LaunchInfo& x = p->info[i];
  *bucket = x.bucket;
  *instances = x.instances;
  *algo = x.algo;
  *blocks_per_cu = x.blocks_per_cu;
  *ms = x.ms;
  return LCO_OK;
}

lco_status lco_batch_plan_destroy(lco_batch_plan p) {
  destroy_plan(p);
  return LCO_OK;
}

}  // extern "C"
