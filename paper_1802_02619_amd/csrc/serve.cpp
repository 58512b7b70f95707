// Request server: continuous batching of contractions over worker streams.
//
// Each worker thread owns a HIP stream (default priority) and a context that
// keeps its released device blocks for reuse.  A free worker takes every
// pending request that fits the device-memory budget, in arrival order, and
// runs them as one batched contraction (a batch of one as a plain call);
// requests arriving meanwhile wait for the next free worker, so the batches of
// different workers overlap on the device.  An outer-product or doubly
// compressed request runs in a batch of its own, and waits while another such
// request is on the GPU.  A request's result does not depend on the batch it ran in: the
// batched path computes every row with the same device code and summation
// order as the per-call path.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>

#include "lco_internal.h"

namespace lco {
lco_status set_error(const Error& e);
lco_status set_error_msg(lco_status s, const char* msg);
}  // namespace lco

using namespace lco;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  lco_tensor a = nullptr, b = nullptr;
  std::vector<int> la, lb, lc;  // never empty, so .data() is valid for order-0 operands
  int c_order = 0;
  uint32_t flags = 0;
  bool solo = false;   // runs in a batch of its own
  bool heavy = false;  // outer product or doubly compressed: also one at a time
  uint64_t est = 0;      // estimated device footprint (bytes)
  uint64_t charged = 0;  // what was taken from the budget
  Clock::time_point arrival, start;
  lco_server_result res{};
};

// Device bytes a request may need beyond its resident operands: the product,
// the multiplication datatype, and (for the outer product and the doubly
// compressed path) the expanded product list with its sort buffers.
uint64_t footprint(const ContractDetail& d, int64_t nnz_a, int64_t nnz_b, bool rowwise) {
  const uint64_t nn = (uint64_t)(nnz_a + nnz_b);
  return (rowwise ? 128ull : 512ull) * nn + (1ull << 20) + (d.pub.permute_a ? 32ull * nnz_a : 0) +
         (d.pub.permute_b ? 32ull * nnz_b : 0);
}

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct lco_server_s {
  lco_server_config cfg{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_done;
  // Idle workers wait on their own condition variable; new work wakes the
  // worker that went idle last, so that at low load one warm worker (thread,
  // stream and scratch) serves the requests.
  std::vector<std::unique_ptr<std::condition_variable>> cv_worker;
  std::vector<int> idle;     // stack of idle workers
  std::vector<char> woken;   // per worker: woken by wake_one

  std::deque<Request*> pending, done;
  uint64_t budget_left = 0;
  bool heavy_running = false;  // an outer-product or doubly compressed request is on the GPU
  int64_t next_ticket = 0;
  int64_t outstanding = 0;  // submitted and not yet complete
  bool stop = false;
  std::vector<hipStream_t> streams;
  std::vector<lco_ctx> ctxs;
  std::vector<std::vector<hipEvent_t>> events;  // per worker: completion events, grown on demand
  std::vector<std::thread> threads;
};

namespace {

// Called with the lock held: wakes the worker that went idle last.
void wake_one(lco_server s) {
  if (s->idle.empty()) return;
  const int w = s->idle.back();
  s->idle.pop_back();
  s->woken[w] = 1;
  s->cv_worker[w]->notify_one();
}

// Called with the lock held: moves the next batch out of `pending`.
bool take_batch(lco_server s, std::vector<Request*>& batch) {
  const uint64_t total = s->cfg.hbm_budget;
  for (auto it = s->pending.begin(); it != s->pending.end() && (int)batch.size() < s->cfg.max_batch;) {
    Request* r = *it;
    const bool idle = s->budget_left == total && batch.empty();
    // the outer-product and doubly compressed requests (sorts of every product)
    // also run one at a time: two of them on the GPU together would each take
    // about twice as long
    if ((r->est > s->budget_left && !idle) || (r->solo && !batch.empty()) || (r->heavy && s->heavy_running)) {
      ++it;
      continue;
    }
    r->charged = std::min(r->est, s->budget_left);
    s->budget_left -= r->charged;
    batch.push_back(r);
    it = s->pending.erase(it);
    if (r->heavy) s->heavy_running = true;
    if (r->solo) break;
  }
  return !batch.empty();
}

void run_batch(lco_server s, int w, std::vector<Request*>& batch) {
  lco_ctx ctx = s->ctxs[w];
  hipStream_t stream = s->streams[w];
  const int n = (int)batch.size();
  std::vector<lco_tensor> outs(n, nullptr);
  std::vector<lco_status> st(n, LCO_OK);
  // Each request completes on an event of its own: its result is handed back
  // once its own work is done, not when the rest of its batch is.  Requests
  // of one batched call share the call's event (one launch computes them all).
  std::vector<hipEvent_t>& ev = s->events[w];
  while ((int)ev.size() < n) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) break;
    ev.push_back(e);
  }
  std::vector<int> done_at(n, -1);  // index of the event that completes request i (-1: synchronise the stream)
  int nev = 0;
  auto mark = [&](int first, int last) {
    if (nev < (int)ev.size() && hipEventRecord(ev[nev], stream) == hipSuccess) {
      for (int i = first; i < last; ++i) done_at[i] = nev;
      ++nev;
    }
  };
  auto alone = [&](int i) {
    Request* r = batch[i];
    st[i] = lco_contract(ctx, r->a, r->la.data(), r->b, r->lb.data(), r->c_order, r->lc.data(), r->flags, &outs[i]);
    mark(i, i + 1);
  };
  if (s->cfg.plain || n == 1) {
    // a batch of one takes the per-call path, which is the faster one for a single product
    for (int i = 0; i < n; ++i) alone(i);
  } else {
    std::vector<lco_contract_desc> d(n);
    for (int i = 0; i < n; ++i) {
      Request* r = batch[i];
      d[i] = {r->a, r->la.data(), r->b, r->lb.data(), r->c_order, r->lc.data(), r->flags};
    }
    if (lco_contract_batch(ctx, n, d.data(), outs.data()) == LCO_OK) {
      mark(0, n);
    } else {
      // isolate the failure: every request gets its own outcome
      nev = 0;
      for (int i = 0; i < n; ++i) done_at[i] = -1;
      for (int i = 0; i < n; ++i) alone(i);
    }
  }
  // hand results back in completion order (the events complete in the order recorded)
  int i = 0;
  while (i < n) {
    int j = i + 1;
    if (done_at[i] >= 0) {
      while (j < n && done_at[j] == done_at[i]) ++j;
      (void)hipEventSynchronize(ev[done_at[i]]);
    } else {
      j = n;  // no event: the rest complete together
      (void)hipStreamSynchronize(stream);
    }
    const Clock::time_point t_done = Clock::now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (int q = i; q < j; ++q) {
        Request* r = batch[q];
        if (r->heavy) s->heavy_running = false;
        r->res.status = st[q];
        r->res.out = st[q] == LCO_OK ? outs[q] : nullptr;
        r->res.latency_ms = ms_between(r->arrival, t_done);
        r->res.queue_ms = ms_between(r->arrival, r->start);
        r->res.batch_size = n;
        s->budget_left += r->charged;
        s->done.push_back(r);
        s->outstanding--;
      }
      // finished requests free budget (and possibly the running solo request):
      // another worker may now take what this one does not
      if (!s->pending.empty()) wake_one(s);
    }
    s->cv_done.notify_all();
    i = j;
  }
  (void)hipStreamSynchronize(stream);  // nothing of this batch is still in flight when the worker moves on
}

void worker_main(lco_server s, int w) {
  (void)hipSetDevice(s->device);
  std::vector<Request*> batch;
  for (;;) {
    batch.clear();
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (take_batch(s, batch)) break;
        if (s->stop && s->pending.empty()) return;
        s->idle.push_back(w);
        s->cv_worker[w]->wait(lk, [&] { return s->woken[w] || s->stop; });
        s->woken[w] = 0;
        s->idle.erase(std::remove(s->idle.begin(), s->idle.end(), w), s->idle.end());
      }
      // more work than this batch: let another worker look at it
      if (!s->pending.empty()) wake_one(s);
    }
    const Clock::time_point t_start = Clock::now();
    for (Request* r : batch) r->start = t_start;
    run_batch(s, w, batch);
  }
}

void release(lco_server s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto& cv : s->cv_worker) cv->notify_all();
  }
  for (std::thread& t : s->threads)
    if (t.joinable()) t.join();
  for (Request* r : s->done) {
    if (r->res.out) lco_destroy(r->res.out);
    delete r;
  }
  for (Request* r : s->pending) delete r;
  for (lco_ctx c : s->ctxs) lco_ctx_destroy(c);
  for (auto& v : s->events)
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
}

}  // namespace

extern "C" {

lco_status lco_server_create(int device, const lco_server_config* cfg, lco_server* out) {
  if (!out) return set_error_msg(LCO_E_ARG, "lco_server_create: out is NULL");
  *out = nullptr;
  if (!cfg || cfg->workers < 1 || cfg->workers > 64 || cfg->max_batch < 1 || (cfg->plain != 0 && cfg->plain != 1) ||
      cfg->hbm_budget == 0)
    return set_error_msg(LCO_E_ARG, "lco_server_create: bad configuration");
  lco_server s = new lco_server_s;
  s->cfg = *cfg;
  if (s->cfg.plain) s->cfg.max_batch = 1;
  s->device = device;
  s->budget_left = cfg->hbm_budget;
  try {
    int count = 0;
    LCO_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) fail(LCO_E_ARG, "lco_server_create: no such device");
    LCO_HIP(hipSetDevice(device));
    for (int w = 0; w < cfg->workers; ++w) {
      hipStream_t st;
      LCO_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      s->streams.push_back(st);
      lco_ctx c = nullptr;
      const lco_status r = lco_ctx_create(device, st, nullptr, nullptr, nullptr, &c);
      if (r != LCO_OK) fail(r, "lco_server_create: context creation failed");
      s->ctxs.push_back(c);
    }
    s->events.resize(cfg->workers);
    s->woken.assign(cfg->workers, 0);
    for (int w = 0; w < cfg->workers; ++w) s->cv_worker.emplace_back(new std::condition_variable);
    for (int w = 0; w < cfg->workers; ++w) s->threads.emplace_back(worker_main, s, w);
  } catch (const Error& e) {
    release(s);
    return set_error(e);
  } catch (const std::exception& e) {
    release(s);
    return set_error_msg(LCO_E_HIP, e.what());
  }
  *out = s;
  return LCO_OK;
}

lco_status lco_server_submit(lco_server s, const lco_contract_desc* d, int64_t* ticket) {
  if (!s || !d || !ticket || !d->a || !d->b) return set_error_msg(LCO_E_ARG, "lco_server_submit: bad argument");
  *ticket = -1;
  try {
    if (d->a->ctx->device != s->device || d->b->ctx->device != s->device)
      fail(LCO_E_ARG, "lco_server_submit: operand lives on another device");
    if (d->c_order < 0 || d->c_order > LCO_MAX_ORDER) fail(LCO_E_ARG, "lco_server_submit: bad output order");
    // argument errors surface here, before the request is queued; the algorithm
    // is the one the workers' contexts will select
    const ContractDetail plan = plan_contract(d->a->order, d->a->dims, d->a_labels, d->a->nnz, d->b->order,
                                              d->b->dims, d->b_labels, d->b->nnz, d->c_order, d->c_labels,
                                              d->flags, &s->ctxs[0]->sel);
    Request* r = new Request;
    r->a = d->a;
    r->b = d->b;
    r->la.assign(d->a_labels, d->a_labels + d->a->order);
    r->lb.assign(d->b_labels, d->b_labels + d->b->order);
    r->lc.assign(d->c_labels, d->c_labels + d->c_order);
    if (r->la.empty()) r->la.push_back(0);
    if (r->lb.empty()) r->lb.push_back(0);
    if (r->lc.empty()) r->lc.push_back(0);
    r->c_order = d->c_order;
    r->flags = d->flags;
    const int algo = plan.pub.algo;
    const bool rowwise = !plan.empty && (algo == LCO_ALG_CSR || algo == LCO_ALG_CSC || algo == LCO_ALG_CSRNA ||
                                         algo == LCO_ALG_CSCNA);
    const int64_t nn = d->a->nnz + d->b->nnz;
    r->solo = !plan.empty && (!rowwise || (s->cfg.solo_nnz > 0 && nn > s->cfg.solo_nnz));
    r->heavy = !plan.empty && !rowwise;
    r->est = footprint(plan, d->a->nnz, d->b->nnz, rowwise || plan.empty);
    r->arrival = Clock::now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      r->res.ticket = s->next_ticket++;
      *ticket = r->res.ticket;
      s->pending.push_back(r);
      s->outstanding++;
      wake_one(s);
    }
    return LCO_OK;
  } catch (const Error& e) {
    return set_error(e);
  } catch (const std::exception& e) {
    return set_error_msg(LCO_E_HIP, e.what());
  }
}

lco_status lco_server_poll(lco_server s, lco_server_result* results, int cap, int* count) {
  if (!s || !count || cap < 0 || (cap > 0 && !results)) return set_error_msg(LCO_E_ARG, "lco_server_poll: bad argument");
  std::lock_guard<std::mutex> lk(s->mu);
  int n = 0;
  while (n < cap && !s->done.empty()) {
    Request* r = s->done.front();
    s->done.pop_front();
    results[n++] = r->res;
    delete r;
  }
  *count = n;
  return LCO_OK;
}

lco_status lco_server_drain(lco_server s) {
  if (!s) return set_error_msg(LCO_E_ARG, "lco_server_drain: server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
  return LCO_OK;
}

lco_status lco_server_destroy(lco_server s) {
  if (!s) return LCO_OK;
  release(s);
  return LCO_OK;
}

}  // extern "C"
