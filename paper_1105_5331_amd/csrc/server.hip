// Continuous-batching decomposition server.
//
// Requests (a prepared-or-not data tensor, a rank, a tolerance and an
// initial guess, all device-resident and owned by the caller) enter a FIFO.
// A fixed number of slots run decompositions concurrently, each on its own
// HIP stream with its own library handle, so the kernels of different
// requests overlap on the device.  Small dense requests (batch_elems) go to a
// second FIFO instead: a batch thread admits them into one batch of the
// batched engine (batch.hip) as places and memory free up and advances all of
// them with one kernel launch per step.  A request is admitted when a slot
// (or batch place) is free and its HBM footprint fits in the budget next to
// the requests already running; admission is in arrival order per FIFO.
// Finished requests go to a completion list that cp_server_poll drains.
// Results do not depend on what else runs: every kernel's work split depends
// only on the request's own shapes, a batched request is computed by its own
// workgroup, and no reduction uses atomics.
#include "common.hpp"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

using cpng::BatchEngine;
using cpng::BatchItem;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id = 0;
  uint64_t tag = 0;
  cp_tensor T{};
  int R = 0;
  double tol = 0.0;
  double* u = nullptr;
  size_t footprint = 0;
  cp_result res{};
};

}  // namespace

struct cp_server {
  int device = 0;
  int slots = 1;
  size_t budget = 0;
  cp_options opt{};
  int64_t batch_elems = 0;   // > 0: small dense requests take the batched path
  int batch_cap = 256;
  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  std::deque<Request*> queue;
  std::deque<Request*> bqueue;   // waiting for the batched path
  std::vector<Request*> done;
  size_t in_use = 0;
  int active = 0;
  int bactive = 0;               // requests in the batch
  std::thread batcher;
  bool stop = false;
  int64_t next_id = 0;
  std::vector<std::thread> workers;
  std::vector<int> worker_rc;
  Clock::time_point t0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

size_t request_footprint(const cp_tensor& T, int R, int window) {
  int64_t sum = 0, maxd = 0, total = 1;
  for (int k = 0; k < T.order; ++k) {
    sum += T.dims[k];
    maxd = std::max<int64_t>(maxd, T.dims[k]);
    total *= T.dims[k];
  }
  const size_t L = (size_t)sum * R;
  const size_t elem = T.dtype == CP_F32 ? 4 : 8;
  const size_t tensor = T.sparse ? (size_t)T.nnz * (elem + 4 * T.order) * (T.order + 1)
                                 : (size_t)total * elem;
  const size_t state = sizeof(double) * L * (9 + 2 * (size_t)window);
  const size_t work = sizeof(double) * (3 * L + 4096) + 2048 * (size_t)maxd * 32 * 8 +
                      ((size_t)64 << 20);
  // the mode-group partials of the two-level evaluation (dense, order >= 3)
  size_t ybuf = 0;
  if (!T.sparse && T.order >= 3 && T.order <= CP_MAX_ORDER) {
    cpng::Shape sh;
    sh.N = T.order;
    for (int k = 0; k < T.order; ++k) {
      sh.dims[k] = T.dims[k];
      sh.off[k + 1] = sh.off[k] + T.dims[k];
    }
    const int split = cpng::tree_split(&T, sh, CP_PREC_FP64);
    if (split)
      ybuf = sizeof(double) * (cpng::tree_partial_elems(sh, split, R, true) +
                               cpng::tree_partial_elems(sh, split, R, false));
  }
  return tensor + state + work + ybuf;
}

void worker_main(cp_server* s, int slot) {
  int rc = CP_OK;
  cp_handle* h = nullptr;
  hipStream_t st = nullptr;
  if (hipSetDevice(s->device) != hipSuccess || cp_create(s->device, 0, &h) != CP_OK ||
      hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    rc = CP_EDEVICE;
  }
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] {
        return s->stop || (!s->queue.empty() &&
                           s->in_use + s->queue.front()->footprint <= s->budget);
      });
      if (s->stop) break;
      r = s->queue.front();
      s->queue.pop_front();
      s->in_use += r->footprint;
      s->active++;
    }
    r->res.t_start = s->now();
    r->res.slot = slot;
    int status = rc;
    cp_report rep{};
    if (status == CP_OK) status = cp_tensor_prepare(h, &r->T, st);
    if (status == CP_OK) status = cp_decompose(h, &r->T, r->R, r->tol, &s->opt, r->u, &rep, st);
    cp_tensor_release(h, &r->T);
    r->res.status = status;
    r->res.iters = rep.iters;
    r->res.converged = rep.converged;
    r->res.n_fg = rep.n_fg;
    r->res.f = rep.f;
    r->res.rho = rep.rho;
    r->res.switch_iter = rep.switch_iter;
    r->res.t_end = s->now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->in_use -= r->footprint;
      s->active--;
      s->done.push_back(r);
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
  if (st) (void)hipStreamDestroy(st);
  if (h) cp_destroy(h);
  std::lock_guard<std::mutex> lk(s->mu);
  s->worker_rc[slot] = rc;
}

// Result of a batched request, then the completion list.
void finish_batched(cp_server* s, cp_handle* h, Request* r, int status, const cp_report* rep) {
  r->res.status = status;
  if (rep) {
    r->res.iters = rep->iters;
    r->res.converged = rep->converged;
    r->res.n_fg = rep->n_fg;
    r->res.f = rep->f;
    r->res.rho = rep->rho;
  }
  r->res.switch_iter = -1;
  r->res.t_end = s->now();
  if (h) cp_tensor_release(h, &r->T);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->in_use -= r->footprint;
    s->bactive--;
    s->done.push_back(r);
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

// The batch thread: admits queued small requests in arrival order while the
// batch has places and the budget allows, then advances every request of the
// batch by one step (one launch), and returns the finished ones.
void batch_main(cp_server* s) {
  int rc = CP_OK;
  cp_handle* h = nullptr;
  hipStream_t st = nullptr;
  BatchEngine* e = nullptr;
  if (hipSetDevice(s->device) != hipSuccess || cp_create(s->device, 0, &h) != CP_OK ||
      hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
      !(e = cpng::batch_engine_create(h, st, s->opt, s->batch_cap)))
    rc = CP_EDEVICE;
  std::vector<BatchItem*> fin;
  for (;;) {
    std::vector<Request*> admit;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] {
        return s->stop || s->bactive > 0 ||
               (!s->bqueue.empty() && s->in_use + s->bqueue.front()->footprint <= s->budget);
      });
      if (s->stop) break;
      while (!s->bqueue.empty() && s->bactive < s->batch_cap &&
             s->in_use + s->bqueue.front()->footprint <= s->budget) {
        Request* r = s->bqueue.front();
        s->bqueue.pop_front();
        s->in_use += r->footprint;
        s->bactive++;
        admit.push_back(r);
      }
    }
    for (Request* r : admit) {
      r->res.t_start = s->now();
      r->res.slot = -1;
      int status = rc;
      if (status == CP_OK) status = cp_tensor_prepare(h, &r->T, st);
      if (status == CP_OK)
        status = cpng::batch_engine_add(e, &r->T, r->R, r->tol, r->u, r->u,
                                  (uint64_t)reinterpret_cast<uintptr_t>(r), nullptr, 0, nullptr);
      if (status != CP_OK) finish_batched(s, h, r, status, nullptr);
    }
    if (!e || cpng::batch_engine_active(e) == 0) continue;
    fin.clear();
    if (cpng::batch_engine_tick(e, &fin) != CP_OK) cpng::batch_engine_drain(e, &fin);
    for (BatchItem* it : fin) {
      cp_report rep{};
      int status = CP_OK;
      uint64_t tag = 0;
      cpng::batch_item_report(it, &rep, &status, &tag);
      cpng::batch_item_delete(it);
      finish_batched(s, h, reinterpret_cast<Request*>(static_cast<uintptr_t>(tag)), status, &rep);
    }
  }
  if (e) cpng::batch_engine_destroy(e);   // frees what a stop left active (their results are dropped)
  if (st) (void)hipStreamDestroy(st);
  if (h) cp_destroy(h);
}

}  // namespace

extern "C" {

int cp_server_create(int device, const cp_server_opts* o, cp_server** out) {
  if (!out) return CP_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CP_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return CP_EDEVICE;
  auto* s = new (std::nothrow) cp_server();
  if (!s) return CP_ENOMEM;
  s->device = device;
  s->slots = o && o->slots > 0 ? o->slots : 4;
  if (s->slots > 16) s->slots = 16;
  if (o) s->opt = o->decompose;
  else cp_options_default(&s->opt);
  s->opt.trace = nullptr;
  s->opt.trace_cap = 0;
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  s->budget = o && o->hbm_budget > 0 ? o->hbm_budget : free_b / 10 * 8;
  if (o && o->batch_elems > 0 && s->opt.method == CP_METHOD_NGMRES && s->opt.window <= 21) {
    s->batch_elems = std::min<int64_t>(o->batch_elems, CP_BATCH_MAX_ELEMS);
    s->batch_cap = o->batch_capacity > 0 ? o->batch_capacity : 256;
  }
  s->t0 = Clock::now();
  s->worker_rc.assign(s->slots, CP_OK);
  for (int i = 0; i < s->slots; ++i) s->workers.emplace_back(worker_main, s, i);
  if (s->batch_elems > 0) s->batcher = std::thread(batch_main, s);
  *out = s;
  return CP_OK;
}

int cp_server_submit(cp_server* s, const cp_tensor* T, int32_t R, double tol, double* u_inout,
                     uint64_t tag, int64_t* req_id) {
  if (!s || !T || !u_inout || R < 1 || R > 64 || !(tol >= 0.0)) return CP_EINVAL;
  auto* r = new (std::nothrow) Request();
  if (!r) return CP_ENOMEM;
  r->T = *T;
  r->T.prepared = nullptr;
  r->R = R;
  r->tol = tol;
  r->u = u_inout;
  r->tag = tag;
  const bool batched = s->batch_elems > 0 && cpng::batch_eligible(T, R, s->batch_elems);
  r->footprint = batched ? (size_t)cpng::batch_footprint(T, R, s->opt.window)
                         : request_footprint(*T, R, s->opt.window);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    r->res.req_id = r->id;
    r->res.tag = tag;
    r->res.t_submit = s->now();
    if (r->footprint > s->budget) {   // can never be admitted
      r->res.status = CP_ENOMEM;
      r->res.t_start = r->res.t_end = r->res.t_submit;
      s->done.push_back(r);
    } else if (batched) {
      s->bqueue.push_back(r);
    } else {
      s->queue.push_back(r);
    }
  }
  if (req_id) *req_id = r->id;
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  return CP_OK;
}

int cp_server_poll(cp_server* s, int32_t wait_for, cp_result* out, int32_t max_out,
                   int32_t* n_out) {
  if (!s || !out || max_out < 0 || !n_out) return CP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (wait_for > 0) {
    const int need = std::min(wait_for, max_out);
    // until enough results are there, or nothing queued or running could add one
    s->cv_done.wait(lk, [&] {
      return (int)s->done.size() >= need ||
             (s->queue.empty() && s->active == 0 && s->bqueue.empty() && s->bactive == 0);
    });
  }
  int n = std::min<int>(max_out, (int)s->done.size());
  for (int i = 0; i < n; ++i) {
    out[i] = s->done[i]->res;
    delete s->done[i];
  }
  s->done.erase(s->done.begin(), s->done.begin() + n);
  *n_out = n;
  return CP_OK;
}

int cp_server_stats(cp_server* s, int32_t* queued, int32_t* active, size_t* in_use,
                    size_t* budget) {
  if (!s) return CP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = (int32_t)(s->queue.size() + s->bqueue.size());
  if (active) *active = s->active + s->bactive;
  if (in_use) *in_use = s->in_use;
  if (budget) *budget = s->budget;
  return CP_OK;
}

int cp_server_destroy(cp_server* s) {
  if (!s) return CP_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (Request* r : s->queue) delete r;
    s->queue.clear();
    for (Request* r : s->bqueue) delete r;
    s->bqueue.clear();
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  if (s->batcher.joinable()) s->batcher.join();
  for (Request* r : s->done) delete r;
  delete s;
  return CP_OK;
}

}  // extern "C"
