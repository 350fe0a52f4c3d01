// Serving loop: queued interval queries on resident pencils, admitted by a
// device-memory estimate, run by worker threads that each own a HIP stream
// (so queries overlap on the GPU), with queries that share a filter batched
// into one joint Algorithm 1 run.  The arithmetic is zolo_solve's; this file
// only schedules it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "zolo_internal.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kMaxJointColumns = 512;  // zolo_solve's subspace limit

}  // namespace

struct zolo_query {
  zolo_server* srv = nullptr;
  zolo_pencil* P = nullptr;
  double a = 0.0, b = 0.0;
  int n_lambda = 0;
  int nss = 0;
  zolo_opts o{};
  std::vector<double> Q0;  // host start block when the caller passed one
  // completion (guarded by the server mutex)
  bool done = false;
  zolo_status rc = ZOLO_OK;
  zolo_result* res = nullptr;
  zolo_query_info info{};
};

struct zolo_server {
  zolo_ctx* ctx = nullptr;
  int device = 0;
  size_t budget = 0, in_use = 0;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<zolo_query*> queue;
  bool stop = false;
  std::vector<std::thread> workers;
};

namespace {

bool same_filter(const zolo_query* x, const zolo_query* y) {
  return x->P == y->P && x->a == y->a && x->b == y->b && x->o.a_minus == y->o.a_minus && x->o.a_plus == y->o.a_plus &&
         x->o.b_minus == y->o.b_minus && x->o.b_plus == y->o.b_plus && x->o.r1 == y->o.r1 && x->o.r2 == y->o.r2 &&
         x->o.filter_eps == y->o.filter_eps && x->o.precision == y->o.precision;
}

// The head query and the queued queries sharing its filter, in arrival order.
std::vector<zolo_query*> head_batch(zolo_server* S, int* cols) {
  std::vector<zolo_query*> batch;
  zolo_query* h = S->queue.front();
  batch.push_back(h);
  int c = h->nss;
  for (size_t i = 1; i < S->queue.size(); ++i) {
    zolo_query* q = S->queue[i];
    if (same_filter(q, h) && c + q->nss <= kMaxJointColumns) {
      batch.push_back(q);
      c += q->nss;
    }
  }
  *cols = c;
  return batch;
}

size_t batch_bytes(const zolo_query* h, int cols) {
  const int maxit = h->o.max_gmres_iter > 0 ? h->o.max_gmres_iter : 60;
  return (size_t)zolo::query_bytes_estimate(h->P, std::max(h->o.r1, 1), cols, maxit, h->o.precision, h->o.block_cols);
}

void finish(zolo_server* S, const std::vector<zolo_query*>& batch, zolo_status rc, zolo_result* res, double t_start,
            size_t est) {
  const double t_end = now_s();
  std::vector<zolo_result*> out(batch.size(), nullptr);
  if (res) {
    out[0] = res;
    for (size_t i = 1; i < batch.size(); ++i) out[i] = zolo::result_clone(res);
  }
  std::lock_guard<std::mutex> lk(S->m);
  for (size_t i = 0; i < batch.size(); ++i) {
    zolo_query* q = batch[i];
    q->rc = (res && !out[i]) ? ZOLO_ENOMEM : rc;
    q->res = out[i];
    q->info.t_start = t_start;
    q->info.t_end = t_end;
    q->info.batch = (int)batch.size();
    q->info.est_bytes = (long long)est;
    q->info.done = 1;
    q->done = true;
  }
  S->cv_done.notify_all();
}

void worker(zolo_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  for (;;) {
    std::vector<zolo_query*> batch;
    int cols = 0;
    size_t est = 0;
    bool too_big = false;
    {
      std::unique_lock<std::mutex> lk(S->m);
      S->cv_work.wait(lk, [&] {
        if (S->queue.empty()) return S->stop;
        int c = 0;
        std::vector<zolo_query*> b = head_batch(S, &c);
        const size_t e = batch_bytes(b[0], c);
        return e > S->budget || S->in_use + e <= S->budget;
      });
      if (S->queue.empty()) break;  // stop requested and nothing left
      batch = head_batch(S, &cols);
      est = batch_bytes(batch[0], cols);
      if (est > S->budget) {  // cannot run even alone: fail the head query only
        too_big = true;
        batch.resize(1);
      } else {
        S->in_use += est;
      }
      for (zolo_query* q : batch) S->queue.erase(std::find(S->queue.begin(), S->queue.end(), q));
    }
    S->cv_work.notify_all();  // the next head may fit beside this one
    const double t_start = now_s();
    if (too_big) {
      finish(S, batch, ZOLO_ENOMEM, nullptr, t_start, est);
      continue;
    }
    // joint start block: every query's own block, side by side (N x cols row-major)
    zolo_query* h = batch[0];
    const int64_t n = zolo::pencil_n(h->P);
    std::vector<double> hq((size_t)n * cols);
    int c0 = 0;
    for (zolo_query* q : batch) {
      std::vector<double> g;
      const std::vector<double>* src = &q->Q0;
      if (q->Q0.empty()) {
        zolo::gaussian_block(q->o.seed, (size_t)n * q->nss, &g);
        src = &g;
      }
      for (int64_t i = 0; i < n; ++i)
        std::copy(src->begin() + i * q->nss, src->begin() + (i + 1) * q->nss, hq.begin() + i * cols + c0);
      c0 += q->nss;
    }
    zolo_status rc = ZOLO_OK;
    zolo_result* res = nullptr;
    double* dq = nullptr;
    if (hipMalloc(&dq, sizeof(double) * hq.size()) != hipSuccess) {
      rc = ZOLO_ENOMEM;
    } else if (hipMemcpyAsync(dq, hq.data(), sizeof(double) * hq.size(), hipMemcpyHostToDevice, st) != hipSuccess) {
      rc = ZOLO_EDEVICE;
    } else {
      zolo_opts o = h->o;
      o.n_ss = cols;
      int nl = 0;
      for (zolo_query* q : batch) nl += q->n_lambda;
      rc = zolo_solve(S->ctx, h->P, h->a, h->b, nl, &o, dq, st, &res);
    }
    if (dq) (void)hipFree(dq);
    finish(S, batch, rc, res, t_start, est);
    {
      std::lock_guard<std::mutex> lk(S->m);
      S->in_use -= est;
    }
    S->cv_work.notify_all();
  }
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" zolo_status zolo_server_create(zolo_ctx* ctx, int slots, size_t hbm_budget_bytes, zolo_server** out) {
  if (!ctx || !out || slots < 1 || slots > 64) {
    zolo::set_error("zolo_server_create: invalid argument");
    return ZOLO_EINVAL;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::unique_ptr<zolo_server> S(new zolo_server());
  S->ctx = ctx;
  S->device = dev;
  size_t budget = hbm_budget_bytes;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      zolo::set_error("zolo_server_create: hipMemGetInfo failed");
      return ZOLO_EDEVICE;
    }
    budget = fr / 10 * 8;
  }
  S->budget = budget;
  for (int i = 0; i < slots; ++i) S->workers.emplace_back(worker, S.get());
  *out = S.release();
  return ZOLO_OK;
}

extern "C" zolo_status zolo_submit(zolo_server* srv, zolo_pencil* p, double a, double b, int n_lambda_est,
                                   const zolo_opts* opts, const double* h_Q0, zolo_query** out) {
  if (!srv || !p || !out || !(a < b) || n_lambda_est < 0) {
    zolo::set_error("zolo_submit: invalid argument");
    return ZOLO_EINVAL;
  }
  std::unique_ptr<zolo_query> q(new zolo_query());
  q->srv = srv;
  q->P = p;
  q->a = a;
  q->b = b;
  q->n_lambda = n_lambda_est;
  if (opts)
    q->o = *opts;
  else
    zolo_opts_default(&q->o);
  const int64_t n = zolo::pencil_n(p);
  int nss = q->o.n_ss > 0 ? q->o.n_ss : (int)std::ceil(1.5 * std::max(n_lambda_est, 1));
  nss = (int)std::min<int64_t>(nss, n);
  if (nss > kMaxJointColumns) {
    zolo::set_error("zolo_submit: subspace size %d above %d", nss, kMaxJointColumns);
    return ZOLO_EINVAL;
  }
  q->nss = nss;
  if (h_Q0) q->Q0.assign(h_Q0, h_Q0 + (size_t)n * nss);
  q->info.t_submit = now_s();
  q->info.batch = 0;
  zolo_query* qp = q.release();
  {
    std::lock_guard<std::mutex> lk(srv->m);
    if (srv->stop) {
      delete qp;
      zolo::set_error("zolo_submit: server is shutting down");
      return ZOLO_EINVAL;
    }
    srv->queue.push_back(qp);
  }
  srv->cv_work.notify_all();
  *out = qp;
  return ZOLO_OK;
}

extern "C" zolo_status zolo_wait(zolo_query* q, int timeout_ms, zolo_result** out) {
  if (!q) {
    zolo::set_error("zolo_wait: null query");
    return ZOLO_EINVAL;
  }
  zolo_server* S = q->srv;
  std::unique_lock<std::mutex> lk(S->m);
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, [&] { return q->done; });
  } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return q->done; })) {
    zolo::set_error("zolo_wait: query still running");
    return ZOLO_ETIMEOUT;
  }
  if (out) {
    *out = q->res;
    q->res = nullptr;
  }
  if (q->rc != ZOLO_OK) zolo::set_error("query finished with status %d", (int)q->rc);
  return q->rc;
}

extern "C" zolo_status zolo_query_get_info(const zolo_query* q, zolo_query_info* out) {
  if (!q || !out) {
    zolo::set_error("zolo_query_get_info: null argument");
    return ZOLO_EINVAL;
  }
  std::lock_guard<std::mutex> lk(q->srv->m);
  *out = q->info;
  return ZOLO_OK;
}

extern "C" void zolo_query_free(zolo_query* q) {
  if (!q) return;
  zolo_server* S = q->srv;
  {
    std::unique_lock<std::mutex> lk(S->m);
    S->cv_done.wait(lk, [&] { return q->done; });
  }
  if (q->res) zolo_result_free(q->res);
  delete q;
}

extern "C" void zolo_server_destroy(zolo_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->m);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (std::thread& t : srv->workers) t.join();
  delete srv;
}
