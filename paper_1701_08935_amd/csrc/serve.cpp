// Serving loop: queued interval queries on resident pencils, admitted by a
// device-memory estimate, run by worker threads that each own a HIP stream
// (so queries overlap on the GPU).  Queued queries asking for the same result
// (same pencil, interval, filter and tolerances) are answered by one run;
// factorizations stay resident after their query and serve later queries of
// the same filter.  Queries that opt in keep the eigenpairs (the subspace) they
// returned resident too: a later such query asking for the same result gets
// them back once their residuals, recomputed on the device, still meet its
// tolerance.  Least recently used factorizations and subspaces are evicted
// first when admission needs the memory.  The arithmetic is zolo_solve's; this
// file only schedules it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <string>
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
  std::string err;  // the worker's error message
  zolo_query_info info{};
};

// a resident factorization: the filter it belongs to, in use by at most one
// query at a time
struct FactorEntry {
  zolo_pencil* P = nullptr;
  double am = 0, ap = 0, bm = 0, bp = 0, eps = 0;
  int r1 = 0, r2 = 0, prec = 0, kind = 0;
  // queries that left the eigengaps (and r1) to the library: their interval and
  // estimate, and the gaps and r1 the library chose (reused instead of a new
  // inertia search)
  bool estimated = false;
  double a = 0, b = 0;
  int n_est = 0, r1_asked = 0;
  double e_am = 0, e_ap = 0, e_bm = 0, e_bp = 0;
  int e_r1 = 0;
  long long e_count = -1;
  zolo_factors* F = nullptr;
  size_t bytes = 0;
  bool busy = false;
  double last = 0.0;
};

// a resident subspace: the eigenpairs a finished query returned, for later
// queries asking for the same result
struct SubspaceEntry {
  zolo_pencil* P = nullptr;
  double a = 0.0, b = 0.0;
  zolo_opts o{};
  int nss = 0;  // subspace size of the run
  int64_t n = 0;  // the pencil's size when the entry was made
  zolo_result* res = nullptr;
  size_t bytes = 0;
  bool busy = false;
  double last = 0.0;
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
  std::vector<FactorEntry> fcache;  // resident factorizations (guarded by m)
  std::list<SubspaceEntry> scache;  // resident subspaces (guarded by m)
  size_t cached = 0;                // bytes of both
  long long hits = 0, misses = 0, sub_hits = 0;
  std::vector<zolo_pencil*> running;  // pencil of each run in progress (guarded by m)
};

namespace {

// the same result: pencil, interval, filter, precision and every tolerance and limit
bool same_request(const zolo_pencil* P1, double a1, double b1, const zolo_opts& u, const zolo_pencil* P2, double a2,
                  double b2, const zolo_opts& v) {
  auto eq = [](double p, double q) { return p == q || (std::isnan(p) && std::isnan(q)); };
  return P1 == P2 && a1 == a2 && b1 == b2 && eq(u.a_minus, v.a_minus) && eq(u.a_plus, v.a_plus) &&
         eq(u.b_minus, v.b_minus) && eq(u.b_plus, v.b_plus) && u.r1 == v.r1 && u.r2 == v.r2 &&
         u.filter_eps == v.filter_eps && u.precision == v.precision && u.tol_resid == v.tol_resid &&
         u.tol_gmres == v.tol_gmres && u.max_subspace_iter == v.max_subspace_iter &&
         u.max_gmres_iter == v.max_gmres_iter && u.max_refine == v.max_refine && u.tol_refine == v.tol_refine &&
         u.block_cols == v.block_cols && u.filter_kind == v.filter_kind && u.gmres_restart == v.gmres_restart;
}
bool same_filter(const zolo_query* x, const zolo_query* y) {
  return same_request(x->P, x->a, x->b, x->o, y->P, y->a, y->b, y->o);
}
// a resident subspace answers a query for the same result whose subspace is
// no larger than the one the subspace was computed with
bool subspace_matches(const SubspaceEntry& e, const zolo_query* q) {
  return q->o.reuse_subspace && q->nss <= e.nss && same_request(e.P, e.a, e.b, e.o, q->P, q->a, q->b, q->o);
}
SubspaceEntry* find_subspace(zolo_server* S, const zolo_query* q) {
  for (SubspaceEntry& e : S->scache)
    if (!e.busy && subspace_matches(e, q)) return &e;
  return nullptr;
}

bool gaps_estimated(const zolo_opts& o) { return std::isnan(o.a_minus); }

bool entry_matches(const FactorEntry& e, const zolo_query* q) {
  const zolo_opts& o = q->o;
  if (e.P != q->P || e.r2 != o.r2 || e.eps != o.filter_eps || e.prec != o.precision || e.kind != o.filter_kind)
    return false;
  if (gaps_estimated(o))
    return e.estimated && e.a == q->a && e.b == q->b && e.n_est == q->n_lambda && e.r1_asked == o.r1;
  return !e.estimated && e.am == o.a_minus && e.ap == o.a_plus && e.bm == o.b_minus && e.bp == o.b_plus &&
         e.r1 == o.r1;
}

// free least recently used idle factorizations and subspaces until `need` more
// bytes fit beside the running queries and the remaining cache (caller holds
// S->m; the caller frees what lands in to_free / to_free_res)
void evict_for(zolo_server* S, size_t need, std::vector<zolo_factors*>* to_free,
               std::vector<zolo_result*>* to_free_res) {
  while (S->in_use + S->cached + need > S->budget) {
    int lru = -1;
    for (int i = 0; i < (int)S->fcache.size(); ++i)
      if (!S->fcache[i].busy && (lru < 0 || S->fcache[i].last < S->fcache[lru].last)) lru = i;
    auto lrs = S->scache.end();
    for (auto it = S->scache.begin(); it != S->scache.end(); ++it)
      if (!it->busy && (lrs == S->scache.end() || it->last < lrs->last)) lrs = it;
    const bool sub = lrs != S->scache.end() && (lru < 0 || lrs->last < S->fcache[lru].last);
    if (sub) {
      S->cached -= lrs->bytes;
      to_free_res->push_back(lrs->res);
      S->scache.erase(lrs);
    } else if (lru >= 0) {
      S->cached -= S->fcache[lru].bytes;
      to_free->push_back(S->fcache[lru].F);
      S->fcache.erase(S->fcache.begin() + lru);
    } else {
      return;
    }
  }
}

// The head query and the queued queries asking for the same result, in
// arrival order; they are answered by one run with the largest subspace among
// them (cols).
std::vector<zolo_query*> head_batch(zolo_server* S, int* cols) {
  std::vector<zolo_query*> batch;
  zolo_query* h = S->queue.front();
  batch.push_back(h);
  int c = h->nss;
  for (size_t i = 1; i < S->queue.size(); ++i) {
    zolo_query* q = S->queue[i];
    if (same_filter(q, h)) {
      batch.push_back(q);
      c = std::max(c, q->nss);
    }
  }
  *cols = c;
  return batch;
}

// shifts a worker's inertia counts (eigengap estimates) factor together
constexpr int kInertiaShifts = 2;

// device bytes a run needs: the query's estimate (r1 = 0 counted as the
// largest choice, 4 poles) and, when the library estimates the eigengaps,
// the inertia factorizations that precede it
size_t batch_bytes(const zolo_query* h, int cols) {
  const int maxit = h->o.max_gmres_iter > 0 ? h->o.max_gmres_iter : 60;
  const int r1 = h->o.r1 > 0 ? h->o.r1 : 4;
  size_t e = (size_t)zolo::query_bytes_estimate(h->P, r1, cols, maxit, h->o.gmres_restart, h->o.precision, h->o.block_cols);
  if (std::isnan(h->o.a_minus))
    e = std::max(e, (size_t)(kInertiaShifts * zolo::inertia_shift_bytes(h->P)));
  return e;
}

// the run on pencil P has ended and left whatever it keeps resident (caller holds S->m)
void unmark_running(zolo_server* S, zolo_pencil* P) {
  auto it = std::find(S->running.begin(), S->running.end(), P);
  if (it != S->running.end()) S->running.erase(it);
}

// hands the result to the batch (copies for all but the first) and marks it
// done; err: the run's error message (null: the calling thread's last error)
void finish(zolo_server* S, const std::vector<zolo_query*>& batch, zolo_status rc, zolo_result* res, double t_start,
            size_t est, const std::string* err_in = nullptr) {
  const double t_end = now_s();
  const std::string err = rc == ZOLO_OK ? std::string() : err_in ? *err_in : std::string(zolo_last_error());
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
    q->err = err;
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
  zolo::set_inertia_cap(kInertiaShifts);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  if (st) zolo::register_stream(st);
  for (;;) {
    std::vector<zolo_query*> batch;
    int cols = 0;
    size_t est = 0;
    bool too_big = false;
    zolo_factors* F_in = nullptr;
    FactorEntry hit;
    SubspaceEntry* sub = nullptr;
    std::vector<zolo_factors*> to_free;
    std::vector<zolo_result*> to_free_res;
    {
      std::unique_lock<std::mutex> lk(S->m);
      S->cv_work.wait(lk, [&] {
        if (S->queue.empty()) return S->stop;
        if (find_subspace(S, S->queue.front())) return true;  // answered from a resident subspace
        int c = 0;
        std::vector<zolo_query*> b = head_batch(S, &c);
        const size_t e = batch_bytes(b[0], c);
        if (e > S->budget || S->in_use + S->cached + e <= S->budget) return true;
        size_t idle = 0;  // resident factorizations that could be evicted
        for (const FactorEntry& fe : S->fcache)
          if (!fe.busy) idle += fe.bytes;
        return S->in_use + S->cached - idle + e <= S->budget;
      });
      if (S->queue.empty()) break;  // stop requested and nothing left
      batch = head_batch(S, &cols);
      sub = find_subspace(S, batch[0]);
      est = sub ? 0 : batch_bytes(batch[0], cols);
      if (sub) {
        batch.erase(std::remove_if(batch.begin(), batch.end(),
                                   [&](const zolo_query* q) { return !subspace_matches(*sub, q); }),
                    batch.end());
        sub->busy = true;
      } else if (est > S->budget) {  // cannot run even alone: fail the head query only
        too_big = true;
        batch.resize(1);
      } else {
        evict_for(S, est, &to_free, &to_free_res);
        S->in_use += est;
        for (FactorEntry& fe : S->fcache)
          if (!fe.busy && entry_matches(fe, batch[0])) {
            fe.busy = true;
            F_in = fe.F;
            hit = fe;
            ++S->hits;
            break;
          }
        if (!F_in) ++S->misses;
      }
      for (zolo_query* q : batch) S->queue.erase(std::find(S->queue.begin(), S->queue.end(), q));
      S->running.push_back(batch[0]->P);
    }
    for (zolo_factors* f : to_free) zolo_factors_free(f);
    for (zolo_result* r : to_free_res) zolo_result_free(r);
    to_free.clear();
    to_free_res.clear();
    S->cv_work.notify_all();  // the next head may fit beside this one
    const double t_start = now_s();
    if (too_big) {
      zolo::set_error("zolo_submit: the query needs about %zu bytes, above the server's budget of %zu", est,
                      S->budget);
      const std::string err = zolo_last_error();
      {
        std::lock_guard<std::mutex> lk(S->m);
        unmark_running(S, batch[0]->P);
      }
      finish(S, batch, ZOLO_ENOMEM, nullptr, t_start, est, &err);
      continue;
    }
    if (sub) {
      // the eigenpairs of an earlier query for the same result, handed out
      // again once their residuals, recomputed now, meet this query's tolerance
      const double tol = batch[0]->o.tol_resid > 0 ? batch[0]->o.tol_resid : 1e-8;
      double worst = 0.0;
      const bool ok = zolo::pencil_n(sub->P) == sub->n && zolo::result_verify(sub->P, sub->res, st, &worst) == ZOLO_OK &&
                      worst <= tol;
      zolo_result* out = ok ? zolo::result_clone(sub->res) : nullptr;
      if (out) zolo::result_mark_reused(out, worst, now_s() - t_start);
      {
        std::lock_guard<std::mutex> lk(S->m);
        sub->busy = false;
        sub->last = now_s();
        unmark_running(S, batch[0]->P);
        if (out) S->sub_hits += (long long)batch.size();
        if (!out) {  // stale, or no memory for the copy: drop it and queue the batch again
          S->cached -= sub->bytes;
          to_free_res.push_back(sub->res);
          for (auto it = S->scache.begin(); it != S->scache.end(); ++it)
            if (&*it == sub) {
              S->scache.erase(it);
              break;
            }
          for (auto it = batch.rbegin(); it != batch.rend(); ++it) S->queue.push_front(*it);
        }
      }
      for (zolo_result* r : to_free_res) zolo_result_free(r);
      to_free_res.clear();
      if (out) finish(S, batch, ZOLO_OK, out, t_start, 0);
      S->cv_work.notify_all();
      S->cv_done.notify_all();
      continue;
    }
    // one run for the batch: the start block of its member with the largest
    // subspace (its own block, or the Gaussian block of its seed)
    zolo_query* h = batch[0];
    for (zolo_query* q : batch)
      if (q->nss > h->nss) h = q;
    const int64_t n = zolo::pencil_n(h->P);
    zolo_status rc = ZOLO_OK;
    zolo_result* res = nullptr;
    zolo_factors* F_new = nullptr;
    double* dq = nullptr;
    // eigengaps left to the library and no subspace size given: the subspace
    // follows the inertia count, and the library draws its own start block
    const bool free_nss = gaps_estimated(h->o) && h->o.n_ss <= 0 && h->Q0.empty();
    // the start block: the caller's (copied to the device) or the seeded Gaussian
    // block, drawn on the device
    const size_t q0_len = (size_t)n * h->nss * (zolo::pencil_cplx(h->P) ? 2 : 1);
    if (free_nss) {
      zolo_opts o = h->o;
      if (F_in && hit.estimated) {
        o.a_minus = hit.e_am;
        o.a_plus = hit.e_ap;
        o.b_minus = hit.e_bm;
        o.b_plus = hit.e_bp;
        o.r1 = hit.e_r1;
        if (hit.e_count >= 0)
          o.n_ss = (int)std::max<long long>((long long)std::ceil(1.5 * std::max<long long>(hit.e_count, 1)),
                                            hit.e_count + 8);
      }
      rc = zolo::solve_resident(S->ctx, h->P, h->a, h->b, h->n_lambda, &o, nullptr, st, F_in,
                                F_in ? nullptr : &F_new, &res);
    } else if (hipMalloc(&dq, sizeof(double) * q0_len) != hipSuccess) {
      rc = ZOLO_ENOMEM;
    } else if (!h->Q0.empty() &&
               hipMemcpyAsync(dq, h->Q0.data(), sizeof(double) * q0_len, hipMemcpyHostToDevice, st) != hipSuccess) {
      rc = ZOLO_EDEVICE;
    } else {
      if (h->Q0.empty()) zolo::gaussian_device(h->o.seed, (int64_t)q0_len, dq, st);
      zolo_opts o = h->o;
      o.n_ss = h->nss;
      if (F_in && hit.estimated) {  // the gaps and r1 the library chose for this interval before
        o.a_minus = hit.e_am;
        o.a_plus = hit.e_ap;
        o.b_minus = hit.e_bm;
        o.b_plus = hit.e_bp;
        o.r1 = hit.e_r1;
        if (o.n_ss == 0 && hit.n_est > 0) o.n_ss = h->nss;
      }
      rc = zolo::solve_resident(S->ctx, h->P, h->a, h->b, h->n_lambda, &o, dq, st, F_in, F_in ? nullptr : &F_new,
                                &res);
    }
    if (dq) (void)hipFree(dq);
    const std::string err = rc == ZOLO_OK ? std::string() : std::string(zolo_last_error());
    // The server's state is brought up to date before the queries are marked
    // done, so that what a caller sees after zolo_wait (zolo_server_get_info,
    // residency) already includes this run.
    zolo_result* keep = (rc == ZOLO_OK && res && h->o.reuse_subspace) ? zolo::result_clone(res) : nullptr;
    // a resident factorization keeps only its factors (this worker holds both)
    if (F_in) zolo::factors_keep_only(F_in);
    if (F_new) zolo::factors_keep_only(F_new);
    {
      std::lock_guard<std::mutex> lk(S->m);
      S->in_use -= est;
      const double t = now_s();
      for (FactorEntry& fe : S->fcache)
        if (fe.F == F_in) {
          fe.busy = false;
          fe.last = t;
        }
      // keep the new factorization resident when it fits beside the running queries
      if (F_new) {
        const size_t fb = (size_t)zolo::factors_bytes(F_new);
        evict_for(S, fb, &to_free, &to_free_res);
        if (S->in_use + S->cached + fb <= S->budget) {
          FactorEntry fe;
          fe.P = h->P;
          fe.am = h->o.a_minus;
          fe.ap = h->o.a_plus;
          fe.bm = h->o.b_minus;
          fe.bp = h->o.b_plus;
          fe.eps = h->o.filter_eps;
          fe.r1 = h->o.r1;
          fe.r2 = h->o.r2;
          fe.prec = h->o.precision;
          fe.kind = h->o.filter_kind;
          if (gaps_estimated(h->o) && res) {
            zolo_stats rs{};
            zolo_result_stats(res, &rs);
            fe.estimated = true;
            fe.a = h->a;
            fe.b = h->b;
            fe.n_est = h->n_lambda;
            fe.r1_asked = h->o.r1;
            fe.e_am = rs.a_minus;
            fe.e_ap = rs.a_plus;
            fe.e_bm = rs.b_minus;
            fe.e_bp = rs.b_plus;
            fe.e_r1 = rs.r1;
            fe.e_count = rs.inertia_count;
          }
          fe.F = F_new;
          fe.bytes = fb;
          fe.last = t;
          S->fcache.push_back(fe);
          S->cached += fb;
          F_new = nullptr;
        }
      }
      // keep the eigenpairs resident for later queries asking for the same result
      if (keep) {
        const size_t rb = (size_t)zolo::result_bytes(keep);
        evict_for(S, rb, &to_free, &to_free_res);
        if (S->in_use + S->cached + rb <= S->budget && !find_subspace(S, h)) {
          SubspaceEntry e;
          e.P = h->P;
          e.a = h->a;
          e.b = h->b;
          e.o = h->o;
          e.nss = h->nss;
          e.n = n;
          e.res = keep;
          e.bytes = rb;
          e.last = t;
          S->scache.push_back(e);
          S->cached += rb;
          keep = nullptr;
        }
      }
      unmark_running(S, batch[0]->P);
    }
    if (keep) zolo_result_free(keep);
    if (F_new) zolo_factors_free(F_new);
    for (zolo_factors* f : to_free) zolo_factors_free(f);
    for (zolo_result* r : to_free_res) zolo_result_free(r);
    finish(S, batch, rc, res, t_start, est, &err);
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
  if (st) {
    zolo::retire_stream(st);
    (void)hipStreamDestroy(st);
  }
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
    budget = fr / 10 * 6;
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
  if (h_Q0) q->Q0.assign(h_Q0, h_Q0 + (size_t)n * nss * (zolo::pencil_cplx(p) ? 2 : 1));
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
  if (q->rc != ZOLO_OK) zolo::set_error("query finished with status %d: %s", (int)q->rc, q->err.c_str());
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

extern "C" zolo_status zolo_server_get_info(zolo_server* srv, zolo_server_info* out) {
  if (!srv || !out) {
    zolo::set_error("zolo_server_get_info: null argument");
    return ZOLO_EINVAL;
  }
  std::lock_guard<std::mutex> lk(srv->m);
  out->budget_bytes = (long long)srv->budget;
  out->running_bytes = (long long)srv->in_use;
  out->resident_factors = (int)srv->fcache.size();
  out->resident_bytes = (long long)srv->cached;
  out->factor_hits = srv->hits;
  out->factor_misses = srv->misses;
  out->queued = (int)srv->queue.size();
  out->subspace_hits = srv->sub_hits;
  out->resident_subspaces = (int)srv->scache.size();
  return ZOLO_OK;
}

extern "C" zolo_status zolo_server_drop_pencil(zolo_server* srv, zolo_pencil* p) {
  if (!srv || !p) {
    zolo::set_error("zolo_server_drop_pencil: null argument");
    return ZOLO_EINVAL;
  }
  std::vector<zolo_factors*> ff;
  std::vector<zolo_result*> rr;
  {
    std::unique_lock<std::mutex> lk(srv->m);
    // no queued or running query on p: nothing can make p's entries busy or add new ones
    srv->cv_done.wait(lk, [&] {
      for (const zolo_query* q : srv->queue)
        if (q->P == p) return false;
      return std::find(srv->running.begin(), srv->running.end(), p) == srv->running.end();
    });
    for (auto it = srv->fcache.begin(); it != srv->fcache.end();) {
      if (it->P == p) {
        srv->cached -= it->bytes;
        ff.push_back(it->F);
        it = srv->fcache.erase(it);
      } else {
        ++it;
      }
    }
    for (auto it = srv->scache.begin(); it != srv->scache.end();) {
      if (it->P == p) {
        srv->cached -= it->bytes;
        rr.push_back(it->res);
        it = srv->scache.erase(it);
      } else {
        ++it;
      }
    }
  }
  for (zolo_factors* f : ff) zolo_factors_free(f);
  for (zolo_result* r : rr) zolo_result_free(r);
  srv->cv_work.notify_all();  // the freed memory may admit a waiting query
  return ZOLO_OK;
}

extern "C" void zolo_server_destroy(zolo_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->m);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (std::thread& t : srv->workers) t.join();
  for (FactorEntry& fe : srv->fcache) zolo_factors_free(fe.F);
  for (SubspaceEntry& e : srv->scache) zolo_result_free(e.res);
  delete srv;
}
