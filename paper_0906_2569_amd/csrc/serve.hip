// Serving loop for a stream of independent requests (one cell at one
// k-point each, different sizes): a FIFO queue drained by worker host
// threads, each with its own stream.  A request is admitted as soon as a
// worker is idle and the device memory its plan needs fits in the budget
// next to the requests already running (continuous batching: no waiting for
// a batch to fill, no head request overtaken).  The worker builds the plan,
// runs davidson_solve, frees the plan and records the request's times.
// Plans take their device and pinned host memory from one pool that the
// server allocates once (the admission budget), and their set-up and
// teardown synchronize only the worker's own streams: a request never calls
// hipMalloc / hipFree nor waits on another request's work.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "plan.h"

struct pw_server_s {
  pw_ctx ctx = nullptr;
  pw_server_opts opts{};
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_coop;
  int coop_units = 0;   // cooperative workgroups reserved by running requests
  pw::MemPool pool;     // device memory (the budget) and pinned host memory of the plans
  int64_t served = 0;   // requests whose plan was built
  size_t pool_peak = 0; // largest pool use seen at a plan's completion
  struct Req {
    int64_t id;
    pw_problem prob;
    int32_t nb, ldpsi;
    pw_c128* psi;
    double *eig, *resid;
    pw_david_opts dopts;
    size_t bytes;
    double t_submit = 0, t_start = 0, t_end = 0;
    pw_status st = PW_OK;
    std::string msg;
    pw_david_stats stats{};
    bool done = false;
    bool cancel = false;        // pw_server_cancel was called for it
    pw_plan plan = nullptr;     // while its solve runs (guarded by mu)
  };
  std::deque<Req*> queue;
  std::map<int64_t, Req*> all;
  size_t in_use = 0;
  int64_t next_id = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  void run(int w) {
    (void)hipSetDevice(ctx->device);
    for (;;) {
      Req* r = nullptr;
      {
        std::unique_lock<std::mutex> l(mu);
        cv_work.wait(l, [&] {
          return stop || (!queue.empty() && (in_use == 0 || in_use + queue.front()->bytes <= opts.mem_budget));
        });
        if (stop) return;   // the queue was drained before stop was set
        r = queue.front();
        queue.pop_front();
        in_use += r->bytes;
        r->t_start = now();
      }
      pw_plan_opts po{opts.precision, r->nb, r->dopts.ndim};
      po.gamma = opts.gamma;
      pw_plan plan = nullptr;
      pw_status st = pw::plan_create(ctx, &r->prob, &po, &pool, streams[w], &plan);
      if (st == PW_OK) {
        // Cooperative reduced-eigensolver kernels need every workgroup of a
        // launch resident at once.  The request reserves the workgroups of its
        // launch from the device budget for its whole solve (waiting while
        // other requests hold theirs), so the launches that can spin at one
        // time never exceed the budget; a launch larger than the whole budget
        // runs without them.
        const bool wide = opts.nworkers > 1;
        const int pcoop = pw::coop_workgroups(r->dopts.ndim * r->nb, wide);
        int reserved = 0;
        if (pcoop <= pw::kCoopWgBudget) {
          std::unique_lock<std::mutex> l(mu);
          cv_coop.wait(l, [&] { return coop_units + pcoop <= pw::kCoopWgBudget; });
          coop_units += pcoop;
          reserved = pcoop;
        }
        (void)pw::dav_set_coop(plan, reserved > 0, wide);
        {
          std::lock_guard<std::mutex> l(mu);
          r->plan = plan;
          if (r->cancel) (void)pw_cancel(plan);   // cancelled while its plan was built: stops at the first check
        }
        st = davidson_solve(plan, r->nb, r->psi, r->ldpsi, r->eig, r->resid, &r->dopts, &r->stats, streams[w]);
        {
          std::lock_guard<std::mutex> l(mu);
          r->plan = nullptr;
        }
        if (st != PW_OK) r->msg = pw_last_error();
        (void)hipStreamSynchronize(streams[w]);
        if (reserved > 0) {
          {
            std::lock_guard<std::mutex> l(mu);
            coop_units -= reserved;
          }
          cv_coop.notify_all();
        }
        {
          std::lock_guard<std::mutex> l(mu);
          ++served;
          pool_peak = std::max(pool_peak, pool.dev.used());
        }
        pw::plan_destroy(plan);
      } else {
        r->msg = pw_last_error();
      }
      {
        std::lock_guard<std::mutex> l(mu);
        r->st = st;
        r->t_end = now();
        r->done = true;
        in_use -= r->bytes;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" void pw_server_opts_default(pw_server_opts* o) {
  if (!o) return;
  o->nworkers = 4;
  o->mem_budget = 0;
  o->precision = PW_MIXED;
  o->gamma = 0;
}

extern "C" pw_status pw_server_create(pw_ctx ctx, const pw_server_opts* opts, pw_server* out) {
  PW_CHECK(ctx && out, PW_EINVAL, "NULL context or output");
  *out = nullptr;
  pw_server_opts o;
  if (opts) o = *opts; else pw_server_opts_default(&o);
  PW_CHECK(o.nworkers >= 1 && o.nworkers <= 64, PW_EINVAL, "nworkers out of range [1, 64]");
  PW_CHECK(o.precision == PW_FP64 || o.precision == PW_MIXED, PW_EINVAL, "bad precision");
  PW_CHECK(o.gamma == 0 || o.gamma == 1, PW_EINVAL, "gamma must be 0 or 1");
  PW_HIP(hipSetDevice(ctx->device));
  if (o.mem_budget == 0) {
    size_t fr = 0, tot = 0;
    PW_HIP(hipMemGetInfo(&fr, &tot));
    o.mem_budget = fr / 10 * 6;
  }
  auto* s = new pw_server_s();
  s->ctx = ctx;
  s->opts = o;
  s->t0 = std::chrono::steady_clock::now();
  // one device block of the admission budget, and pinned host memory for
  // the per-plan flags of the solvers (a few KB per running request)
  {
    const pw_status st = s->pool.dev.init(o.mem_budget, false);
    if (st != PW_OK) {
      delete s;
      return st;
    }
    const pw_status sh = s->pool.host.init((size_t)o.nworkers * 64 * 1024, true);
    if (sh != PW_OK) {
      delete s;
      return sh;
    }
  }
  for (int w = 0; w < o.nworkers; ++w) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return pw::fail(PW_EDEVICE, "stream creation failed");
    }
    s->streams.push_back(st);
  }
  for (int w = 0; w < o.nworkers; ++w) s->workers.emplace_back([s, w] { s->run(w); });
  *out = s;
  return PW_OK;
}

extern "C" pw_status pw_server_submit(pw_server s, const pw_problem* problem, int32_t nb, pw_c128* psi,
                                      int32_t ldpsi, double* eig, double* resid, const pw_david_opts* opts,
                                      int64_t* ticket) {
  PW_CHECK(s && problem && psi && eig && resid && ticket, PW_EINVAL, "NULL argument");
  pw_david_opts o;
  if (opts) o = *opts; else pw_david_opts_default(&o);
  PW_CHECK(o.history == nullptr, PW_EINVAL, "history is not supported for served requests");
  PW_CHECK(nb >= 1 && nb <= problem->npw && ldpsi >= problem->npw, PW_EINVAL, "bad nb or ldpsi");
  pw_plan_opts po{s->opts.precision, nb, o.ndim};
  po.gamma = s->opts.gamma;
  const size_t bytes = pw_footprint_bytes(problem, &po);
  PW_CHECK(bytes > 0, PW_EINVAL, std::string("invalid problem: ") + pw_last_error());
  PW_CHECK(bytes <= s->opts.mem_budget, PW_ENOMEM, "request needs more device memory than the budget");
  auto* r = new pw_server_s::Req();
  r->prob = *problem;
  r->nb = nb;
  r->ldpsi = ldpsi;
  r->psi = psi;
  r->eig = eig;
  r->resid = resid;
  r->dopts = o;
  r->bytes = bytes;
  {
    std::lock_guard<std::mutex> l(s->mu);
    r->id = s->next_id++;
    r->t_submit = s->now();
    s->all[r->id] = r;
    s->queue.push_back(r);
    *ticket = r->id;
  }
  s->cv_work.notify_one();
  return PW_OK;
}

extern "C" pw_status pw_server_wait(pw_server s, int64_t ticket, pw_david_stats* stats, double times[3]) {
  PW_CHECK(s != nullptr, PW_EINVAL, "NULL server");
  std::unique_lock<std::mutex> l(s->mu);
  auto it = s->all.find(ticket);
  PW_CHECK(it != s->all.end(), PW_EINVAL, "unknown ticket");
  pw_server_s::Req* r = it->second;
  s->cv_done.wait(l, [&] { return r->done; });
  if (stats) *stats = r->stats;
  if (times) { times[0] = r->t_submit; times[1] = r->t_start; times[2] = r->t_end; }
  const pw_status st = r->st;
  const std::string msg = r->msg;
  s->all.erase(it);
  delete r;
  l.unlock();
  if (st < 0) return pw::fail(st, msg);
  return st;
}

extern "C" pw_status pw_server_poll(pw_server s, int64_t ticket, int32_t* done) {
  PW_CHECK(s && done, PW_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> l(s->mu);
  auto it = s->all.find(ticket);
  PW_CHECK(it != s->all.end(), PW_EINVAL, "unknown ticket");
  *done = it->second->done ? 1 : 0;
  return PW_OK;
}

extern "C" double pw_server_clock(pw_server s) { return s ? s->now() : 0.0; }

extern "C" pw_status pw_server_destroy(pw_server s) {
  if (!s) return PW_OK;
  {
    // finish everything submitted, then stop the workers
    std::unique_lock<std::mutex> l(s->mu);
    s->cv_done.wait(l, [&] { return s->queue.empty() && s->in_use == 0; });
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
  for (auto& kv : s->all) delete kv.second;
  delete s;
  return PW_OK;
}

extern "C" pw_status pw_server_cancel(pw_server s, int64_t ticket) {
  PW_CHECK(s != nullptr, PW_EINVAL, "NULL server");
  bool dequeued = false;
  {
    std::lock_guard<std::mutex> l(s->mu);
    auto it = s->all.find(ticket);
    PW_CHECK(it != s->all.end(), PW_EINVAL, "unknown ticket");
    pw_server_s::Req* r = it->second;
    if (r->done) return PW_OK;
    r->cancel = true;
    for (auto q = s->queue.begin(); q != s->queue.end(); ++q) {
      if (*q == r) {
        s->queue.erase(q);
        r->st = PW_ECANCELLED;
        r->msg = "request cancelled before it started";
        r->t_start = r->t_end = s->now();
        r->done = true;
        dequeued = true;
        break;
      }
    }
    if (!dequeued && r->plan) (void)pw_cancel(r->plan);
  }
  if (dequeued) {
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
  return PW_OK;
}

extern "C" pw_status pw_server_info(pw_server s, int64_t out[4]) {
  PW_CHECK(s != nullptr && out != nullptr, PW_EINVAL, "NULL server or output");
  std::lock_guard<std::mutex> l(s->mu);
  out[0] = s->served;
  out[1] = (int64_t)s->pool.dev.size();
  out[2] = (int64_t)s->pool_peak;
  out[3] = s->pool.fallbacks.load();
  return PW_OK;
}
