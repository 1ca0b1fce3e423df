// Many independent problems on one device: the cells and k-points of a batch,
// or the requests of a serving loop.  They are the paper's pool level of
// parallelism (k-points, and images, distributed with little communication);
// on one GPU they become concurrent streams.
//
// hpsi_apply_batched launches every product on a pool of worker streams of
// the context (round robin), ordered after the caller's stream and joined
// back into it.  davidson_solve_batched runs one host worker thread per
// worker stream; each takes the next unsolved problem and runs
// davidson_solve on its own stream, so the latency-bound reduced eigensolves
// and small transforms of different problems share the device.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <string>
#include <thread>
#include <vector>

#include "plan.h"

namespace {

constexpr int kMaxWorkers = 32;

pw_status ensure_pool(pw_ctx ctx, int nw) {
  std::lock_guard<std::mutex> l(ctx->mu);
  while ((int)ctx->pool.size() < nw) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    PW_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(s);
      return pw::fail(PW_EDEVICE, "event creation failed");
    }
    ctx->pool.push_back(s);
    ctx->pool_events.push_back(e);
  }
  return PW_OK;
}

// worker streams [0, nw) wait for the work already queued on `caller`
pw_status fork_from(pw_ctx ctx, hipStream_t caller, int nw) {
  hipEvent_t e = ctx->pool_events[0];
  PW_HIP(hipEventRecord(e, caller));
  for (int w = 0; w < nw; ++w) PW_HIP(hipStreamWaitEvent(ctx->pool[w], e, 0));
  return PW_OK;
}

// `caller` waits for everything queued on worker streams [0, nw)
pw_status join_into(pw_ctx ctx, hipStream_t caller, int nw) {
  for (int w = 0; w < nw; ++w) {
    PW_HIP(hipEventRecord(ctx->pool_events[w], ctx->pool[w]));
    PW_HIP(hipStreamWaitEvent(caller, ctx->pool_events[w], 0));
  }
  return PW_OK;
}

}  // namespace

void pw::ctx_release_pool(pw_ctx ctx) {
  std::lock_guard<std::mutex> l(ctx->mu);
  for (hipStream_t s : ctx->pool) (void)hipStreamDestroy(s);
  for (hipEvent_t e : ctx->pool_events) (void)hipEventDestroy(e);
  ctx->pool.clear();
  ctx->pool_events.clear();
}

extern "C" pw_status hpsi_apply_batched(pw_ctx ctx, int32_t n, const pw_plan* plans, pw_precision prec,
                                        const int32_t* nb, const pw_c128* const* psi, const int32_t* ldpsi,
                                        pw_c128* const* hpsi, const int32_t* ldhpsi, int32_t nstreams,
                                        void* stream) {
  PW_CHECK(ctx != nullptr, PW_EINVAL, "NULL context");
  PW_CHECK(n >= 0, PW_EINVAL, "n < 0");
  if (n == 0) return PW_OK;
  PW_CHECK(plans && nb && psi && ldpsi && hpsi && ldhpsi, PW_EINVAL, "NULL array argument");
  {
    std::vector<pw_plan> seen(plans, plans + n);
    std::sort(seen.begin(), seen.end());
    PW_CHECK(std::adjacent_find(seen.begin(), seen.end()) == seen.end(), PW_EINVAL,
             "a plan appears twice in the batch (its workspace cannot serve two products at once)");
  }
  for (int i = 0; i < n; ++i) {
    PW_CHECK(plans[i] != nullptr, PW_EINVAL, "NULL plan in batch");
    PW_CHECK(plans[i]->ctx == ctx, PW_EINVAL, "plan of another context in batch");
  }
  PW_HIP(hipSetDevice(ctx->device));
  const int nw = std::max(1, std::min({n, nstreams > 0 ? (int)nstreams : 8, kMaxWorkers}));
  PW_TRY(ensure_pool(ctx, nw));
  hipStream_t caller = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> l(ctx->mu);   // one batched call per context at a time
  PW_TRY(fork_from(ctx, caller, nw));
  pw_status result = PW_OK;
  for (int i = 0; i < n && result == PW_OK; ++i)
    result = hpsi_apply(plans[i], prec, nb[i], psi[i], ldpsi[i], hpsi[i], ldhpsi[i], ctx->pool[i % nw]);
  if (result != PW_OK) {
    const std::string msg = std::string("batch item: ") + pw_last_error();
    (void)join_into(ctx, caller, nw);
    return pw::fail(result, msg);
  }
  PW_TRY(join_into(ctx, caller, nw));
  return PW_OK;
}

extern "C" pw_status davidson_solve_batched(pw_ctx ctx, int32_t n, const pw_plan* plans, const int32_t* nb,
                                            pw_c128* const* psi, const int32_t* ldpsi, double* const* eig,
                                            double* const* resid, const pw_david_opts* opts,
                                            pw_david_stats* stats, pw_status* status, int32_t nworkers,
                                            void* stream) {
  PW_CHECK(ctx != nullptr, PW_EINVAL, "NULL context");
  PW_CHECK(n >= 0, PW_EINVAL, "n < 0");
  if (n == 0) return PW_OK;
  PW_CHECK(plans && nb && psi && ldpsi && eig && resid, PW_EINVAL, "NULL array argument");
  pw_david_opts o;
  if (opts) o = *opts; else pw_david_opts_default(&o);
  PW_CHECK(o.history == nullptr, PW_EINVAL, "history is not supported in batched solves");
  {
    std::vector<pw_plan> seen(plans, plans + n);
    std::sort(seen.begin(), seen.end());
    PW_CHECK(std::adjacent_find(seen.begin(), seen.end()) == seen.end(), PW_EINVAL,
             "a plan appears twice in the batch (its workspace cannot serve two solves at once)");
  }
  for (int i = 0; i < n; ++i) {
    PW_CHECK(plans[i] != nullptr, PW_EINVAL, "NULL plan in batch");
    PW_CHECK(plans[i]->ctx == ctx, PW_EINVAL, "plan of another context in batch");
    PW_CHECK(plans[i]->dav != nullptr, PW_EINVAL, "plan without Davidson workspace in batch");
  }
  const int nw = std::max(1, std::min({n, nworkers > 0 ? (int)nworkers : 8, kMaxWorkers}));
  // concurrent solves take the cooperative form with fewer workgroups per launch
  const bool wide = nw > 1;
  PW_HIP(hipSetDevice(ctx->device));
  PW_TRY(ensure_pool(ctx, nw));
  hipStream_t caller = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> l(ctx->mu);
  PW_TRY(fork_from(ctx, caller, nw));

  // Cooperative kernels need every workgroup of a launch resident at once:
  // each solve reserves the workgroups of its launch from the device budget
  // while it runs (waiting while other solves hold theirs), so the launches
  // that can spin at one time stay within the budget.  A solve whose launch
  // is larger than the whole budget runs without them.
  std::mutex cmu;
  std::condition_variable ccv;
  int coop_units = 0;

  std::vector<pw_status> st(n, PW_OK);
  std::vector<std::string> msg(n);
  std::atomic<int> next{0};
  auto work = [&](int w) {
    if (hipSetDevice(ctx->device) != hipSuccess) return;
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n) break;
      const bool allowed = pw::dav_get_coop(plans[i]);
      const int pcoop = pw::coop_workgroups(o.ndim * nb[i], wide);
      int reserved = 0;
      if (allowed && (nw == 1 || pcoop <= pw::kCoopWgBudget)) {
        std::unique_lock<std::mutex> cl(cmu);
        ccv.wait(cl, [&] { return nw == 1 || coop_units + pcoop <= pw::kCoopWgBudget; });
        coop_units += pcoop;
        reserved = pcoop;
      }
      (void)pw::dav_set_coop(plans[i], reserved > 0, wide);
      pw_david_stats one{};
      st[i] = davidson_solve(plans[i], nb[i], psi[i], ldpsi[i], eig[i], resid[i], &o, &one, ctx->pool[w]);
      if (stats) stats[i] = one;
      if (st[i] != PW_OK) msg[i] = pw_last_error();
      (void)hipStreamSynchronize(ctx->pool[w]);
      (void)pw::dav_set_coop(plans[i], allowed);
      if (reserved > 0) {
        {
          std::lock_guard<std::mutex> cl(cmu);
          coop_units -= reserved;
        }
        ccv.notify_all();
      }
    }
  };
  std::vector<std::thread> threads;
  threads.reserve(nw);
  for (int w = 1; w < nw; ++w) threads.emplace_back(work, w);
  work(0);
  for (auto& t : threads) t.join();
  if (status)
    for (int i = 0; i < n; ++i) status[i] = st[i];
  PW_TRY(join_into(ctx, caller, nw));
  pw_status result = PW_OK;
  for (int i = 0; i < n; ++i) {
    if (st[i] < 0) return pw::fail(st[i], "batch item " + std::to_string(i) + ": " + msg[i]);
    if (st[i] == PW_ENOTCONV) result = PW_ENOTCONV;
  }
  return result;
}
