// Per-kernel event timing (off by default).  Each timed scope records a pair
// of events on its stream; pw_profile_read synchronizes and sums the elapsed
// times of the closed scopes per kernel class.
#include <mutex>
#include <unordered_map>
#include <vector>

#include "plan.h"
#include "profile.h"

namespace {
const char* kNames[pw::PK_COUNT] = {"k_zinv", "k_plane", "k_zfwd", "calbec_gemm", "calbec_reduce_dapply",
                                    "add_nl_gemm", "zgemm_cn", "zgemm_cn_reduce", "zgemm_nn", "k_chol",
                                    "k_trinv", "k_tridiag", "k_bisect", "k_invit", "k_backtr", "vector_ops",
                                    "density"};
struct Rec {
  int k;
  double units;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
int g_only = -1;                            // the one class timed, or -1 for all
uint64_t g_next = 1;
std::unordered_map<uint64_t, Rec> g_open;   // scopes whose end event is not yet recorded
std::vector<Rec> g_recs;                    // closed scopes, not yet summed
std::vector<hipEvent_t> g_pool;
double g_ms[pw::PK_COUNT];
double g_units[pw::PK_COUNT];
long g_n[pw::PK_COUNT];

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void drain() {
  for (Rec& r : g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g_ms[r.k] += ms;
      g_n[r.k] += 1;
      g_units[r.k] += r.units;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}
}  // namespace

bool pw::prof_on(int kernel) { return g_on && (g_only < 0 || g_only == kernel); }

uint64_t pw::prof_begin(int k, hipStream_t s, double units) {
  std::lock_guard<std::mutex> l(g_mu);
  Rec r{k, units, take(), take()};
  (void)hipEventRecord(r.a, s);
  const uint64_t id = g_next++;
  g_open.emplace(id, r);
  return id;
}

void pw::prof_end(uint64_t id, hipStream_t s) {
  std::lock_guard<std::mutex> l(g_mu);
  auto it = g_open.find(id);
  if (it == g_open.end()) return;   // profiling was reset while the scope was open
  (void)hipEventRecord(it->second.b, s);
  g_recs.push_back(it->second);
  g_open.erase(it);
  if (g_recs.size() > 4096) drain();
}

extern "C" pw_status pw_profile_enable(int on) {
  std::lock_guard<std::mutex> l(g_mu);
  drain();
  for (auto& kv : g_open) {   // scopes still open are dropped
    g_pool.push_back(kv.second.a);
    g_pool.push_back(kv.second.b);
  }
  g_open.clear();
  for (int k = 0; k < pw::PK_COUNT; ++k) { g_ms[k] = 0.0; g_n[k] = 0; g_units[k] = 0.0; }
  g_on = on != 0;
  g_only = -1;
  return PW_OK;
}

extern "C" pw_status pw_profile_only(int32_t k) {
  PW_CHECK(k >= -1 && k < pw::PK_COUNT, PW_EINVAL, "bad profile class");
  const pw_status st = pw_profile_enable(1);
  std::lock_guard<std::mutex> l(g_mu);
  g_only = k;
  return st;
}

extern "C" int32_t pw_profile_count(void) { return pw::PK_COUNT; }

extern "C" const char* pw_profile_name(int32_t k) {
  return (k >= 0 && k < pw::PK_COUNT) ? kNames[k] : "";
}

extern "C" pw_status pw_profile_read(int32_t k, int64_t* launches, double* total_ms, double* units) {
  PW_CHECK(k >= 0 && k < pw::PK_COUNT && launches && total_ms && units, PW_EINVAL, "bad profile query");
  std::lock_guard<std::mutex> l(g_mu);
  drain();
  *launches = g_n[k];
  *total_ms = g_ms[k];
  *units = g_units[k];
  return PW_OK;
}
