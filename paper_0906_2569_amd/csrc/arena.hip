// Memory pool of the serving loop: first-fit sub-allocation of one device
// block and one pinned host block, and the plan-level allocation helpers
// that use it (or hipMalloc / hipHostMalloc for plans built outside a pool).
#include <string>

#include "plan.h"

namespace {
constexpr size_t kGranule = 256;
size_t round_up(size_t b) { return (std::max<size_t>(b, 1) + kGranule - 1) / kGranule * kGranule; }
}  // namespace

pw_status pw::Arena::init(size_t bytes, bool host) {
  std::lock_guard<std::mutex> l(mu_);
  PW_CHECK(base_ == nullptr, PW_EINVAL, "arena already initialised");
  const size_t n = round_up(bytes);
  void* q = nullptr;
  const hipError_t e = host ? hipHostMalloc(&q, n, hipHostMallocDefault) : hipMalloc(&q, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return pw::fail(PW_ENOMEM, std::string("memory pool: ") + (host ? "hipHostMalloc" : "hipMalloc") + " of " +
                                   std::to_string(n) + " bytes failed");
  }
  base_ = static_cast<char*>(q);
  size_ = n;
  host_ = host;
  free_.clear();
  used_.clear();
  free_[0] = n;
  return PW_OK;
}

void pw::Arena::release() {
  std::lock_guard<std::mutex> l(mu_);
  if (base_ != nullptr) {
    if (host_) (void)hipHostFree(base_);
    else (void)hipFree(base_);
  }
  base_ = nullptr;
  size_ = 0;
  free_.clear();
  used_.clear();
}

void* pw::Arena::alloc(size_t bytes) {
  const size_t n = round_up(bytes);
  std::lock_guard<std::mutex> l(mu_);
  if (base_ == nullptr) return nullptr;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < n) continue;
    const size_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > n) free_[off + n] = len - n;
    used_[off] = n;
    return base_ + off;
  }
  return nullptr;
}

bool pw::Arena::free(void* p) {
  if (p == nullptr) return true;
  std::lock_guard<std::mutex> l(mu_);
  if (base_ == nullptr) return false;
  char* c = static_cast<char*>(p);
  if (c < base_ || c >= base_ + size_) return false;
  const size_t off = (size_t)(c - base_);
  auto u = used_.find(off);
  if (u == used_.end()) return false;
  size_t start = off, len = u->second;
  used_.erase(u);
  // merge with the free range after it, then with the one before it
  auto nx = free_.find(start + len);
  if (nx != free_.end()) {
    len += nx->second;
    free_.erase(nx);
  }
  auto pv = free_.lower_bound(start);
  if (pv != free_.begin()) {
    --pv;
    if (pv->first + pv->second == start) {
      start = pv->first;
      len += pv->second;
      free_.erase(pv);
    }
  }
  free_[start] = len;
  return true;
}

size_t pw::Arena::used() const {
  std::lock_guard<std::mutex> l(mu_);
  size_t t = 0;
  for (const auto& kv : used_) t += kv.second;
  return t;
}

pw_status pw::dev_alloc(pw_plan p, size_t bytes, void** out) {
  *out = nullptr;
  if (p != nullptr && p->pool != nullptr) {
    *out = p->pool->dev.alloc(bytes);
    if (*out != nullptr) return PW_OK;
    p->pool->fallbacks.fetch_add(1);
  }
  if (hipMalloc(out, std::max<size_t>(bytes, kGranule)) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return pw::fail(PW_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return PW_OK;
}

void pw::dev_free(pw_plan p, void* q) {
  if (q == nullptr) return;
  if (p != nullptr && p->pool != nullptr && p->pool->dev.free(q)) return;
  (void)hipFree(q);
}

pw_status pw::host_alloc(pw_plan p, size_t bytes, void** out) {
  *out = nullptr;
  if (p != nullptr && p->pool != nullptr) {
    *out = p->pool->host.alloc(bytes);
    if (*out != nullptr) return PW_OK;
    p->pool->fallbacks.fetch_add(1);
  }
  if (hipHostMalloc(out, std::max<size_t>(bytes, kGranule), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return pw::fail(PW_ENOMEM, "hipHostMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return PW_OK;
}

void pw::host_free(pw_plan p, void* q) {
  if (q == nullptr) return;
  if (p != nullptr && p->pool != nullptr && p->pool->host.free(q)) return;
  (void)hipHostFree(q);
}
