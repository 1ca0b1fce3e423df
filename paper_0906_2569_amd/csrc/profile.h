// Optional per-kernel timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pw {
enum ProfKernel {
  PK_ZINV = 0, PK_PLANE, PK_ZFWD, PK_CALBEC, PK_CALBEC_RED, PK_ADDNL, PK_GEMM_CN, PK_GEMM_RED, PK_GEMM_NN,
  PK_CHOL, PK_TRINV, PK_TRIDIAG, PK_BISECT, PK_INVIT, PK_BACKTR, PK_VECTOR, PK_DENSITY, PK_COUNT
};
// timing is enabled for kernel class `kernel`
bool prof_on(int kernel);
// returns the id of the open scope, passed back to prof_end
uint64_t prof_begin(int kernel, hipStream_t s, double units);
void prof_end(uint64_t id, hipStream_t s);

// RAII helper: times everything launched on `s` during its lifetime.
// `units` is the algorithmic work of the scope: bytes for memory-bound
// kernels, flops for the matrix products and factorizations.
struct ProfScope {
  uint64_t id = 0;
  hipStream_t s;
  ProfScope(int kernel, hipStream_t st, double units = 0.0) : s(st) {
    // no event scopes inside a stream capture (the events would become graph nodes)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (prof_on(kernel) && hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
      id = prof_begin(kernel, s, units);
  }
  ~ProfScope() { if (id) prof_end(id, s); }
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;
};
}  // namespace pw
