// Optional per-kernel timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

namespace pw {
enum ProfKernel {
  PK_ZINV = 0, PK_PLANE, PK_ZFWD, PK_CALBEC, PK_CALBEC_RED, PK_ADDNL, PK_GEMM_CN, PK_GEMM_RED, PK_GEMM_NN,
  PK_CHOL, PK_TRINV, PK_TRIDIAG, PK_BISECT, PK_INVIT, PK_BACKTR, PK_VECTOR, PK_COUNT
};
bool prof_on();
void prof_begin(int kernel, hipStream_t s, double units);
void prof_end(int kernel, hipStream_t s);

// RAII helper: times everything launched on `s` during its lifetime.
// `units` is the algorithmic work of the scope: bytes for memory-bound
// kernels, flops for the matrix products and factorizations.
struct ProfScope {
  int k;
  hipStream_t s;
  bool on;
  ProfScope(int kernel, hipStream_t st, double units = 0.0) : k(kernel), s(st), on(prof_on()) {
    if (on) prof_begin(k, s, units);
  }
  ~ProfScope() { if (on) prof_end(k, s); }
};
}  // namespace pw
