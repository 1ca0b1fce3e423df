// Shared device/host helpers of the plane-wave library (complex arithmetic,
// status handling).  gfx950 only.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>

#include "pwdft.h"

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};
using c128 = cpx<double>;
using c64 = cpx<float>;

template <typename T>
__host__ __device__ __forceinline__ cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
// multiply by i*s (s = +1 or -1)
template <typename T>
__host__ __device__ __forceinline__ cpx<T> mul_is(cpx<T> a, T s) { return {-a.y * s, a.x * s}; }

// ---------------------------------------------------------------------------
// status plumbing (host)
// ---------------------------------------------------------------------------
namespace pw {
void set_error(const std::string& msg);
pw_status fail(pw_status st, const std::string& msg);
}  // namespace pw

#define PW_STR2(x) #x
#define PW_STR(x) PW_STR2(x)
#define PW_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      (void)hipGetLastError(); /* the status carries it; do not leave it to other HIP users */ \
      return pw::fail(PW_EDEVICE, std::string(__FILE__ ":" PW_STR(__LINE__) ": ") + #call ": " + \
                                      hipGetErrorString(e_));                                 \
    }                                                                                         \
  } while (0)

#define PW_CHECK(cond, st, msg)             \
  do {                                      \
    if (!(cond)) return pw::fail(st, msg);  \
  } while (0)

#define PW_TRY(expr)                     \
  do {                                   \
    pw_status s_ = (expr);               \
    if (s_ != PW_OK) return s_;          \
  } while (0)

static inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
