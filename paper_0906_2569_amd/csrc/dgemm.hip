// Real GEMMs on the matrix cores (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32,
// one MFMA per 16x16x4 block) for the Gamma-point real-wavefunction path.
//
// At Gamma a real function f(r) has f(-G) = conj(f(G)), so only the half
// sphere is stored.  Viewing a half-sphere column of complex values as a
// real column of twice the length (re, im interleaved), the full-sphere inner
// product of two such functions is
//     <a|b> = sum_{G in full} conj(a(G)) b(G) = 2 sum_k a_k b_k - a(0) b(0),
// k over the interleaved reals and G = 0 at half-sphere index 0 (a(0), b(0)
// real).  So the projector and subspace products become real products with
// K = 2 npw_half and a rank-one correction, and combinations with real
// coefficients (Ritz rotations, the projector add-back) real products with
// M = 2 npw_half: a quarter of the complex products' flops.
//
//   tn : C[m, n] = alpha (2 sum_k A[m*lda + k] B[n*ldb + k] - w0 A[m*lda] B[n*ldb]) + beta C
//        (split K, partials summed in a fixed order: deterministic)
//   nn : C[n*ldc + m] = alpha sum_k A[k*lda + m] B[n*ldb + k] + beta C[n*ldc + m]
#include <algorithm>

#include "plan.h"
#include "profile.h"

namespace {

template <typename T>
struct RMma;
template <>
struct RMma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct RMma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// result element q of lane l: row as below, column l % 16 (same placement as
// the complex kernels)
template <typename T>
__device__ __forceinline__ int rrow(int lane, int q);
template <>
__device__ __forceinline__ int rrow<float>(int lane, int q) { return 4 * (lane >> 4) + q; }
template <>
__device__ __forceinline__ int rrow<double>(int lane, int q) { return 4 * q + (lane >> 4); }

constexpr int BM = 64, BN = 64, BK = 32, NT = 256;

template <typename T>
struct RTile {
  T a[BK][BM + 1], b[BK][BN + 1];
};

// workgroups of one output tile range share an XCD (round-robin launch order)
__device__ __forceinline__ void xcd_map(int& bx, int& by, int& bz, bool yfast) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int T = gx * gy * gridDim.z;
  const int L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int x = L & 7, s = L >> 3, per = T >> 3, rem = T & 7;
  const int w = x < rem ? x * (per + 1) + s : rem * (per + 1) + (x - rem) * per + s;
  if (yfast) {
    by = w % gy;
    bx = (w / gy) % gx;
  } else {
    bx = w % gx;
    by = (w / gx) % gy;
  }
  bz = w / (gx * gy);
}

template <typename T>
__device__ __forceinline__ void rtile_mma(const RTile<T>& t, typename RMma<T>::v4 (&c)[2][2], int wm, int wn,
                                          int lane) {
  const int r = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int k4 = 0; k4 < BK; k4 += 4) {
    const int kk = k4 + kq;
    T a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = t.a[kk][wm * 32 + i * 16 + r];
      b[i] = t.b[kk][wn * 32 + i * 16 + r];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) c[i][j] = RMma<T>::run(a[i], b[j], c[i][j]);
  }
}

// P[z][n][m] = sum_{k in chunk z} A[m*lda + k] B[n*ldb + k]
template <typename T, typename TA, typename TB>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3)))
k_dgemm_tn(int M, int N, int K, int kchunk, const TA* __restrict__ A, long lda, const TB* __restrict__ B, long ldb,
           T* __restrict__ P) {
  __shared__ RTile<T> t;
  typedef typename RMma<T>::v4 v4;
  int bx, by, bz;
  xcd_map(bx, by, bz, false);
  const int m0 = bx * BM, n0 = by * BN;
  const int kbeg = bz * kchunk, kend = min(K, kbeg + kchunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  v4 c[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) c[i][j] = v4{0, 0, 0, 0};
  constexpr int PER = BM * BK / NT;
  TA ra[PER];
  TB rb[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int kk = idx % BK, mi = idx / BK;
      const int k = k0 + kk;
      ra[it] = (m0 + mi < M && k < kend) ? A[(size_t)(m0 + mi) * lda + k] : TA(0);
      rb[it] = (n0 + mi < N && k < kend) ? B[(size_t)(n0 + mi) * ldb + k] : TB(0);
    }
  };
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int kk = idx % BK, mi = idx / BK;
      t.a[kk][mi] = (T)ra[it];
      t.b[kk][mi] = (T)rb[it];
    }
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);
    rtile_mma<T>(t, c, wm, wn, lane);
    __syncthreads();
  }
  T* out = P + (size_t)bz * M * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm * 32 + i * 16 + rrow<T>(lane, q);
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m < M && n < N) out[(size_t)n * M + m] = c[i][j][q];
      }
}

// C[n*ldc + m] = alpha (2 sum_z P[z][n][m] - w0 A[m*lda] B[n*ldb]) + beta C, in
// increasing z; C real (cplx = 0) or the real part of a complex matrix whose
// imaginary part is set to 0 (cplx = 1)
template <typename T, typename TA, typename TB>
__global__ void k_dreduce(int M, int N, int nsplit, const T* __restrict__ P, const TA* __restrict__ A, long lda,
                          const TB* __restrict__ B, long ldb, double w0, double alpha, double beta,
                          double* __restrict__ C, int ldc, int cplx) {
  const size_t total = (size_t)M * N;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += (double)P[(size_t)z * total + idx];
    const int m = (int)(idx % M), n = (int)(idx / M);
    double v = 2.0 * s - w0 * (double)A[(size_t)m * lda] * (double)B[(size_t)n * ldb];
    v *= alpha;
    if (cplx) {
      double* c = C + 2 * ((size_t)n * ldc + m);
      if (beta != 0.0) v += beta * c[0];
      c[0] = v;
      c[1] = 0.0;
    } else {
      double* c = C + (size_t)n * ldc + m;
      if (beta != 0.0) v += beta * *c;
      *c = v;
    }
  }
}

// C[n*ldc + m] = alpha sum_k A[k*lda + m] B[n*ldb + k] + beta C[n*ldc + m]  (C double)
template <typename T, typename TA, typename TB>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3)))
k_dgemm_nn(int M, int N, int K, double alpha, const TA* __restrict__ A, long lda, const TB* __restrict__ B,
           long ldb, double beta, double* __restrict__ C, long ldc, const int* __restrict__ guard) {
  if (guard != nullptr && *guard != 0) return;
  __shared__ RTile<T> t;
  typedef typename RMma<T>::v4 v4;
  int bx, by, bz;
  xcd_map(bx, by, bz, true);
  const int m0 = bx * BM, n0 = by * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  v4 c[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) c[i][j] = v4{0, 0, 0, 0};
  constexpr int PER = BM * BK / NT;
  TA ra[PER];
  TB rb[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int idx = threadIdx.x + it * NT;
      {
        const int mi = idx % BM, kk = idx / BM;
        ra[it] = (m0 + mi < M && k0 + kk < K) ? A[(size_t)(k0 + kk) * lda + m0 + mi] : TA(0);
      }
      {
        const int kk = idx % BK, ni = idx / BK;
        rb[it] = (n0 + ni < N && k0 + kk < K) ? B[(size_t)(n0 + ni) * ldb + k0 + kk] : TB(0);
      }
    }
  };
  if (K > 0) load(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int idx = threadIdx.x + it * NT;
      t.a[idx / BM][idx % BM] = (T)ra[it];
      t.b[idx % BK][idx / BK] = (T)rb[it];
    }
    __syncthreads();
    if (k0 + BK < K) load(k0 + BK);
    rtile_mma<T>(t, c, wm, wn, lane);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm * 32 + i * 16 + rrow<T>(lane, q);
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m < M && n < N) {
          double* p = C + (size_t)n * ldc + m;
          double v = alpha * (double)c[i][j][q];
          if (beta != 0.0) v += beta * *p;
          *p = v;
        }
      }
}

int dsplit(int M, int N, int K, int& kchunk) {
  const int tiles = ceil_div(M, BM) * ceil_div(N, BN);
  int ns = std::max(1, ceil_div(512, tiles));
  if (ns < 8 && K >= 8 * 256 * BK) ns = 8;   // one K range per XCD (see the complex products)
  ns = std::min(ns, std::max(1, ceil_div(K, 4 * BK)));
  kchunk = std::max(BK, ceil_div(ceil_div(K, ns), BK) * BK);
  return std::max(1, ceil_div(K, kchunk));
}

}  // namespace

size_t pw::dgemm_part_bytes(int M, int N) {
  const size_t mn = (size_t)std::max(M, 1) * std::max(N, 1);
  return std::max((size_t)512 * BM * BN + mn, 8 * mn) * sizeof(double) + 256;
}

template <typename T, typename TA, typename TB>
pw_status pw::dgemm_tn(int M, int N, int K, const TA* A, long lda, const TB* B, long ldb, double w0, double alpha,
                       double beta, double* C, int ldc, bool cplx_out, void* part, size_t part_bytes,
                       hipStream_t s, int prof) {
  if (M <= 0 || N <= 0) return PW_OK;
  int kchunk = 0;
  const int ns = dsplit(M, N, K, kchunk);
  PW_CHECK((size_t)ns * M * N * sizeof(T) <= part_bytes, PW_ENOMEM, "split-K workspace too small");
  T* P = static_cast<T*>(part);
  {
    pw::ProfScope ps(prof >= 0 ? prof : pw::PK_GEMM_CN, s, 2.0 * M * N * (double)K);
    k_dgemm_tn<T, TA, TB><<<dim3(ceil_div(M, BM), ceil_div(N, BN), ns), NT, 0, s>>>(M, N, K, kchunk, A, lda, B, ldb,
                                                                                   P);
  }
  const int g = std::min(4096, ceil_div((size_t)M * N, 256));
  k_dreduce<T, TA, TB><<<g, 256, 0, s>>>(M, N, ns, P, A, lda, B, ldb, w0, alpha, beta, C, ldc, cplx_out ? 1 : 0);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

template <typename T, typename TA, typename TB>
pw_status pw::dgemm_nn(int M, int N, int K, double alpha, const TA* A, long lda, const TB* B, long ldb, double beta,
                       double* C, long ldc, hipStream_t s, const int* guard, int prof) {
  if (M <= 0 || N <= 0) return PW_OK;
  pw::ProfScope ps(prof >= 0 ? prof : pw::PK_GEMM_NN, s, 2.0 * M * N * (double)K);
  k_dgemm_nn<T, TA, TB><<<dim3(ceil_div(M, BM), ceil_div(N, BN), 1), NT, 0, s>>>(M, N, K, alpha, A, lda, B, ldb,
                                                                                beta, C, ldc, guard);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

template pw_status pw::dgemm_tn<double, double, double>(int, int, int, const double*, long, const double*, long,
                                                        double, double, double, double*, int, bool, void*, size_t,
                                                        hipStream_t, int);
template pw_status pw::dgemm_tn<float, float, double>(int, int, int, const float*, long, const double*, long, double,
                                                      double, double, double*, int, bool, void*, size_t, hipStream_t,
                                                      int);
template pw_status pw::dgemm_nn<double, double, double>(int, int, int, double, const double*, long, const double*,
                                                        long, double, double*, long, hipStream_t, const int*, int);
template pw_status pw::dgemm_nn<float, float, float>(int, int, int, double, const float*, long, const float*, long,
                                                     double, double*, long, hipStream_t, const int*, int);
// float32 arithmetic on float64 operands (subspace products of the float32 stage)
template pw_status pw::dgemm_tn<float, double, double>(int, int, int, const double*, long, const double*, long,
                                                       double, double, double, double*, int, bool, void*, size_t,
                                                       hipStream_t, int);
template pw_status pw::dgemm_nn<float, double, double>(int, int, int, double, const double*, long, const double*,
                                                       long, double, double*, long, hipStream_t, const int*, int);
