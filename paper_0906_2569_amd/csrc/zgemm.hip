// Complex GEMMs on the matrix cores (v_mfma_f64_16x16x4f64 for float64,
// v_mfma_f32_16x16x4f32 for float32), used for the projector term of H.psi
// (<beta|psi>, then sum_j beta_j (D <beta|psi>)_j) and for the Davidson
// subspace products (phi^H H phi, phi^H phi, Ritz rotations).
//
// Complex products use three real MFMAs per 16x16x4 block (Gauss's product,
// as in the 3M complex GEMMs): t1 += Re A Re B, t2 += Im A Im B,
// t3 += (Re A + Im A)(Re B + Im B), and at the end Re C = t1 - t2,
// Im C = t3 - t1 - t2.  That is 6 M N K real flops on the matrix cores
// instead of the 8 of the four-product form.  The error bound of the
// imaginary part grows from about K u (|Re A||Im B| + |Im A||Re B|) to about
// K u (|Re A| + |Im A|)(|Re B| + |Im B|) (u the unit roundoff of the
// precision), a small constant factor on the same order.  Im A is negated
// once, at the LDS store, when A enters conjugated.  The four-product form
// is kept (kGauss = false) for comparison.
//
// Two shapes:
//   cn : C[m, n] = sum_k conj(A[k, m]) B[k, n]; A and B are stored as
//        K-contiguous columns (the plane-wave index runs fastest).  K is the
//        long plane-wave dimension, so K is split over workgroups and the
//        partial tiles are summed in a fixed order by a second kernel
//        (deterministic, no atomics).
//   nn : C[m, n] = alpha sum_k A[m, k] B[k, n] + beta C[m, n]; A is M-contiguous
//        (a block of plane-wave vectors), B K-contiguous (small coefficients).
#include <algorithm>

#include "plan.h"
#include "profile.h"

namespace {

template <typename T>
struct Mma;
template <>
struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Operand / result placement of the 16x16x4 MFMAs (64 lanes): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Result element q (0..3) of lane l
// is D[4 (l / 16) + q][l % 16] for the float32 instruction and
// D[4 q + l / 16][l % 16] for the float64 one (checked on gfx950).
template <typename T>
__device__ __forceinline__ int mrow(int lane, int q);
template <>
__device__ __forceinline__ int mrow<float>(int lane, int q) { return 4 * (lane >> 4) + q; }
template <>
__device__ __forceinline__ int mrow<double>(int lane, int q) { return 4 * q + (lane >> 4); }
__device__ __forceinline__ int mcol(int lane) { return lane & 15; }

// The float32 GEMM kernels are built for at least three waves per SIMD (at
// most 168 registers, spill-free): three 64x64 tiles then share a CU, and a
// product of 18277 x 128 rows and columns (572 tiles) is resident in one
// round.  The float64 ones hold three float64 accumulator sets (96
// registers) and are built for two waves per SIMD, each MFMA there taking
// twice as many cycles.
constexpr int BN = 64, BK = 16, NT = 256;
// Output tile rows per workgroup (BM) and waves per SIMD the kernels are
// built for.  The calbec-shaped product (k_gemm_cn) in float32 takes 128 rows
// (each wave a 64 x 32 block of 4 x 2 MFMA tiles: twice the products per
// operand byte loaded and per LDS read of a 64 x 64 tile; 22.4 against
// 23.7 ms at the 512-atom cell) at two waves per SIMD; the add-back
// (k_gemm_nn) keeps 64 rows, which measured faster there (20.9 against
// 21.4 ms), at three; float64 takes 64 rows at two waves per SIMD (its three
// accumulator sets).
template <typename T, bool CN>
struct GT {
  static constexpr int BM = (sizeof(T) == 4 && CN) ? 128 : 64;
  static constexpr int IM = BM / 32;   // 16-row MFMA tiles per wave (two waves along M)
  static constexpr int waves = (sizeof(T) == 4 && !CN) ? 3 : 2;
};

// Workgroups go to the 8 XCDs round-robin in linear launch order.  Each XCD is
// given one contiguous range of a work order in which tile y (YFAST) or tile x
// runs fastest, then the other, then z: the workgroups that read the same
// operand strips then run on one XCD at about the same time and share its L2.
template <bool YFAST>
__device__ __forceinline__ void xcd_block(int& bx, int& by, int& bz) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int T = gx * gy * gridDim.z;
  const int L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int x = L & 7, s = L >> 3, per = T >> 3, rem = T & 7;
  // XCD x holds slots s < per + (x < rem): a bijection onto [0, T)
  const int w = x < rem ? x * (per + 1) + s : rem * (per + 1) + (x - rem) * per + s;
  if (YFAST) {
    by = w % gy;
    bx = (w / gy) % gx;
  } else {
    bx = w % gx;
    by = (w / gx) % gy;
  }
  bz = w / (gx * gy);
}

template <typename T, int BM>
struct Tile {
  T ar[BK][BM + 1], ai[BK][BM + 1], br[BK][BN + 1], bi[BK][BN + 1];
};

// Accumulators of one wave's 32x32 quadrant (2x2 blocks of 16x16): a = t1,
// b = t2, c = t3 of the three-product form (a = Re C, b = Im C in the
// four-product form).
constexpr bool kGauss = true;

template <typename T, int IM>
struct CAcc {
  typedef typename Mma<T>::v4 v4;
  static constexpr bool k3 = kGauss;
  v4 a[IM][2], b[IM][2], c[IM][2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) a[i][j] = b[i][j] = c[i][j] = v4{0, 0, 0, 0};
  }
  __device__ __forceinline__ cpx<T> get(int i, int j, int q) const {
    if constexpr (k3) {
      const T t1 = a[i][j][q], t2 = b[i][j][q];
      return cpx<T>{t1 - t2, (c[i][j][q] - t1) - t2};
    } else {
      return cpx<T>{a[i][j][q], b[i][j][q]};
    }
  }
};

// One BK slice of a BM x 64 tile product held in LDS; each of the 4 waves
// owns a (BM / 2) x 32 block (IM x 2 MFMA tiles of 16 x 16).
template <typename T, int BM>
__device__ __forceinline__ void tile_mma(const Tile<T, BM>& t, CAcc<T, BM / 32>& acc, int wm, int wn, int lane) {
  constexpr int IM = BM / 32, WM = BM / 2;
  const int r = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int k4 = 0; k4 < BK; k4 += 4) {
    const int kk = k4 + kq;
    T ar[IM], ai[IM], br[2], bi[2];
#pragma unroll
    for (int i = 0; i < IM; ++i) {
      ar[i] = t.ar[kk][wm * WM + i * 16 + r];
      ai[i] = t.ai[kk][wm * WM + i * 16 + r];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      br[j] = t.br[kk][wn * 32 + j * 16 + r];
      bi[j] = t.bi[kk][wn * 32 + j * 16 + r];
    }
    if constexpr (CAcc<T, IM>::k3) {
      T sa[IM], sb[2];
#pragma unroll
      for (int i = 0; i < IM; ++i) sa[i] = ar[i] + ai[i];
#pragma unroll
      for (int j = 0; j < 2; ++j) sb[j] = br[j] + bi[j];
#pragma unroll
      for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc.a[i][j] = Mma<T>::run(ar[i], br[j], acc.a[i][j]);
          acc.b[i][j] = Mma<T>::run(ai[i], bi[j], acc.b[i][j]);
          acc.c[i][j] = Mma<T>::run(sa[i], sb[j], acc.c[i][j]);
        }
    } else {
#pragma unroll
      for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc.a[i][j] = Mma<T>::run(ar[i], br[j], acc.a[i][j]);
          acc.a[i][j] = Mma<T>::run(-ai[i], bi[j], acc.a[i][j]);
          acc.b[i][j] = Mma<T>::run(ar[i], bi[j], acc.b[i][j]);
          acc.b[i][j] = Mma<T>::run(ai[i], br[j], acc.b[i][j]);
        }
    }
  }
}

// partial[z][n][m] = sum_{k in chunk z} conj(A[m*lda + k]) B[n*ldb + k]
// gridDim.z = 2 nsplit for two products of one launch: z >= nsplit takes B1
// and writes the partials after those of the first product
template <typename T, typename TA, typename TB>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(GT<T, true>::waves)))
k_gemm_cn(int M, int N, int K, int kchunk, int nsplit, const cpx<TA>* __restrict__ A, int lda,
          const cpx<TB>* __restrict__ B0, const cpx<TB>* __restrict__ B1, int ldb, cpx<T>* __restrict__ P) {
  constexpr int BM = GT<T, true>::BM, IM = GT<T, true>::IM;
  __shared__ Tile<T, BM> t;
  int bx, by, bz;
  xcd_block<false>(bx, by, bz);   // the output tiles of one K chunk share an XCD
  const int m0 = bx * BM, n0 = by * BN;
  const int zs = bz % nsplit;
  const cpx<TB>* __restrict__ B = bz >= nsplit ? B1 : B0;
  const int kbeg = zs * kchunk, kend = min(K, kbeg + kchunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  CAcc<T, IM> acc;
  acc.zero();

  // the next K slice is loaded into registers while the current one is
  // multiplied out of LDS
  constexpr int PA = BM * BK / NT, PB = BN * BK / NT;
  cpx<TA> ra[PA];
  cpx<TB> rb[PB];
  auto load = [&](int k0) {
#pragma unroll
    for (int it = 0; it < PA; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int kk = idx % BK, mi = idx / BK;
      const int k = k0 + kk, m = m0 + mi;
      ra[it] = (m < M && k < kend) ? A[(size_t)m * lda + k] : cpx<TA>{TA(0), TA(0)};
    }
#pragma unroll
    for (int it = 0; it < PB; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int kk = idx % BK, ni = idx / BK;
      const int k = k0 + kk, n = n0 + ni;
      rb[it] = (n < N && k < kend) ? B[(size_t)n * ldb + k] : cpx<TB>{TB(0), TB(0)};
    }
  };
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int it = 0; it < PA; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int kk = idx % BK, mi = idx / BK;
      t.ar[kk][mi] = (T)ra[it].x;
      t.ai[kk][mi] = -(T)ra[it].y;  // conj(A)
    }
#pragma unroll
    for (int it = 0; it < PB; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int kk = idx % BK, ni = idx / BK;
      t.br[kk][ni] = (T)rb[it].x;
      t.bi[kk][ni] = (T)rb[it].y;
    }
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);
    tile_mma<T, BM>(t, acc, wm, wn, lane);
    __syncthreads();
  }
  cpx<T>* out = P + (size_t)bz * M * N;
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm * (BM / 2) + i * 16 + mrow<T>(lane, q);
        const int n = n0 + wn * 32 + j * 16 + mcol(lane);
        if (m < M && n < N) out[(size_t)n * M + m] = acc.get(i, j, q);
      }
}

// C[n*ldc + m] = alpha sum_k A[k*lda + m] B[n*ldb + k] + beta C[n*ldc + m]
// The z index of the grid selects the product: (A0, C0) or (A1, C1), same B (two products of
// one launch fill the device better than two launches).
// SPLIT: the z index is instead the K chunk [z kchunk, (z + 1) kchunk) of the one
// product (A0), whose partial tile goes to P[z][n][m] unscaled, for k_reduce.
template <typename T, typename TA, typename TB, bool SPLIT = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(GT<T, false>::waves)))
k_gemm_nn(int M, int N, int K, double alpha, const cpx<TA>* __restrict__ A0, const cpx<TA>* __restrict__ A1,
          int lda, const cpx<TB>* __restrict__ B, int ldb, double beta, c128* __restrict__ C0,
          c128* __restrict__ C1, int ldc, const int* __restrict__ guard, int kchunk = 0,
          cpx<T>* __restrict__ P = nullptr, const double* __restrict__ kin = nullptr,
          const c128* __restrict__ X = nullptr, int ldx = 0) {
  if (guard != nullptr && *guard != 0) return;
  int bx, by, bz;
  xcd_block<true>(bx, by, bz);    // the column tiles of one row strip of A share an XCD
  const cpx<TA>* __restrict__ A = (!SPLIT && bz) ? A1 : A0;
  c128* __restrict__ C = (!SPLIT && bz) ? C1 : C0;
  const int kbeg = SPLIT ? bz * kchunk : 0;
  const int kend = SPLIT ? min(K, kbeg + kchunk) : K;
  constexpr int BM = GT<T, false>::BM, IM = GT<T, false>::IM;
  __shared__ Tile<T, BM> t;
  const int m0 = bx * BM, n0 = by * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  CAcc<T, IM> acc;
  acc.zero();

  constexpr int PA = BM * BK / NT, PB = BN * BK / NT;
  cpx<TA> ra[PA];
  cpx<TB> rb[PB];
  auto load = [&](int k0) {
#pragma unroll
    for (int it = 0; it < PA; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int mi = idx % BM, kk = idx / BM;
      const int m = m0 + mi, k = k0 + kk;
      ra[it] = (m < M && k < kend) ? A[(size_t)k * lda + m] : cpx<TA>{TA(0), TA(0)};
    }
#pragma unroll
    for (int it = 0; it < PB; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int kk = idx % BK, ni = idx / BK;
      const int n = n0 + ni, k = k0 + kk;
      rb[it] = (n < N && k < kend) ? B[(size_t)n * ldb + k] : cpx<TB>{TB(0), TB(0)};
    }
  };
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int it = 0; it < PA; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int mi = idx % BM, kk = idx / BM;
      t.ar[kk][mi] = (T)ra[it].x;
      t.ai[kk][mi] = (T)ra[it].y;
    }
#pragma unroll
    for (int it = 0; it < PB; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int kk = idx % BK, ni = idx / BK;
      t.br[kk][ni] = (T)rb[it].x;
      t.bi[kk][ni] = (T)rb[it].y;
    }
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);
    tile_mma<T, BM>(t, acc, wm, wn, lane);
    __syncthreads();
  }
  if constexpr (SPLIT) {
    cpx<T>* out = P + (size_t)bz * M * N;
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int m = m0 + wm * (BM / 2) + i * 16 + mrow<T>(lane, q);
          const int n = n0 + wn * 32 + j * 16 + mcol(lane);
          if (m < M && n < N) out[(size_t)n * M + m] = acc.get(i, j, q);
        }
    return;
  }
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm * (BM / 2) + i * 16 + mrow<T>(lane, q);
        const int n = n0 + wn * 32 + j * 16 + mcol(lane);
        if (m < M && n < N) {
          c128* c = C + (size_t)n * ldc + m;
          const cpx<T> v = acc.get(i, j, q);
          double re = alpha * (double)v.x, im = alpha * (double)v.y;
          if (beta != 0.0) {
            const c128 old = *c;
            re += beta * old.x;
            im += beta * old.y;
          }
          if (kin != nullptr) {   // + diag(kin) X (kinetic term of H.psi)
            const c128 x = X[(size_t)n * ldx + m];
            re += kin[m] * x.x;
            im += kin[m] * x.y;
          }
          *c = c128{re, im};
        }
      }
}

// In k_reduce the split-K partials of one output element are summed by RZ
// thread groups:
// group y adds the partials z in [y nsplit / RZ, (y + 1) nsplit / RZ) in
// increasing z, then the RZ group sums are added in increasing y.  The order
// is fixed, so results are reproducible, and the groups keep RZ times more
// loads in flight than one thread per element would.
constexpr int RZ = 4;

// sum_z P[z * stride + off] for z0 <= z < z1 in increasing z; the loads of
// eight partials are issued before they are added
template <typename T>
__device__ __forceinline__ cpx<T> sum_partials(const cpx<T>* __restrict__ P, int z0, int z1, size_t stride,
                                               size_t off) {
  T re = 0, im = 0;
  int z = z0;
  for (; z + 8 <= z1; z += 8) {
    cpx<T> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = P[(size_t)(z + u) * stride + off];
#pragma unroll
    for (int u = 0; u < 8; ++u) { re += v[u].x; im += v[u].y; }
  }
  for (; z < z1; ++z) {
    const cpx<T> v = P[(size_t)z * stride + off];
    re += v.x;
    im += v.y;
  }
  return cpx<T>{re, im};
}

template <typename T>
__device__ __forceinline__ cpx<T> add_groups(const cpx<T> (*s)[64], int x) {
  cpx<T> v = s[0][x];
#pragma unroll
  for (int y = 1; y < RZ; ++y) v = cpx<T>{v.x + s[y][x].x, v.y + s[y][x].y};
  return v;
}

// C[n*ldc + m] = alpha sum_z P[z][n][m] + beta Cin[n*ldcin + m]; block (64, RZ).
// Cin = C (in place) unless another matrix is given.  gridDim.y = 2 sums two
// products in one launch: blockIdx.y = 1 takes the partials after the first
// product's (nsplit M N of them) into C1.
template <typename T>
__global__ void __launch_bounds__(64 * RZ) k_reduce(int M, int N, int nsplit, const cpx<T>* __restrict__ P0,
                                                    c128* __restrict__ C0, c128* __restrict__ C1, int ldc,
                                                    double alpha, double beta, const c128* __restrict__ Cin = nullptr,
                                                    int ldcin = 0) {
  __shared__ cpx<T> s[RZ][64];
  const cpx<T>* __restrict__ P = P0 + (size_t)blockIdx.y * nsplit * M * N;
  c128* __restrict__ C = blockIdx.y ? C1 : C0;
  const size_t total = (size_t)M * N;
  const int x = threadIdx.x, y = threadIdx.y;
  const int z0 = y * nsplit / RZ, z1 = (y + 1) * nsplit / RZ;
  // the loop bound depends on the block only, so every thread reaches the barriers
  for (size_t base = (size_t)blockIdx.x * 64; base < total; base += (size_t)gridDim.x * 64) {
    const size_t idx = base + x;
    if (idx < total) s[y][x] = sum_partials(P, z0, z1, total, idx);
    __syncthreads();
    if (y == 0 && idx < total) {
      const cpx<T> sum = add_groups<T>(s, x);
      const int m = (int)(idx % M), n = (int)(idx / M);
      c128* c = C + (size_t)n * ldc + m;
      double r = alpha * (double)sum.x, i = alpha * (double)sum.y;
      if (beta != 0.0) {
        const c128 cin = Cin ? Cin[(size_t)n * ldcin + m] : *c;
        r += beta * cin.x;
        i += beta * cin.y;
      }
      *c = c128{r, i};
    }
    __syncthreads();
  }
}

// One workgroup per band n: becp[j] = sum_z P[z][n][j] into LDS, then
// out[n][j] = sum_{t < dlen_j} drow[j][t] becp[dstart_j + t].  It runs beside
// the transform passes, so its workgroups stay small (256 threads) to find
// room on CUs those passes occupy.
template <typename T>
__global__ void k_reduce_dapply(int M, int N, int nsplit, const cpx<T>* __restrict__ P,
                                const int* __restrict__ dstart, const int* __restrict__ dlen,
                                const cpx<T>* __restrict__ drow, int nhmax,
                                cpx<T>* __restrict__ out) {
  extern __shared__ __align__(16) char smem_raw[];
  cpx<T>* red = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n = blockIdx.x;
  const size_t total = (size_t)M * N;
  for (int j = threadIdx.x; j < M; j += blockDim.x)
    red[j] = sum_partials(P, 0, nsplit, total, (size_t)n * M + j);
  __syncthreads();
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    const int j0 = dstart[j], nh = dlen[j];
    cpx<T> acc{T(0), T(0)};
    for (int t = 0; t < nh; ++t) acc = acc + cmul(drow[(size_t)j * nhmax + t], red[j0 + t]);
    out[(size_t)n * M + j] = acc;
  }
}

struct Split {
  int nsplit, kchunk;
};

Split choose_split(int M, int N, int K, int BM) {
  const int tiles = ceil_div(M, BM) * ceil_div(N, BN);
  const int target = 512;
  int nsplit = std::max(1, ceil_div(target, tiles));
  // A long K splits into at least one chunk per XCD even when the tiles alone
  // fill the device: the work order then gives each XCD its own K range, and
  // every operand element is read from memory once instead of by every tile
  // row or column (calbec of the 512-atom cell read its operands 9 times)
  if (nsplit < 8 && K >= 8 * 256 * BK) nsplit = 8;
  nsplit = std::min(nsplit, std::max(1, ceil_div(K, 4 * BK)));
  int kchunk = ceil_div(ceil_div(K, nsplit), BK) * BK;
  kchunk = std::max(kchunk, BK);
  nsplit = std::max(1, ceil_div(K, kchunk));
  return Split{nsplit, kchunk};
}

}  // namespace

size_t pw::splitk_part_bytes(int M, int N, int K, int elem_bytes) {
  // Upper bound over every M' <= M, N' <= N: nsplit <= 512/tiles + 1, so
  // nsplit M' N' <= 512 BM BN + M N; a long K adds the 8-chunk minimum.
  // Complex64 partials come from the 128-row tiles, complex128 ones from the
  // 64-row tiles; a complex128-sized bound covers the complex64 partials of
  // the same product (512 x 128 x 64 x 8 B = 512 x 64 x 64 x 16 B).
  const size_t mn = (size_t)std::max(M, 1) * std::max(N, 1);
  const size_t bm = elem_bytes <= 8 ? (size_t)GT<float, true>::BM : (size_t)GT<double, true>::BM;
  size_t e = (size_t)512 * bm * BN + mn;
  if (K >= 8 * 256 * BK) e = std::max(e, 8 * mn);
  return e * elem_bytes + 256;
}

template <typename T, typename TA, typename TB>
pw_status pw::zgemm_cn(int M, int N, int K, const cpx<TA>* A, int lda, const cpx<TB>* B, int ldb,
                       c128* C, int ldc, void* part, size_t part_bytes, hipStream_t s, double alpha,
                       double beta, const c128* Cin, int ldcin) {
  if (M <= 0 || N <= 0) return PW_OK;
  const Split sp = choose_split(M, N, K, GT<T, true>::BM);
  const size_t need = (size_t)sp.nsplit * M * N * sizeof(cpx<T>);
  PW_CHECK(need <= part_bytes, PW_ENOMEM, "split-K workspace too small");
  cpx<T>* P = static_cast<cpx<T>*>(part);
  if (K <= 0) {
    // a sum over no partials is zero: C = beta C
    k_reduce<T><<<std::min(4096, ceil_div((size_t)M * N, 64)), dim3(64, RZ), 0, s>>>(M, N, 0, P, C, C, ldc,
                                                                                   alpha, beta, Cin, ldcin);
    PW_HIP(hipGetLastError());
    return PW_OK;
  }
  {
    pw::ProfScope ps(pw::PK_GEMM_CN, s, 8.0 * M * N * K);
    k_gemm_cn<T, TA, TB><<<dim3(ceil_div(M, GT<T, true>::BM), ceil_div(N, BN), sp.nsplit), NT, 0, s>>>(
        M, N, K, sp.kchunk, sp.nsplit, A, lda, B, B, ldb, P);
  }
  {
    pw::ProfScope ps(pw::PK_GEMM_RED, s, (double)sp.nsplit * M * N * sizeof(cpx<T>) + 16.0 * M * N);
    k_reduce<T><<<std::min(4096, ceil_div((size_t)M * N, 64)), dim3(64, RZ), 0, s>>>(M, N, sp.nsplit, P, C, C,
                                                                                   ldc, alpha, beta, Cin, ldcin);
  }
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw::zgemm_cn_pair(int M, int N, int K, const c128* A, int lda, const c128* B0, const c128* B1,
                            int ldb, c128* C0, c128* C1, int ldc, void* part, size_t part_bytes, hipStream_t s) {
  if (M <= 0 || N <= 0) return PW_OK;
  Split sp = choose_split(M, N, K, GT<double, true>::BM);
  // half the splits per product: the two products together fill the device
  const int ns = std::max(1, sp.nsplit / 2);
  const int kchunk = std::max(BK, ceil_div(ceil_div(K, ns), BK) * BK);
  const int nsplit = std::max(1, ceil_div(K, kchunk));
  const size_t need = 2 * (size_t)nsplit * M * N * sizeof(c128);
  if (K <= 0 || need > part_bytes) {
    PW_TRY((zgemm_cn<double, double, double>(M, N, K, A, lda, B0, ldb, C0, ldc, part, part_bytes, s)));
    return zgemm_cn<double, double, double>(M, N, K, A, lda, B1, ldb, C1, ldc, part, part_bytes, s);
  }
  c128* P = static_cast<c128*>(part);
  {
    pw::ProfScope ps(pw::PK_GEMM_CN, s, 16.0 * M * N * K);
    k_gemm_cn<double, double, double><<<dim3(ceil_div(M, GT<double, true>::BM), ceil_div(N, BN), 2 * nsplit), NT, 0, s>>>(
        M, N, K, kchunk, nsplit, A, lda, B0, B1, ldb, P);
  }
  {
    pw::ProfScope ps(pw::PK_GEMM_RED, s, 2.0 * ((double)nsplit * M * N * sizeof(c128) + 16.0 * M * N));
    const int g = std::min(4096, ceil_div((size_t)M * N, 64));
    k_reduce<double><<<dim3(g, 2), dim3(64, RZ), 0, s>>>(M, N, nsplit, P, C0, C1, ldc, 1.0, 0.0);
  }
  PW_HIP(hipGetLastError());
  return PW_OK;
}

template <typename T>
pw_status pw::calbec_d(pw_plan p, int nb, const c128* psi, int ldpsi, cpx<T>* out, hipStream_t s,
                       const cpx<T>* rows) {
  const int M = p->nbeta, N = nb, K = p->npw;
  const Split sp = choose_split(M, N, K, GT<T, true>::BM);
  const size_t need = (size_t)sp.nsplit * M * N * sizeof(cpx<T>);
  PW_CHECK(need <= p->part_bytes, PW_ENOMEM, "split-K workspace too small");
  cpx<T>* P = static_cast<cpx<T>*>(p->part);
  const cpx<T>* beta = sizeof(T) == 8 ? (const cpx<T>*)p->beta64 : (const cpx<T>*)p->beta32;
  const cpx<T>* drow = rows ? rows : (sizeof(T) == 8 ? (const cpx<T>*)p->drow64 : (const cpx<T>*)p->drow32);
  {
    pw::ProfScope ps(pw::PK_CALBEC, s, 8.0 * M * N * K);
    k_gemm_cn<T, T, double><<<dim3(ceil_div(M, GT<T, true>::BM), ceil_div(N, BN), sp.nsplit), NT, 0, s>>>(
        M, N, K, sp.kchunk, sp.nsplit, beta, p->ldb, psi, psi, ldpsi, P);
  }
  {
    pw::ProfScope ps(pw::PK_CALBEC_RED, s, (double)sp.nsplit * M * N * sizeof(cpx<T>) + (double)M * N * sizeof(cpx<T>));
    k_reduce_dapply<T><<<N, 256, sizeof(cpx<T>) * M, s>>>(M, N, sp.nsplit, P, p->dstart, p->dlen,
                                                        drow, p->nhmax, out);
  }
  PW_HIP(hipGetLastError());
  return PW_OK;
}

template <typename T, typename TA, typename TB>
pw_status pw::zgemm_nn(int M, int N, int K, double alpha, const cpx<TA>* A, int lda,
                       const cpx<TB>* B, int ldb, double beta, c128* C, int ldc, hipStream_t s,
                       const int* guard, const double* kin, const c128* X, int ldx) {
  if (M <= 0 || N <= 0) return PW_OK;
  pw::ProfScope ps(pw::PK_GEMM_NN, s, 8.0 * M * N * K);
  k_gemm_nn<T, TA, TB><<<dim3(ceil_div(M, GT<T, false>::BM), ceil_div(N, BN), 1), NT, 0, s>>>(
      M, N, K, alpha, A, A, lda, B, ldb, beta, C, C, ldc, guard, 0, nullptr, kin, X, ldx);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw::zgemm_nn_sk(int M, int N, int K, double alpha, const c128* A, int lda, const c128* B, int ldb,
                          double beta, c128* C, int ldc, void* part, size_t part_bytes, hipStream_t s) {
  if (M <= 0 || N <= 0) return PW_OK;
  const int tiles = ceil_div(M, GT<double, false>::BM) * ceil_div(N, BN);
  // chunks of at least two K slices, up to about 512 workgroups in all
  const int ns = std::min(ceil_div(512, tiles), ceil_div(K, 2 * BK));
  const int kchunk = std::max(BK, ceil_div(ceil_div(K, std::max(ns, 1)), BK) * BK);
  const int nsplit = ceil_div(K, kchunk);
  const size_t need = (size_t)nsplit * M * N * sizeof(c128);
  if (tiles >= 128 || nsplit < 2 || need > part_bytes)
    return zgemm_nn<double, double, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
  c128* P = static_cast<c128*>(part);
  {
    pw::ProfScope ps(pw::PK_GEMM_NN, s, 8.0 * M * N * K);
    k_gemm_nn<double, double, double, true><<<dim3(ceil_div(M, GT<double, false>::BM), ceil_div(N, BN), nsplit), NT, 0, s>>>(
        M, N, K, 1.0, A, A, lda, B, ldb, 0.0, nullptr, nullptr, ldc, nullptr, kchunk, P);
  }
  {
    pw::ProfScope ps(pw::PK_GEMM_RED, s, (double)nsplit * M * N * sizeof(c128) + 16.0 * M * N);
    k_reduce<double><<<std::min(4096, ceil_div((size_t)M * N, 64)), dim3(64, RZ), 0, s>>>(M, N, nsplit, P, C, C,
                                                                                         ldc, alpha, beta);
  }
  PW_HIP(hipGetLastError());
  return PW_OK;
}

template <typename T>
pw_status pw::zgemm_nn_pair(int M, int N, int K, const c128* A0, const c128* A1, int lda, const c128* B,
                            int ldb, c128* C0, c128* C1, int ldc, hipStream_t s, const int* guard) {
  if (M <= 0 || N <= 0) return PW_OK;
  pw::ProfScope ps(pw::PK_GEMM_NN, s, 16.0 * M * N * K);
  k_gemm_nn<T, double, double><<<dim3(ceil_div(M, GT<T, false>::BM), ceil_div(N, BN), 2), NT, 0, s>>>(
      M, N, K, 1.0, A0, A1, lda, B, ldb, 0.0, C0, C1, ldc, guard);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

template pw_status pw::zgemm_nn_pair<double>(int, int, int, const c128*, const c128*, int, const c128*, int, c128*,
                                             c128*, int, hipStream_t, const int*);
template pw_status pw::zgemm_nn_pair<float>(int, int, int, const c128*, const c128*, int, const c128*, int, c128*,
                                            c128*, int, hipStream_t, const int*);
template pw_status pw::zgemm_cn<double, double, double>(int, int, int, const c128*, int, const c128*,
                                                        int, c128*, int, void*, size_t, hipStream_t,
                                                        double, double, const c128*, int);
template pw_status pw::zgemm_cn<float, double, double>(int, int, int, const c128*, int, const c128*,
                                                       int, c128*, int, void*, size_t, hipStream_t,
                                                       double, double, const c128*, int);
template pw_status pw::calbec_d<double>(pw_plan, int, const c128*, int, c128*, hipStream_t, const c128*);
template pw_status pw::calbec_d<float>(pw_plan, int, const c128*, int, c64*, hipStream_t, const c64*);
template pw_status pw::zgemm_nn<double, double, double>(int, int, int, double, const c128*, int,
                                                        const c128*, int, double, c128*, int,
                                                        hipStream_t, const int*, const double*, const c128*,
                                                        int);
template pw_status pw::zgemm_nn<float, float, float>(int, int, int, double, const c64*, int,
                                                     const c64*, int, double, c128*, int,
                                                     hipStream_t, const int*, const double*, const c128*,
                                                     int);
template pw_status pw::zgemm_nn<float, double, double>(int, int, int, double, const c128*, int,
                                                       const c128*, int, double, c128*, int,
                                                        hipStream_t, const int*, const double*, const c128*,
                                                        int);
