// Float64 dense linear algebra for the Davidson reduced problem, on the GPU.
//
// The reduced problem of the block Davidson iteration is the generalized
// Hermitian eigenproblem  H_red c = eps S_red c  on the current basis
// (the "conventional algorithms for matrix diagonalization" step).  It is
// solved as
//   S = L L^H (Cholesky),  X = L^-H,  A = X^H H X,
//   A = Q T Q^H (Householder tridiagonalization, T real symmetric),
//   lowest nev eigenvalues of T by multisection bisection on Sturm counts,
//   eigenvectors of T by inverse iteration (reorthogonalized inside clusters
//   of equal eigenvalues), back-transformed by the reflectors, and c = X Y.
// The matrix products run on the MFMA GEMMs of zgemm.hip; the sequential
// factorizations run inside one workgroup each.
#include <cfloat>
#include <cmath>

#include <mutex>
#include <string>

#include "linalg.h"
#include "profile.h"

namespace {

constexpr int NTL = 1024;  // threads of the single-workgroup factorizations
// release flags of the cooperative tridiagonalization's barrier, 128 bytes
// apart (workgroup q polls flag q mod kGoLines)
constexpr int kGoLines = 8;
constexpr int kGoMinP = 24;   // up to this many workgroups the counter itself is polled

__device__ __forceinline__ c128 cconj(c128 a) { return c128{a.x, -a.y}; }

// block-wide sum of a double (all threads call; result valid in all threads)
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];   // fixed order: deterministic
  __syncthreads();
  return s;
}

__device__ c128 block_sum_c(c128 v, double* red) {
  const double re = block_sum(v.x, red);
  const double im = block_sum(v.y, red);
  return c128{re, im};
}


// partial[s * m + i] = sum_{j = s, s + ns, ...} S[j * ld + i] v[j]: four
// independent accumulators keep several L2 loads in flight per thread
__device__ __forceinline__ void matvec_slices(int m, int ns, const c128* __restrict__ S, int ld,
                                              const c128* __restrict__ v, c128* __restrict__ part) {
  for (int idx = threadIdx.x; idx < m * ns; idx += blockDim.x) {
    const int i = idx % m, sl = idx / m;
    double r0 = 0, i0 = 0, r1 = 0, i1 = 0, r2 = 0, i2 = 0, r3 = 0, i3 = 0;
    int j = sl;
    for (; j + 3 * ns < m; j += 4 * ns) {
      const c128 a0 = S[(size_t)j * ld + i], a1 = S[(size_t)(j + ns) * ld + i];
      const c128 a2 = S[(size_t)(j + 2 * ns) * ld + i], a3 = S[(size_t)(j + 3 * ns) * ld + i];
      const c128 b0 = v[j], b1 = v[j + ns], b2 = v[j + 2 * ns], b3 = v[j + 3 * ns];
      r0 += a0.x * b0.x - a0.y * b0.y; i0 += a0.x * b0.y + a0.y * b0.x;
      r1 += a1.x * b1.x - a1.y * b1.y; i1 += a1.x * b1.y + a1.y * b1.x;
      r2 += a2.x * b2.x - a2.y * b2.y; i2 += a2.x * b2.y + a2.y * b2.x;
      r3 += a3.x * b3.x - a3.y * b3.y; i3 += a3.x * b3.y + a3.y * b3.x;
    }
    for (; j < m; j += ns) {
      const c128 a0 = S[(size_t)j * ld + i], b0 = v[j];
      r0 += a0.x * b0.x - a0.y * b0.y; i0 += a0.x * b0.y + a0.y * b0.x;
    }
    part[idx] = c128{(r0 + r1) + (r2 + r3), (i0 + i1) + (i2 + i3)};
  }
}

// ---------------------------------------------------------------------------
// Cholesky S = L L^H (lower), in place on a copy of S, dropping dependent
// directions: a pivot below drop_tol times the original diagonal entry (a
// basis vector that lies, to rounding, in the span of the earlier ones) gets
// L[j][j] = 1 and a zero column, and drop[j] = 1.  info = 1 when fewer than
// nev directions remain or a pivot is not finite.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NTL) k_chol(int n, int nev, double drop_tol, c128* __restrict__ L, int ld,
                                              int* __restrict__ drop, int* __restrict__ info) {
  extern __shared__ __align__(16) char smem_raw[];
  c128* col = reinterpret_cast<c128*>(smem_raw);               // [n]
  double* diag0 = reinterpret_cast<double*>(col + n);          // [n]
  __shared__ double s_r;
  __shared__ int s_keep, s_bad, s_ndrop;
  if (threadIdx.x == 0) { s_bad = 0; s_ndrop = 0; }
  for (int i = threadIdx.x; i < n; i += blockDim.x) diag0[i] = L[(size_t)i * ld + i].x;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      const double d = L[(size_t)j * ld + j].x;
      // a dependent direction leaves a pivot at rounding level (a zero basis
      // vector a zero one); a clearly negative pivot (or a negative diagonal)
      // means S is not positive definite
      if (!isfinite(d) || !(diag0[j] >= 0.0) || d < -drop_tol * diag0[j]) s_bad = 1;
      s_keep = (d > drop_tol * diag0[j]) ? 1 : 0;
      if (s_keep) {
        s_r = sqrt(d);
        L[(size_t)j * ld + j] = c128{s_r, 0.0};
      } else {
        L[(size_t)j * ld + j] = c128{1.0, 0.0};
        ++s_ndrop;
      }
      drop[j] = 1 - s_keep;
    }
    __syncthreads();
    if (s_bad) break;
    const int m = n - j - 1;
    if (!s_keep) {
      for (int i = threadIdx.x; i < m; i += blockDim.x) L[(size_t)j * ld + j + 1 + i] = c128{0.0, 0.0};
      __syncthreads();
      continue;
    }
    const double inv = 1.0 / s_r;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      c128 v = L[(size_t)j * ld + j + 1 + i];
      v = c128{v.x * inv, v.y * inv};
      L[(size_t)j * ld + j + 1 + i] = v;
      col[i] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      const int ii = idx % m, kk = idx / m;
      if (ii >= kk) {
        c128* a = L + (size_t)(j + 1 + kk) * ld + j + 1 + ii;
        const c128 u = cmulc(col[kk], col[ii]);   // col[ii] conj(col[kk])
        *a = c128{a->x - u.x, a->y - u.y};
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *info = (s_bad || n - s_ndrop < nev) ? 1 : 0;
  // zero the strict upper triangle (the factor is used as a full matrix)
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, k = idx / n;
    if (i < k) L[(size_t)k * ld + i] = c128{0.0, 0.0};
  }
}

// The same factorization with the matrix in registers, for n <= 128: the
// 32 x 32 threads of one workgroup each hold a 4 x 4 set of entries (rows
// tr + 32 p, columns tc + 32 q), so the rank-1 updates touch no memory.  Step
// j reads column j as published (unscaled) by its owners at the end of step
// j - 1 through LDS (two buffers by parity, one barrier per column); every
// thread takes the same pivot decision from the same values.  Operations
// and their order per entry are those of k_chol.
constexpr int kChRegSlots = 4;
constexpr int kChRegN = 32 * kChRegSlots;
// It also does the rank check over all n_all directions of the basis (this
// block is the last n of them; drop_all holds the flags of the earlier rows):
// info = 1 when fewer than nev_all remain.
__global__ void __launch_bounds__(1024) k_chol_reg(int n, int nev, double drop_tol, c128* __restrict__ L, int ld,
                                                  int* __restrict__ drop, int* __restrict__ info,
                                                  const int* __restrict__ drop_all, int n_all, int nev_all) {
  constexpr int S = kChRegSlots;
  __shared__ c128 s_col[2][kChRegN];
  __shared__ double s_diag0[kChRegN];
  const int tr = threadIdx.x & 31, tc = threadIdx.x >> 5;
  c128 a[S][S];
#pragma unroll
  for (int p = 0; p < S; ++p)
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int i = tr + 32 * p, k = tc + 32 * q;
      a[p][q] = (i < n && k < n) ? L[(size_t)k * ld + i] : c128{0.0, 0.0};
    }
  for (int i = threadIdx.x; i < n; i += blockDim.x) s_diag0[i] = L[(size_t)i * ld + i].x;
  if (tc == 0) {
#pragma unroll
    for (int p = 0; p < S; ++p)
      if (tr + 32 * p < n) s_col[0][tr + 32 * p] = a[p][0];
  }
  __syncthreads();
  bool bad = false;
  int ndrop = 0;
  // column j = 32 qj + jj: the slot qj of its entries is a compile-time
  // index in each unrolled copy (no selects over the register array)
#pragma unroll
  for (int qj = 0; qj < S; ++qj) {
    if (bad) break;
    for (int jj = 0; jj < 32; ++jj) {
      const int j = 32 * qj + jj;
      if (j >= n) break;
      const int b = j & 1;
      const double d = s_col[b][j].x;
      const double d0 = s_diag0[j];
      if (!isfinite(d) || !(d0 >= 0.0) || d < -drop_tol * d0) {
        bad = true;   // the same decision in every thread
        break;
      }
      const bool keep = d > drop_tol * d0;
      const double r = keep ? sqrt(d) : 1.0;
      const double inv = keep ? 1.0 / r : 0.0;
      ndrop += keep ? 0 : 1;
      if (threadIdx.x == 0) drop[j] = keep ? 0 : 1;
      // column j of L in its owners' registers: r on the diagonal, a / r below
      // (a dropped direction: 1 and zeros)
      if (tc == jj) {
#pragma unroll
        for (int p = 0; p < S; ++p) {
          const int i = tr + 32 * p;
          if (i == j) a[p][qj] = c128{r, 0.0};
          else if (i > j) a[p][qj] = c128{a[p][qj].x * inv, a[p][qj].y * inv};
        }
      }
      // trailing update L22 -= l l^H on the lower triangle, l_i = col_i / r
      if (keep) {
#pragma unroll
        for (int q = qj; q < S; ++q) {
          const int k = tc + 32 * q;
          if (k <= j || k >= n) continue;
          const c128 ck = s_col[b][k];
          const c128 lk = c128{ck.x * inv, ck.y * inv};
#pragma unroll
          for (int p = q; p < S; ++p) {
            const int i = tr + 32 * p;
            if (i < k || i >= n) continue;
            const c128 ci = s_col[b][i];
            const c128 li = c128{ci.x * inv, ci.y * inv};
            const c128 u = cmulc(lk, li);   // l_i conj(l_k)
            a[p][q] = c128{a[p][q].x - u.x, a[p][q].y - u.y};
          }
        }
      }
      // publish column j + 1 (updated, unscaled) for the next step
      const int j1 = j + 1;
      if (j1 < n && tc == (j1 & 31)) {
        if (jj < 31) {
#pragma unroll
          for (int p = 0; p < S; ++p) {
            const int i = tr + 32 * p;
            if (i >= j1 && i < n) s_col[b ^ 1][i] = a[p][qj];
          }
        } else if (qj + 1 < S) {
#pragma unroll
          for (int p = 0; p < S; ++p) {
            const int i = tr + 32 * p;
            if (i >= j1 && i < n) s_col[b ^ 1][i] = a[p][qj + 1];
          }
        }
      }
      __syncthreads();
    }
  }
  // rank check: the rows before this block (drop_all[0, n_all - n), from
  // earlier factorizations) plus this block's n - ndrop kept directions
  __shared__ int s_kept;
  if (threadIdx.x == 0) s_kept = 0;
  __syncthreads();
  int kept = 0;
  for (int i = threadIdx.x; i < n_all - n; i += blockDim.x) kept += drop_all[i] ? 0 : 1;
  atomicAdd(&s_kept, kept);
  __syncthreads();
  if (threadIdx.x == 0) *info = (bad || n - ndrop < nev || s_kept + (n - ndrop) < nev_all) ? 1 : 0;
  // the factor, with the strict upper triangle cleared (it is used as a full matrix)
#pragma unroll
  for (int p = 0; p < S; ++p)
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int i = tr + 32 * p, k = tc + 32 * q;
      if (i < n && k < n) L[(size_t)k * ld + i] = (i >= k) ? a[p][q] : c128{0.0, 0.0};
    }
}

// Blocked form of the same factorization for large n (right-looking): each
// panel of kChPanel columns is factored with the rule above (k_chol_diag,
// k_chol_trsm below: only the panel's own columns are updated), the
// trailing matrix then receives the panel's rank-kChPanel update as one MFMA
// product
//   L22 -= L21 L21^H   (zgemm with the conjugate transpose PT of L21),
// and a last kernel sets info and clears the strict upper triangle.
// flags[0] = not positive definite (also the guard that skips the products).
constexpr int kChPanel = 32;
constexpr int kChBlockedMinN = 192;

__global__ void k_chol_init(int n, const c128* __restrict__ L, int ld, double* __restrict__ diag0,
                            int* __restrict__ flags) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    diag0[i] = L[(size_t)i * ld + i].x;
  if (blockIdx.x == 0 && threadIdx.x == 0) flags[0] = 0;
}

// A panel in two kernels: its bb x bb diagonal block factored in LDS by one
// workgroup (the drop rule above), then the rows below solved against it,
// L21 = A21 L11^-H, one row per thread over as many workgroups as there are
// rows (57 us a panel at 1000-2000 rows, against 180 us for one workgroup
// updating the whole panel through memory column by column).
__global__ void __launch_bounds__(256) k_chol_diag(int j0, int bb, double drop_tol, c128* __restrict__ L, int ld,
                                                   const double* __restrict__ diag0, int* __restrict__ drop,
                                                   int* __restrict__ flags) {
  if (flags[0] != 0) return;
  __shared__ c128 a[kChPanel][kChPanel + 1];   // a[r][c]: row r, column c of the block (lower triangle)
  __shared__ double s_r;
  __shared__ int s_keep, s_bad;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < bb * bb; idx += blockDim.x) {
    const int r = idx % bb, c = idx / bb;
    if (r >= c) a[r][c] = L[(size_t)(j0 + c) * ld + j0 + r];
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int j = 0; j < bb; ++j) {
    if (tid == 0) {
      const double d = a[j][j].x, d0 = diag0[j0 + j];
      if (!isfinite(d) || !(d0 >= 0.0) || d < -drop_tol * d0) s_bad = 1;
      s_keep = (d > drop_tol * d0) ? 1 : 0;
      s_r = s_keep ? sqrt(d) : 1.0;
      a[j][j] = c128{s_r, 0.0};
      drop[j0 + j] = 1 - s_keep;
      if (s_bad) flags[0] = 1;
    }
    __syncthreads();
    if (s_bad) return;
    // column j below the diagonal: scaled, or zero for a dropped direction
    const double inv = s_keep ? 1.0 / s_r : 0.0;
    for (int i = j + 1 + tid; i < bb; i += blockDim.x) a[i][j] = c128{a[i][j].x * inv, a[i][j].y * inv};
    __syncthreads();
    if (s_keep) {
      const int w = bb - j - 1;
      for (int idx = tid; idx < w * w; idx += blockDim.x) {
        const int ii = j + 1 + idx % w, kk = j + 1 + idx / w;
        if (ii >= kk) {
          const c128 u = cmulc(a[kk][j], a[ii][j]);   // L[ii][j] conj(L[kk][j])
          a[ii][kk] = c128{a[ii][kk].x - u.x, a[ii][kk].y - u.y};
        }
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < bb * bb; idx += blockDim.x) {
    const int r = idx % bb, c = idx / bb;
    if (r >= c) L[(size_t)(j0 + c) * ld + j0 + r] = a[r][c];
  }
}

// rows jend .. n-1 of the panel: x L11^H = a, column c of x zero where
// direction c was dropped; also PT[r * kChPanel + c] = conj(x_c) for the
// trailing product
__global__ void __launch_bounds__(256) k_chol_trsm(int n, int j0, int bb, c128* __restrict__ L, int ld,
                                                   const int* __restrict__ drop, const int* __restrict__ flags,
                                                   c128* __restrict__ PT) {
  if (flags[0] != 0) return;
  __shared__ c128 l11[kChPanel][kChPanel + 1];
  __shared__ int s_drop[kChPanel];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < bb * bb; idx += blockDim.x) {
    const int r = idx % bb, c = idx / bb;
    l11[r][c] = (r >= c) ? L[(size_t)(j0 + c) * ld + j0 + r] : c128{0.0, 0.0};
  }
  if (tid < bb) s_drop[tid] = drop[j0 + tid];
  __syncthreads();
  const int jend = j0 + bb, mt = n - jend;
  const int r = blockIdx.x * blockDim.x + tid;
  if (r >= mt) return;
  c128 x[kChPanel];
#pragma unroll
  for (int c = 0; c < kChPanel; ++c) x[c] = c < bb ? L[(size_t)(j0 + c) * ld + jend + r] : c128{0.0, 0.0};
#pragma unroll
  for (int c = 0; c < kChPanel; ++c) {
    if (c < bb) {
      if (s_drop[c]) {
        x[c] = c128{0.0, 0.0};
      } else {
        c128 v = x[c];
#pragma unroll
        for (int t = 0; t < c; ++t) {
          const c128 u = cmulc(l11[c][t], x[t]);   // x_t conj(L11[c][t])
          v = c128{v.x - u.x, v.y - u.y};
        }
        const double inv = 1.0 / l11[c][c].x;
        x[c] = c128{v.x * inv, v.y * inv};
      }
    }
  }
#pragma unroll
  for (int c = 0; c < kChPanel; ++c)
    if (c < bb) {
      L[(size_t)(j0 + c) * ld + jend + r] = x[c];
      PT[(size_t)r * kChPanel + c] = cconj(x[c]);
    }
}

__global__ void k_chol_finish(int n, c128* __restrict__ L, int ld, const int* __restrict__ flags,
                              int* __restrict__ info) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *info = flags[0] ? 1 : 0;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < (size_t)n * n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % n), k = (int)(idx / n);
    if (i < k) L[(size_t)k * ld + i] = c128{0.0, 0.0};
  }
}

// info |= fewer than nev directions kept in [0, n)
__global__ void k_rank_check(int n, int nev, const int* __restrict__ drop, int* __restrict__ info) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int c = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) c += drop[i] ? 0 : 1;
  atomicAdd(&cnt, c);
  __syncthreads();
  if (threadIdx.x == 0 && *info == 0 && cnt < nev) *info = 1;
}

// L = X = I and no dropped directions on [0, n) (the collapsed, orthonormal basis)
__global__ void k_identity(int n, c128* __restrict__ L, c128* __restrict__ X, int ld, int* __restrict__ drop) {
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x) {
    const int i = idx % n, j = idx / n;
    const c128 v = c128{i == j ? 1.0 : 0.0, 0.0};
    L[(size_t)j * ld + i] = v;
    X[(size_t)j * ld + i] = v;
    if (j == 0) drop[i] = 0;
  }
}

// X[r, c] = 0 for r in [r0, r1), c in [0, c1)
__global__ void k_zero_block(int r0, int r1, int c1, c128* __restrict__ X, int ld) {
  const int nr = r1 - r0;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nr * c1; idx += gridDim.x * blockDim.x)
    X[(size_t)(idx / nr) * ld + r0 + idx % nr] = c128{0.0, 0.0};
}

// Dropped directions are decoupled from the transformed matrix and moved far
// above the spectrum, so they never enter the lowest nev eigenpairs.  The
// launch also clears gamma and, when the cooperative tridiagonalization
// follows, its barrier counter, failure flag and release flags (coop_count,
// coop_fail, coop_go; null otherwise).
__global__ void k_isolate(int n, c128* __restrict__ A, int ld, const int* __restrict__ drop,
                          const int* __restrict__ info, unsigned* __restrict__ coop_count,
                          unsigned* __restrict__ coop_fail, unsigned* __restrict__ coop_go,
                          double* __restrict__ gamma) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *gamma = 0.0;   // maximum taken by k_colnorms at the end of the solve
    if (coop_count != nullptr) {
      *coop_count = 0u;
      *coop_fail = 0u;
      for (int g = 0; g < kGoLines; ++g) coop_go[32 * g] = 0u;
    }
  }
  if (*info != 0) return;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x) {
    const int i = idx % n, j = idx / n;
    if (drop[i] || drop[j]) A[(size_t)j * ld + i] = c128{(i == j) ? 1e12 : 0.0, 0.0};
  }
}

// gamma = max_k || C[:, k] ||_2  (growth factor of the Ritz rotation): one
// wave per column (coalesced rows), then an atomic maximum over the bit
// patterns of the norms (non-negative doubles order as unsigned integers; the
// maximum does not depend on the order).  gamma is cleared by k_isolate
// earlier in the same solve; a NaN norm is left out, as fmax would.
__global__ void __launch_bounds__(256) k_colnorms(int n, int nev, const c128* __restrict__ C, int ldc,
                                                  double* __restrict__ gamma, const int* __restrict__ info) {
  if (*info != 0) return;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (k >= nev) return;
  double s = 0.0;
  for (int i = lane; i < n; i += 64) {
    const c128 v = C[(size_t)k * ldc + i];
    s += v.x * v.x + v.y * v.y;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) {
    const double v = sqrt(s);
    if (v == v)
      atomicMax(reinterpret_cast<unsigned long long*>(gamma), (unsigned long long)__double_as_longlong(v));
  }
}

// ---------------------------------------------------------------------------
// X = L^-H (upper triangular).  One workgroup per column j of Y = L^-1:
// forward substitution L y = e_j, row by row, then X[j, :] = conj(y)^T.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_trinv(int n, const c128* __restrict__ L, int ld,
                                               c128* __restrict__ X, int ldx, const int* __restrict__ info) {
  if (*info != 0) return;
  extern __shared__ __align__(16) char smem_raw[];
  c128* y = reinterpret_cast<c128*>(smem_raw);   // [n] right-hand side / solution
  const int j = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += blockDim.x) y[i] = c128{i == j ? 1.0 : 0.0, 0.0};
  __syncthreads();
  for (int i = j; i < n; ++i) {
    const c128 lii = L[(size_t)i * ld + i];
    const double inv = 1.0 / lii.x;
    const c128 yi = c128{y[i].x * inv, y[i].y * inv};
    __syncthreads();
    for (int k = i + 1 + threadIdx.x; k < n; k += blockDim.x) {
      const c128 u = cmul(L[(size_t)i * ld + k], yi);
      y[k] = c128{y[k].x - u.x, y[k].y - u.y};
    }
    if (threadIdx.x == 0) y[i] = yi;
    __syncthreads();
  }
  // X[j][i] = conj(Y[i][j]) for i >= j (row j of X), zero for i < j
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    X[(size_t)i * ldx + j] = (i >= j) ? cconj(y[i]) : c128{0.0, 0.0};
}

// ---------------------------------------------------------------------------
// Householder tridiagonalization of the full Hermitian A (n x n, col-major).
// For k = 0..n-2 the reflector H_k = I - tau_k v v^H (v_0 = 1) maps
// x = A[k+1:, k] to beta e_1 with beta real; A <- H^H A H on the trailing
// block as A - v w^H - w v^H with w = p - (tau/2)(p^H v) v, p = tau A v.
// v is stored in A[k+1:, k]; d, e get the real tridiagonal.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NTL) k_tridiag(int n, c128* __restrict__ A, int ld,
                                                 double* __restrict__ d, double* __restrict__ e,
                                                 c128* __restrict__ tau, const int* __restrict__ info) {
  if (*info != 0) return;
  extern __shared__ __align__(16) char smem_raw[];
  c128* v = reinterpret_cast<c128*>(smem_raw);   // [n]
  c128* w = v + n;                               // [n]
  c128* part = w + n;                            // [max(n, NTL)]
  __shared__ double red[NTL / 64];
  __shared__ c128 s_tau, s_scale;
  __shared__ double s_beta;
  const int bs = blockDim.x, tid = threadIdx.x;
  for (int k = 0; k < n - 1; ++k) {
    const int m = n - k - 1;
    c128* x = A + (size_t)k * ld + k + 1;
    double ss = 0.0;
    for (int i = 1 + tid; i < m; i += bs) ss += x[i].x * x[i].x + x[i].y * x[i].y;
    const double xn2 = block_sum(ss, red);
    if (tid == 0) {
      const c128 al = x[0];
      if (xn2 == 0.0 && al.y == 0.0) {
        s_tau = c128{0.0, 0.0};
        s_beta = al.x;
        s_scale = c128{0.0, 0.0};
      } else {
        const double nrm = sqrt(al.x * al.x + al.y * al.y + xn2);
        const double beta = al.x >= 0.0 ? -nrm : nrm;
        s_beta = beta;
        s_tau = c128{(beta - al.x) / beta, -al.y / beta};
        // scale = 1 / (alpha - beta)
        const c128 den = c128{al.x - beta, al.y};
        const double dd = den.x * den.x + den.y * den.y;
        s_scale = c128{den.x / dd, -den.y / dd};
      }
      d[k] = A[(size_t)k * ld + k].x;
      e[k] = s_beta;
      tau[k] = s_tau;
    }
    __syncthreads();
    const c128 t = s_tau, sc = s_scale;
    for (int i = tid; i < m; i += bs) {
      const c128 vi = (i == 0) ? c128{1.0, 0.0} : cmul(x[i], sc);
      v[i] = vi;
    }
    __syncthreads();
    for (int i = tid; i < m; i += bs) x[i] = v[i];   // keep v for the back-transform
    if (t.x == 0.0 && t.y == 0.0) {
      __syncthreads();
      continue;
    }
    c128* S = A + (size_t)(k + 1) * ld + k + 1;      // trailing block, m x m
    // p = tau * S v : S slices of rows
    const int ns = max(1, min(bs / m, 64));
    matvec_slices(m, ns, S, ld, v, part);
    __syncthreads();
    double hr = 0.0, hi = 0.0;
    for (int i = tid; i < m; i += bs) {
      c128 acc{0.0, 0.0};
      for (int s = 0; s < ns; ++s) { acc.x += part[s * m + i].x; acc.y += part[s * m + i].y; }
      const c128 pi = cmul(t, acc);
      w[i] = pi;
      const c128 pv = cmulc(pi, v[i]);   // conj(p_i) v_i
      hr += pv.x;
      hi += pv.y;
    }
    // alpha = -1/2 tau (p^H v)
    const c128 pv = block_sum_c(c128{hr, hi}, red);
    const c128 al = cmul(c128{-0.5 * t.x, -0.5 * t.y}, pv);
    for (int i = tid; i < m; i += bs) {
      const c128 u = cmul(al, v[i]);
      w[i] = c128{w[i].x + u.x, w[i].y + u.y};
    }
    __syncthreads();
#pragma unroll 4
    for (int idx = tid; idx < m * m; idx += bs) {
      const int i = idx % m, j = idx / m;
      const c128 a1 = cmulc(w[j], v[i]);   // v_i conj(w_j)
      const c128 a2 = cmulc(v[j], w[i]);   // w_i conj(v_j)
      c128* a = S + (size_t)j * ld + i;
      *a = c128{a->x - a1.x - a2.x, a->y - a1.y - a2.y};
    }
    __syncthreads();
  }
  if (tid == 0) d[n - 1] = A[(size_t)(n - 1) * ld + n - 1].x;
}


// ---------------------------------------------------------------------------
// Panel form of the tridiagonalization: one workgroup computes the reflectors
// of columns k0 .. k0+bb-1 from the trailing matrix as it stood before the
// panel, corrected by the panel's earlier (v_j, w_j):
//   column k  <- A[:, k] - sum_j (v_j conj(w_j[k]) + w_j conj(v_j[k]))
//   p         =  A_stale v - V (W^H v) - W (V^H v),  w = tau p - (tau/2)(..)v
// The trailing block A[k0+bb:, k0+bb:] then takes one rank-2bb update
// (two MFMA GEMMs).  PV / PW hold conj(v_j) / conj(w_j) row-major [n][bmax].
// ---------------------------------------------------------------------------
constexpr int PANEL = 32;
// below this size the unblocked single-workgroup reduction is faster
constexpr int kPanelMinN = 256;

__global__ void __launch_bounds__(NTL) k_tridiag_panel(int n, int k0, int bb, c128* __restrict__ A, int ld,
                                                       c128* __restrict__ PV, c128* __restrict__ PW,
                                                       double* __restrict__ d, double* __restrict__ e,
                                                       c128* __restrict__ tau, const int* __restrict__ info) {
  if (*info != 0) return;
  extern __shared__ __align__(16) char smem_raw[];
  c128* v = reinterpret_cast<c128*>(smem_raw);   // [n]  column, then reflector
  c128* p = v + n;                               // [n]  A v, then w
  c128* part = p + n;                            // [max(n, NTL)]
  __shared__ double red[NTL / 64];
  __shared__ c128 s_tau, s_scale, pvk[PANEL], pwk[PANEL], t1[PANEL], t2[PANEL];
  __shared__ c128 tpart[NTL / PANEL][2 * PANEL];
  __shared__ double s_beta;
  const int bs = blockDim.x, tid = threadIdx.x;
  for (int i = 0; i < bb; ++i) {
    const int k = k0 + i;
    // a. column k, updated by the earlier vectors of the panel
    if (tid < i) {
      pvk[tid] = PV[(size_t)k * PANEL + tid];
      pwk[tid] = PW[(size_t)k * PANEL + tid];
    }
    __syncthreads();
    for (int r = k + tid; r < n; r += bs) {
      c128 a = A[(size_t)k * ld + r];
      const c128* pvr = PV + (size_t)r * PANEL;
      const c128* pwr = PW + (size_t)r * PANEL;
      for (int j = 0; j < i; ++j) {
        // v_j[r] conj(w_j[k]) + w_j[r] conj(v_j[k]) = conj(pv_r) pw_k + conj(pw_r) pv_k
        const c128 u1 = cmulc(pvr[j], pwk[j]);
        const c128 u2 = cmulc(pwr[j], pvk[j]);
        a = c128{a.x - u1.x - u2.x, a.y - u1.y - u2.y};
      }
      A[(size_t)k * ld + r] = a;
      v[r] = a;
    }
    __syncthreads();
    // b. reflector for x = column k below the diagonal
    const int m = n - k - 1;
    double ss = 0.0;
    for (int r = k + 2 + tid; r < n; r += bs) ss += v[r].x * v[r].x + v[r].y * v[r].y;
    const double xn2 = block_sum(ss, red);
    if (tid == 0) {
      const c128 al = v[k + 1];
      if (xn2 == 0.0 && al.y == 0.0) {
        s_tau = c128{0.0, 0.0};
        s_beta = al.x;
        s_scale = c128{0.0, 0.0};
      } else {
        const double nrm = sqrt(al.x * al.x + al.y * al.y + xn2);
        const double beta = al.x >= 0.0 ? -nrm : nrm;
        s_beta = beta;
        s_tau = c128{(beta - al.x) / beta, -al.y / beta};
        const c128 den = c128{al.x - beta, al.y};
        const double dd = den.x * den.x + den.y * den.y;
        s_scale = c128{den.x / dd, -den.y / dd};
      }
      d[k] = v[k].x;
      e[k] = s_beta;
      tau[k] = s_tau;
    }
    __syncthreads();
    const c128 t = s_tau, sc = s_scale;
    for (int r = k + 1 + tid; r < n; r += bs) {
      const c128 vr = (r == k + 1) ? c128{1.0, 0.0} : cmul(v[r], sc);
      v[r] = vr;
      A[(size_t)k * ld + r] = vr;
      PV[(size_t)r * PANEL + i] = c128{vr.x, -vr.y};
    }
    __syncthreads();
    if (t.x == 0.0 && t.y == 0.0) {
      for (int r = k + 1 + tid; r < n; r += bs) PW[(size_t)r * PANEL + i] = c128{0.0, 0.0};
      __syncthreads();
      continue;
    }
    // c. p = A_stale v over the trailing rows/columns
    const c128* S = A + (size_t)(k + 1) * ld + k + 1;
    const c128* vv = v + k + 1;
    const int ns = max(1, min(bs / m, 64));
    matvec_slices(m, ns, S, ld, vv, part);
    //    t1 = W^H v, t2 = V^H v over rows k+1.. (thread = (row slice, j))
    if (i > 0) {
      const int j = tid % PANEL, sl = tid / PANEL, nsl = bs / PANEL;
      c128 a1{0.0, 0.0}, a2{0.0, 0.0};
      if (j < i) {
        for (int r = k + 1 + sl; r < n; r += nsl) {
          const c128 u1 = cmul(PW[(size_t)r * PANEL + j], v[r]);
          const c128 u2 = cmul(PV[(size_t)r * PANEL + j], v[r]);
          a1.x += u1.x; a1.y += u1.y;
          a2.x += u2.x; a2.y += u2.y;
        }
      }
      tpart[sl][j] = a1;
      tpart[sl][PANEL + j] = a2;
    }
    __syncthreads();
    if (i > 0 && tid < 2 * PANEL) {
      c128 acc{0.0, 0.0};
      for (int sl = 0; sl < bs / PANEL; ++sl) { acc.x += tpart[sl][tid].x; acc.y += tpart[sl][tid].y; }
      if (tid < PANEL) t1[tid] = acc; else t2[tid - PANEL] = acc;
    }
    __syncthreads();
    double hr = 0.0, hi = 0.0;
    for (int ii = tid; ii < m; ii += bs) {
      c128 acc{0.0, 0.0};
      for (int sl = 0; sl < ns; ++sl) { acc.x += part[sl * m + ii].x; acc.y += part[sl * m + ii].y; }
      const int r = k + 1 + ii;
      for (int j = 0; j < i; ++j) {
        // - v_j[r] t1_j - w_j[r] t2_j
        const c128 pv = PV[(size_t)r * PANEL + j], pw = PW[(size_t)r * PANEL + j];
        const c128 u1 = cmul(c128{pv.x, -pv.y}, t1[j]);
        const c128 u2 = cmul(c128{pw.x, -pw.y}, t2[j]);
        acc.x -= u1.x + u2.x;
        acc.y -= u1.y + u2.y;
      }
      const c128 wi = cmul(t, acc);
      p[r] = wi;
      const c128 pv = cmulc(wi, v[r]);   // conj(w_r) v_r
      hr += pv.x;
      hi += pv.y;
    }
    const c128 wv = block_sum_c(c128{hr, hi}, red);
    const c128 al = cmul(c128{-0.5 * t.x, -0.5 * t.y}, wv);
    for (int r = k + 1 + tid; r < n; r += bs) {
      const c128 u = cmul(al, v[r]);
      const c128 wr = c128{p[r].x + u.x, p[r].y + u.y};
      PW[(size_t)r * PANEL + i] = c128{wr.x, -wr.y};
    }
    __syncthreads();
  }
}

__global__ void k_tridiag_last(int n, const c128* __restrict__ A, int ld, double* __restrict__ d,
                               const int* __restrict__ info) {
  if (*info != 0) return;
  if (threadIdx.x == 0) d[n - 1] = A[(size_t)(n - 1) * ld + n - 1].x;
}

// ---------------------------------------------------------------------------
// Cooperative Householder tridiagonalization for 64 <= n <= 2048: P =
// ceil(n / CRT) workgroups (CRT = 8 or 16 rows each), workgroup q holding CRT
// rows of the Hermitian matrix B (row r = conj of column r of A) in
// registers.  Rows are dealt cyclically (row r to workgroup r mod P), so every
// workgroup keeps about (n - k) / P live rows at step k; thread t holds
// columns t mod CBW + CBW c (c < NC) of a 512 / CBW-th of its workgroup's
// rows (two waves per SIMD; CBW = 256 or 512 columns per pass).
//
// Step k (the reflector v_k, tau_k is known in every workgroup, and every
// workgroup holds y = B v_k for its rows):
//   1. p_r = tau_k y_r and the partial sum of conj(p_r) v_r are published,
//      and with them B[r][k+1] (updated through k-1) for the own rows r:
//      together they are row k+1, by symmetry (no single workgroup holds
//      the row and publishes it alone);
//   2. one barrier across the workgroups;
//   3. every workgroup reads all of p and forms w = p - 1/2 tau_k (p^H v) v,
//      applies the rank-2 update to its copy of row k+1 and derives the
//      reflector k+1 from it -- the same data and the same instruction
//      sequence in every workgroup, so all agree bit for bit;
//   4. each workgroup updates its rows, B -= v w^H + w v^H, and multiplies
//      them by v_{k+1} in the same pass.
// Reflectors, d, e and tau are stored as k_tridiag stores them.  Every wait
// is bounded: if the workgroups are not all resident, the kernel gives up,
// sets info = 2 and exits.
// ---------------------------------------------------------------------------
constexpr int CR = 16;      // rows per workgroup
constexpr int CT = 512;     // threads per workgroup (two waves per SIMD)
constexpr int CB = 256;     // columns covered by one pass of the threads
constexpr int kCoopMinN = 64, kCoopMaxN = 2048;
constexpr int kCoopMaxP = kCoopMaxN / 8;   // 8 rows per workgroup at the most workgroups
constexpr long kCoopSpin = 1l << 22;   // polls of a barrier before giving up
constexpr int kCoopSmallN = 2 * CB;     // up to here, 8 rows per workgroup

struct CoopBuf {
  c128* p;         // [2][kCoopMaxN]   p_r of every row, by step parity
  c128* s;         // [2][kCoopMaxP]   partial sums conj(p)^T v of each workgroup
  c128* row;       // [2][kCoopMaxN]   row k+1 before the update of step k
  unsigned* count; // barrier arrivals (zeroed before each launch)
  unsigned* fail;  // set when a barrier timed out
  unsigned* go;    // [kGoLines * 32]  the number of the last step every workgroup has reached
};

// The exchanged values are written with agent-scope atomic 64-bit stores,
// which bypass caches that are not coherent across the XCDs, and each
// workgroup's release fence before its barrier arrival makes them visible.
// Readers load them with plain loads after the barrier: wave 0's agent-scope
// acquire fence (which invalidates the non-coherent cache lines) followed by
// the workgroup barrier orders every wave's loads after the publications.
__device__ __forceinline__ void xstore(c128* p, c128 v) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  __hip_atomic_store(q, (unsigned long long)__double_as_longlong(v.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, (unsigned long long)__double_as_longlong(v.y), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Cross-lane moves of a double through DPP (no LDS traffic).  The four row
// permutations used pair lane i with i^1, i^2 (quad permutes), 7-i within
// each half row and 15-i within each row: each is an involution that flips
// bit 0, 1, 2 and 3 of the lane index respectively.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
template <int LEVEL>
__device__ __forceinline__ double row_partner(double v) {
  if constexpr (LEVEL == 0) return dpp_f64<kDppXor1>(v);
  else if constexpr (LEVEL == 1) return dpp_f64<kDppXor2>(v);
  else if constexpr (LEVEL == 2) return dpp_f64<kDppHalfMirror>(v);
  else return dpp_f64<kDppMirror>(v);
}

// sum of one double over the 64 lanes; every lane ends with the same bits
// (each pairwise sum is formed from the same two operands, and the four row
// sums are combined in one fixed order)
__device__ __forceinline__ double wave_sum(double v) {
  v += row_partner<0>(v);
  v += row_partner<1>(v);
  v += row_partner<2>(v);
  v += row_partner<3>(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// sum over the 64 lanes of the V values in v[] (V a power of two <= 16).  The
// row pairings are taken in the order 15-i, 7-i, i^2, i^1 (each leaves the
// lane bits the earlier ones tested unchanged); at the first log2(V) of them
// a lane keeps half of its values (the upper half when the tested bit --
// bit 3, 2, 1, 0 in turn -- is set) and adds its partner's copy of that
// half, at the others it adds the partner's value; then the four rows are
// summed.  Afterwards every lane l < 16 with msum_writer<V>(l) holds in v[0]
// the total of value msum_slot<V>(l).
template <int CNT, int STEP, int V>
__device__ __forceinline__ void msum_level(double (&v)[V], int lane) {
  if constexpr (STEP < 4) {
    constexpr int LEVEL = 3 - STEP;   // pairing: mirror, half mirror, xor 2, xor 1
    const bool up = (lane >> LEVEL) & 1;
    if constexpr (CNT > 1) {
      constexpr int half = CNT / 2;
#pragma unroll
      for (int q = 0; q < half; ++q) {
        const double mine = up ? v[half + q] : v[q];
        const double other = up ? v[q] : v[half + q];
        v[q] = mine + row_partner<LEVEL>(other);
      }
      msum_level<half, STEP + 1, V>(v, lane);
    } else {
      v[0] += row_partner<LEVEL>(v[0]);
      msum_level<1, STEP + 1, V>(v, lane);
    }
  }
}
template <int V>
__device__ __forceinline__ void wave_multi_sum(double (&v)[V]) {
  static_assert(V >= 1 && V <= 16 && (V & (V - 1)) == 0, "V a power of two <= 16");
  msum_level<V, 0, V>(v, threadIdx.x & 63);
  v[0] += __shfl_xor(v[0], 16, 64);
  v[0] += __shfl_xor(v[0], 32, 64);
}
template <int V>
constexpr int ilog2c() { return V <= 1 ? 0 : 1 + ilog2c<V / 2>(); }
template <int V>
__device__ __forceinline__ bool msum_writer(int l) {
  return l < 16 && (l & ((1 << (4 - ilog2c<V>())) - 1)) == 0;
}
template <int V>
__device__ __forceinline__ int msum_slot(int l) {
  int idx = 0, cnt = V, t = 0;
  while (cnt > 1) { cnt >>= 1; if ((l >> (3 - t)) & 1) idx += cnt; ++t; }
  return idx;
}

// Householder vector of x = (alpha, x_1, ...) given alpha and sum |x_i|^2 (i >= 1):
// tau, beta and the scale 1 / (alpha - beta) of x_1.. (the same rule as k_tridiag)
struct Refl { c128 tau, scale; double beta; };
__device__ __forceinline__ Refl householder(c128 al, double xn2) {
  Refl r;
  if (xn2 == 0.0 && al.y == 0.0) {
    r.tau = c128{0.0, 0.0}; r.beta = al.x; r.scale = c128{0.0, 0.0};
  } else {
    const double nrm = sqrt(al.x * al.x + al.y * al.y + xn2);
    const double beta = al.x >= 0.0 ? -nrm : nrm;
    r.beta = beta;
    r.tau = c128{(beta - al.x) / beta, -al.y / beta};
    const c128 den = c128{al.x - beta, al.y};
    const double dd = den.x * den.x + den.y * den.y;
    r.scale = c128{den.x / dd, -den.y / dd};
  }
  return r;
}

template <int NC, int CRT, int CBW = CB>
__global__ void __launch_bounds__(CT) k_tridiag_coop(int n, c128* __restrict__ A, int ld, double* __restrict__ d,
                                                     double* __restrict__ e, c128* __restrict__ tau,
                                                     int* __restrict__ info, CoopBuf cb) {
  constexpr int NW = CT / 64;             // waves
  constexpr int NH = CT / CBW;            // row groups (threads t and t + CBW share columns)
  constexpr int RH = CRT / NH;            // rows per thread
  constexpr int WH = CBW / 64;            // waves per row group
  if (*info != 0) return;
  __shared__ c128 s_colk[CRT];            // B[r][k+1] of the own rows r (row k+1 by symmetry)
  __shared__ double s_red[NW][2 * RH];    // per-wave row sums of B v (re, then im)
  __shared__ c128 s_rv[2][CRT], s_rw[CRT];  // v_k (by step parity) and w on the own rows
  __shared__ double s_xn2[NW];
  __shared__ c128 s_alx;
  __shared__ int s_fail;

  const int P = gridDim.x, q = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int half = tid / CBW;
  // own rows: row(i) = q + P i (cyclic, so that every workgroup keeps about
  // the same number of live rows as the reduction proceeds)
  auto row_of = [&](int i) { return q + P * i; };
  // local index of row r if it is an own row, else -1
  auto local_of = [&](int r) { return (r >= q && (r - q) % P == 0 && (r - q) / P < CRT) ? (r - q) / P : -1; };
  int jc[NC];
  bool ok[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) { jc[c] = (tid % CBW) + CBW * c; ok[c] = jc[c] < n; }

  // rows of B: a[c][i] = B[row(half RH + i)][j_c] = conj(A[row * ld + j_c])
  c128 a[NC][RH];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int i = 0; i < RH; ++i) {
      const int R = row_of(half * RH + i);
      a[c][i] = (ok[c] && R < n) ? cconj(A[(size_t)R * ld + jc[c]]) : c128{0.0, 0.0};
      if (jc[c] == 1 && R < n) s_colk[half * RH + i] = a[c][i];   // column 1: row 1, published at step 0
    }
  if (tid == 0) s_fail = 0;
  // own rows past the end of the matrix are never written: start from zeros
  if (tid < CRT) { s_rv[0][tid] = s_rv[1][tid] = s_rw[tid] = c128{0.0, 0.0}; }
  __syncthreads();

  // own-row values of a column vector to LDS (one copy: the first half writes)
  auto put_own = [&](c128* dst, const c128 (&val)[NC]) {
    if (half != 0) return;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int li = local_of(jc[c]);
      if (li >= 0 && ok[c]) dst[li] = val[c];
    }
  };
  // y = B v on the own rows: per-thread partial sums, then per-wave totals to s_red
  auto rows_times = [&](const c128 (&acc)[RH]) {
    double vr[RH], vi[RH];
#pragma unroll
    for (int i = 0; i < RH; ++i) { vr[i] = acc[i].x; vi[i] = acc[i].y; }
    wave_multi_sum<RH>(vr);
    wave_multi_sum<RH>(vi);
    if (msum_writer<RH>(lane)) {
      const int sl = msum_slot<RH>(lane);
      s_red[wid][sl] = vr[0];
      s_red[wid][RH + sl] = vi[0];
    }
  };

  // reflector 0 from column 0 of B below the diagonal: x_j = conj(B[0][j]) = A[0 * ld + j]
  c128 vk[NC], tk;
  double beta0;
  {
    c128 x[NC];
    double xx = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      x[c] = (ok[c] && jc[c] >= 1) ? A[jc[c]] : c128{0.0, 0.0};
      if (half == 0 && ok[c] && jc[c] >= 2) xx += x[c].x * x[c].x + x[c].y * x[c].y;
      if (half == 0 && jc[c] == 1) s_alx = x[c];
    }
    const double r = wave_sum(xx);
    if (lane == 0) s_xn2[wid] = r;
    __syncthreads();
    const Refl h = householder(s_alx, wave_sum(lane < NW ? s_xn2[lane] : 0.0));
#pragma unroll
    for (int c = 0; c < NC; ++c)
      vk[c] = (jc[c] == 1) ? c128{1.0, 0.0} : (jc[c] > 1 && ok[c] ? cmul(x[c], h.scale) : c128{0.0, 0.0});
    tk = h.tau;
    beta0 = h.beta;
    put_own(s_rv[0], vk);
  }
  {
    c128 acc[RH];
#pragma unroll
    for (int i = 0; i < RH; ++i) {
      acc[i] = c128{0.0, 0.0};
      const int R = row_of(half * RH + i);
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (R >= 1 && R < n && jc[c] >= 1 && ok[c]) acc[i] = acc[i] + cmul(a[c][i], vk[c]);
    }
    rows_times(acc);
  }
  __syncthreads();

  for (int k = 0; k <= n - 2; ++k) {
    const int par = k & 1;
    // 1. wave 0: finish y on the own rows, publish p_r = tau_k y_r, the
    //    partial sum of conj(p_r) v_r, and the own entries of row k+1; then the barrier
    if (wid == 0) {
      c128 p{0.0, 0.0};
      const int R = (lane < CRT) ? row_of(lane) : n;
      if (lane < CRT && R >= k + 1 && R < n) {
        const int hh = lane / RH, ii = lane % RH;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int w = hh * WH; w < hh * WH + WH; ++w) { re += s_red[w][ii]; im += s_red[w][RH + ii]; }
        p = cmul(tk, c128{re, im});
      }
      // rows outside [k+1, n) contribute nothing (and their v entries are not read)
      const c128 t = (lane < CRT && R >= k + 1 && R < n) ? cmulc(p, s_rv[par][lane]) : c128{0.0, 0.0};
      const double sre = wave_sum(t.x), sim = wave_sum(t.y);
      if (lane < CRT && R < n) xstore(&cb.p[par * kCoopMaxN + R], p);
      if (lane == 0) xstore(&cb.s[par * kCoopMaxP + q], c128{sre, sim});
      // row k+1 = conj(column k+1): every workgroup publishes its own entries
      if (lane < CRT && R >= k + 1 && R < n) xstore(&cb.row[par * kCoopMaxN + R], cconj(s_colk[lane]));
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (lane == 0) {
        const unsigned old = __hip_atomic_fetch_add(cb.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // 2. barrier: all P workgroups have published step k.  Beyond
        // kGoMinP workgroups the last to arrive (it sees the count before its
        // own arrival one short of the target) raises the step's release
        // flags, and the others poll one of them each: no address then has
        // more than ceil(P / kGoLines) pollers, which cut the time from the
        // last arrival to the last workgroup seeing it from 2.1 to 1.35 us at
        // 48 workgroups (5.4 to 3.0 us at 256).  The last arrival's fence
        // synchronizes with every arrival's release (the counter's updates
        // form one release sequence) and releases to the flags' readers.
        // Up to kGoMinP workgroups poll the counter itself (the extra hop
        // costs more than the contention it saves there).
        const unsigned target = (unsigned)P * (unsigned)(k + 1);
        const bool flags = P > kGoMinP;
        if (flags && old + 1u == target) {
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
          for (int g = 0; g < kGoLines; ++g)
            __hip_atomic_store(cb.go + 32 * g, (unsigned)(k + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        unsigned* const poll = flags ? cb.go + 32 * (q % kGoLines) : cb.count;
        const unsigned want = flags ? (unsigned)(k + 1) : target;
        // one load per poll; the failure flag of the other workgroups is
        // looked at every 256 polls
        long spins = 0;
        for (;;) {
          if (__hip_atomic_load(poll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want) break;
          if ((++spins & 255) == 0 &&
              (__hip_atomic_load(cb.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spins > kCoopSpin)) {
            __hip_atomic_store(cb.fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_fail = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (s_fail) {
      if (q == 0 && tid == 0) *info = 2;
      return;
    }
    // 3. every wave: p^H v, w, row k+1 after the update, and the partial norm
    //    of the next reflector's vector
    c128 pj[NC], rowj[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const bool live = ok[c] && jc[c] >= k + 1;
      pj[c] = live ? cb.p[par * kCoopMaxN + jc[c]] : c128{0.0, 0.0};
      rowj[c] = live ? cb.row[par * kCoopMaxN + jc[c]] : c128{0.0, 0.0};
    }
    const c128 pk1 = cb.p[par * kCoopMaxN + k + 1];
    c128 sl{0.0, 0.0};   // partial sums of workgroups lane, lane + 64, ... (fixed order)
    for (int w = lane; w < P; w += 64) {
      const c128 t = cb.s[par * kCoopMaxP + w];
      sl.x += t.x;
      sl.y += t.y;
    }
    const c128 psum{wave_sum(sl.x), wave_sum(sl.y)};
    const c128 al = cmul(c128{-0.5 * tk.x, -0.5 * tk.y}, psum);   // -1/2 tau (p^H v)
    const c128 wk1 = pk1 + cmul(al, c128{1.0, 0.0});              // v_k[k+1] = 1
    c128 wj[NC], x[NC];
    double xx = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const bool live = ok[c] && jc[c] >= k + 1;
      wj[c] = live ? pj[c] + cmul(al, vk[c]) : c128{0.0, 0.0};
      // row'_j = row_j - conj(w_j) - w_{k+1} conj(v_j)
      c128 rj{0.0, 0.0};
      if (live) {
        const c128 t = cmulc(vk[c], wk1);
        rj = c128{rowj[c].x - wj[c].x - t.x, rowj[c].y + wj[c].y - t.y};
      }
      if (q == 0 && half == 0 && jc[c] == k + 1) d[k + 1] = rj.x;
      // x_j = conj(row'_j), j >= k+2; alpha = x_{k+2}
      x[c] = (jc[c] >= k + 2) ? cconj(rj) : c128{0.0, 0.0};
      if (half == 0 && ok[c] && jc[c] >= k + 3) xx += x[c].x * x[c].x + x[c].y * x[c].y;
      if (half == 0 && jc[c] == k + 2) s_alx = x[c];
    }
    if (q == 0 && k == 0 && half == 0) {
      // reflector 0 is stored only now: every workgroup has read column 0
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (ok[c] && jc[c] >= 1) A[jc[c]] = vk[c];
      if (tid == 0) { d[0] = A[0].x; e[0] = beta0; tau[0] = tk; }
    }
    put_own(s_rw, wj);
    if (k + 1 > n - 2) break;
    {
      const double r = wave_sum(xx);
      if (lane == 0) s_xn2[wid] = r;
    }
    __syncthreads();
    // 4. every wave: reflector k+1 (identical everywhere)
    const Refl h = householder(s_alx, wave_sum(lane < NW ? s_xn2[lane] : 0.0));
    c128 vk1[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      vk1[c] = (jc[c] == k + 2) ? c128{1.0, 0.0} : (jc[c] > k + 2 && ok[c] ? cmul(x[c], h.scale) : c128{0.0, 0.0});
      if (q == 0 && half == 0 && ok[c] && jc[c] >= k + 2) A[(size_t)(k + 1) * ld + jc[c]] = vk1[c];
      if (q == 0 && half == 0 && jc[c] == k + 2) { e[k + 1] = h.beta; tau[k + 1] = h.tau; }
    }
    // v_{k+1} on the own rows is read by the update of the next step only
    // (three barriers later), and this step's update reads the other parity
    // buffer: no barrier here
    put_own(s_rv[par ^ 1], vk1);
    // 5. B -= v w^H + w v^H on rows and columns >= k+2, and y = B v_{k+1};
    //    the threads of column k+2 keep its entries for the next publication
    {
      c128 acc[RH];
#pragma unroll
      for (int i = 0; i < RH; ++i) acc[i] = c128{0.0, 0.0};
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        // columns of this wave: [64 (wid % WH) + CBW c, + 64)
        const int cbase = 64 * (wid % WH) + CBW * c;
        if (cbase + 63 < k + 2 || cbase >= n) continue;
        if (!(ok[c] && jc[c] >= k + 2)) continue;
        const c128 cw = cconj(wj[c]), cv = cconj(vk[c]);
#pragma unroll
        for (int i = 0; i < RH; ++i) {
          const int li = half * RH + i;
          const int R = row_of(li);
          if (R >= k + 2 && R < n) {
            const c128 u1 = cmul(s_rv[par][li], cw), u2 = cmul(s_rw[li], cv);
            a[c][i] = c128{a[c][i].x - u1.x - u2.x, a[c][i].y - u1.y - u2.y};
            acc[i] = acc[i] + cmul(a[c][i], vk1[c]);
            if (jc[c] == k + 2) s_colk[li] = a[c][i];
          }
        }
      }
      rows_times(acc);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) vk[c] = vk1[c];
    tk = h.tau;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Lowest nev eigenvalues of the real symmetric tridiagonal (d, e): one
// workgroup of one or four waves per eigenvalue, 128 or 512 shifts per round
// (Sturm counts), interval narrowed to the two shifts around the k-th
// eigenvalue.
// ---------------------------------------------------------------------------
// 1/q to a few units in the last place: the hardware reciprocal refined by
// one Newton step (a shorter dependent chain than an IEEE division; a Sturm
// count only needs the signs of the pivots)
__device__ __forceinline__ double fast_rcp(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

// Sturm counts (number of eigenvalues below x) of the tridiagonal (d, e2 =
// e^2) at CH shifts at once: the CH recurrences are independent, so their
// latencies overlap
template <int CH>
__device__ __forceinline__ void sturm_counts(int n, const double* d, const double* e2, const double (&x)[CH],
                                             double pivmin, int (&cnt)[CH]) {
  double q[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    q[c] = d[0] - x[c];
    cnt[c] = q[c] < 0.0 ? 1 : 0;
  }
#pragma unroll 4
  for (int i = 1; i < n; ++i) {
    const double di = d[i], ei = e2[i - 1];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const double qq = (fabs(q[c]) < pivmin) ? -pivmin : q[c];
      q[c] = di - x[c] - ei * fast_rcp(qq);
      cnt[c] += q[c] < 0.0 ? 1 : 0;
    }
  }
}

// One workgroup per wanted eigenvalue k (of 64 or 256 threads: one or four
// waves, one per SIMD): each round evaluates the Sturm count at NW x 64 x CH
// equally spaced shifts and keeps the interval between the two shifts that
// bracket the k-th eigenvalue.
constexpr int kBisectChains = 2;
__global__ void __launch_bounds__(256) k_bisect(int n, const double* __restrict__ dg,
                                                const double* __restrict__ eg, int nev,
                                                double* __restrict__ w, const int* __restrict__ info) {
  if (*info != 0) return;
  constexpr int CH = kBisectChains, NS = 64 * CH;
  extern __shared__ __align__(16) char smem_raw[];
  double* d = reinterpret_cast<double*>(smem_raw);
  double* e2 = d + n;
  __shared__ double s_lo, s_hi, s_piv;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    d[i] = dg[i];
    if (i < n - 1) e2[i] = eg[i] * eg[i];
  }
  __syncthreads();
  // Gershgorin interval of T (the first wave, one row per lane at a time)
  if (threadIdx.x < 64) {
    double lo = 1e300, hi = -1e300, emax = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) {
      const double r = (i > 0 ? sqrt(e2[i - 1]) : 0.0) + (i < n - 1 ? sqrt(e2[i]) : 0.0);
      lo = fmin(lo, d[i] - r);
      hi = fmax(hi, d[i] + r);
      if (i < n - 1) emax = fmax(emax, e2[i]);
    }
    for (int o = 32; o > 0; o >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, o, 64));
      hi = fmax(hi, __shfl_xor(hi, o, 64));
      emax = fmax(emax, __shfl_xor(emax, o, 64));
    }
    if (threadIdx.x == 0) {
      const double nrm = fmax(fabs(lo), fabs(hi));
      const double pad = 4.0 * DBL_EPSILON * nrm * n + 1e-300;
      s_lo = lo - pad;
      s_hi = hi + pad;
      s_piv = DBL_MIN * fmax(1.0, emax);
    }
  }
  __syncthreads();
  // the workgroup's NW waves share eigenvalue k = blockIdx.x: each round
  // evaluates NW x 64 x CH equally spaced shifts (wave v the v-th block of
  // them), one wave per SIMD, and keeps the interval between the two shifts
  // around the k-th eigenvalue
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, NW = blockDim.x >> 6;
  const int k = blockIdx.x;
  __shared__ int s_first[16];
  const int NT = NS * NW;   // shifts per round
  double lo = s_lo, hi = s_hi;
  const double pivmin = s_piv;
  for (int round = 0; round < 64; ++round) {
    // the same decision in every thread (lo and hi are uniform)
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    const double step = (hi - lo) / (double)(NT + 1);
    double x[CH];
    int c[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) x[j] = lo + step * (NS * wv + CH * lane + j + 1);
    sturm_counts<CH>(n, d, e2, x, pivmin, c);
    // first shift (in increasing order) with more than k eigenvalues below it
    int jf = CH;
#pragma unroll
    for (int j = CH - 1; j >= 0; --j)
      if (c[j] > k) jf = j;
    const unsigned long long mask = __ballot(jf < CH);
    const int f = mask != 0ull ? __ffsll((long long)mask) - 1 : 0;
    const int jsel = __shfl(jf, f, 64);   // every lane takes part
    if (lane == 0) s_first[wv] = mask != 0ull ? NS * wv + CH * f + jsel : NT;   // NT: none in this block
    __syncthreads();
    int s0 = NT;
    for (int v = 0; v < NW; ++v) s0 = min(s0, s_first[v]);
    __syncthreads();   // s_first is rewritten next round
    if (s0 == NT) {
      lo = lo + step * NT;
    } else {
      const double xf = lo + step * (s0 + 1);
      const double xp = (s0 > 0) ? lo + step * s0 : lo;
      hi = xf;
      lo = xp;
    }
  }
  if (threadIdx.x == 0) w[k] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// Inverse iteration on T for the eigenvalues w[0..nev): thread i handles the
// cluster that starts at i (eigenvalues within 1e-7 of the wanted spectrum's
// scale of their neighbour),
// solving (T - w I) x = b by Gaussian elimination with partial pivoting,
// three iterations, orthogonalized against the earlier cluster members.
// Z is real [nev][ldz].  The per-thread factors (pivots kept as reciprocals)
// and iterate (5 n doubles and n pivot flags) live in a Work view: LDS for up to TPW threads per
// workgroup when they fit, else the global scratch (element r of thread t at
// [r * S + t], so that neighbouring threads touch neighbouring addresses).
// ---------------------------------------------------------------------------
constexpr int IC = 8;   // recurrence steps whose operands are loaded ahead

struct InvitView {
  double *D, *DL, *DU, *DU2, *X, *Y;
  unsigned char* PV;
  size_t S;   // stride between consecutive elements of one thread (SC when SC > 0)
};

// SC > 0: compile-time stride (the compiler can then overlap the loads of one
// row with the stores of the previous one)
template <int SC>
__device__ void invit_cluster(int n, const double* __restrict__ d, const double* __restrict__ e, int nev,
                              const double* __restrict__ w, double* __restrict__ Z, int ldz, int i0,
                              InvitView v) {
  // scale of the wanted part of the spectrum (dropped basis directions sit
  // far above it and must not widen the clusters)
  const double tn = fmax(fmax(fabs(w[0]), fabs(w[nev - 1])), fmax(w[nev - 1] - w[0], 1e-300));
  const double ctol = 1e-7 * tn;
  if (i0 > 0 && w[i0] - w[i0 - 1] <= ctol) return;   // not a cluster leader
  int i1 = i0 + 1;
  while (i1 < nev && w[i1] - w[i1 - 1] <= ctol) ++i1;
  const double tiny = DBL_EPSILON * tn;
  const size_t S = SC > 0 ? (size_t)SC : v.S;
  double* __restrict__ D = v.D;      // reciprocal pivots
  double* __restrict__ DL = v.DL;
  double* __restrict__ DU = v.DU;
  double* __restrict__ DU2 = v.DU2;
  double* __restrict__ X = v.X;
  double* __restrict__ Y = v.Y;
  unsigned char* __restrict__ PV = v.PV;
  for (int i = i0; i < i1; ++i) {
    const double lam = w[i];
    // factor T - lam I with partial pivoting; the running pivot stays in a
    // register.  The tridiagonal is read IC steps ahead (independent of the
    // recurrence), and the multipliers and reciprocal pivots use the hardware
    // reciprocal refined by one Newton step instead of an IEEE division.
    double dcur = d[0] - lam;
    double du_next = (n > 1) ? e[0] : 0.0;   // DU[r] before row r's update
    auto fstep = [&](int r, double er, double dnext, double du_after) {
      double dr, dlr, dur, du2r, dn, dun;
      unsigned char piv;
      if (fabs(dcur) >= fabs(er)) {
        const double dd = (dcur == 0.0) ? tiny : dcur;
        const double f = er * fast_rcp(dd);
        dr = dd; dlr = f; dur = du_next; du2r = 0.0; dn = dnext - f * du_next; dun = du_after; piv = 0;
      } else {
        const double f = dcur * fast_rcp(er);
        dr = er; dlr = f; dur = dnext; dn = du_next - f * dnext;
        du2r = du_after; dun = -f * du_after; piv = 1;
      }
      D[r * S] = fast_rcp((fabs(dr) < tiny) ? ((dr >= 0.0) ? tiny : -tiny) : dr);
      DL[r * S] = dlr; DU[r * S] = dur; DU2[r * S] = du2r;
      PV[r * S] = piv;
      dcur = dn;
      du_next = dun;
    };
    int r0 = 0;
    for (; r0 + IC < n - 1; r0 += IC) {   // full chunks: rows r0 .. r0+IC-1, all < n-2
      double er_[IC], dn_[IC], ea_[IC];
#pragma unroll
      for (int u = 0; u < IC; ++u) {
        er_[u] = e[r0 + u];
        dn_[u] = d[r0 + u + 1];
        ea_[u] = e[r0 + u + 1];
      }
#pragma unroll
      for (int u = 0; u < IC; ++u) fstep(r0 + u, er_[u], dn_[u] - lam, ea_[u]);
    }
    for (int r = r0; r < n - 1; ++r) fstep(r, e[r], d[r + 1] - lam, (r < n - 2) ? e[r + 1] : 0.0);
    D[(n - 1) * S] = fast_rcp((fabs(dcur) < tiny) ? ((dcur >= 0.0) ? tiny : -tiny) : dcur);
    // generic start vector: an integer hash of (r, i) mapped to [0.5, 1.5)
    for (int r = 0; r < n; ++r) {
      unsigned h = (unsigned)r * 2654435761u ^ ((unsigned)i * 2246822519u + 0x9e3779b9u);
      h ^= h >> 15;
      h *= 2246822519u;
      h ^= h >> 13;
      X[r * S] = 0.5 + (double)(h & 0xffffu) * (1.0 / 65536.0);
    }
    for (int it = 0; it < 3; ++it) {
      // forward substitution with the row interchanges: X -> Y (operands of
      // IC steps loaded ahead of the recurrence)
      double xr = X[0];
      auto sstep = [&](int r, double xn, double dl, unsigned char pv) {
        if (pv) {
          Y[r * S] = xn;
          xr = xr - dl * xn;
        } else {
          Y[r * S] = xr;
          xr = xn - dl * xr;
        }
      };
      int q0 = 0;
      for (; q0 + IC <= n - 1; q0 += IC) {
        double xn_[IC], dl_[IC];
        unsigned char pv_[IC];
#pragma unroll
        for (int u = 0; u < IC; ++u) {
          xn_[u] = X[(q0 + u + 1) * S];
          dl_[u] = DL[(q0 + u) * S];
          pv_[u] = PV[(q0 + u) * S];
        }
#pragma unroll
        for (int u = 0; u < IC; ++u) sstep(q0 + u, xn_[u], dl_[u], pv_[u]);
      }
      for (int r = q0; r < n - 1; ++r) sstep(r, X[(r + 1) * S], DL[r * S], PV[r * S]);
      // back substitution with the upper factor: Y -> X
      double x2 = 0.0, x1 = xr * D[(n - 1) * S];
      X[(n - 1) * S] = x1;
      auto bstep = [&](int r, double yv, double du, double du2, double dd) {
        const double xv = (yv - du * x1 - du2 * x2) * dd;
        X[r * S] = xv;
        x2 = x1;
        x1 = xv;
      };
      int p0 = n - 2;
      for (; p0 - IC + 1 >= 0; p0 -= IC) {
        double y_[IC], du_[IC], du2_[IC], dd_[IC];
#pragma unroll
        for (int u = 0; u < IC; ++u) {
          const int r = p0 - u;
          y_[u] = Y[r * S];
          du_[u] = DU[r * S];
          du2_[u] = DU2[r * S];
          dd_[u] = D[r * S];
        }
#pragma unroll
        for (int u = 0; u < IC; ++u) bstep(p0 - u, y_[u], du_[u], du2_[u], dd_[u]);
      }
      for (int r = p0; r >= 0; --r) bstep(r, Y[r * S], DU[r * S], DU2[r * S], D[r * S]);
      for (int j = i0; j < i; ++j) {
        const double* zj = Z + (size_t)j * ldz;
        double dot = 0.0;
        for (int r = 0; r < n; ++r) dot += zj[r] * X[r * S];
        for (int r = 0; r < n; ++r) X[r * S] -= dot * zj[r];
      }
      double nrm = 0.0;
#pragma unroll 4
      for (int r = 0; r < n; ++r) nrm += X[r * S] * X[r * S];
      const double inv = 1.0 / sqrt(nrm);
#pragma unroll 4
      for (int r = 0; r < n; ++r) X[r * S] *= inv;
    }
    double* z = Z + (size_t)i * ldz;
    for (int r = 0; r < n; ++r) z[r] = X[r * S];
  }
}

// scratch in global memory: 6 n doubles + n bytes per thread
__global__ void __launch_bounds__(64) k_invit(int n, const double* __restrict__ d,
                                              const double* __restrict__ e, int nev,
                                              const double* __restrict__ w, double* __restrict__ Z,
                                              int ldz, double* __restrict__ scratch,
                                              const int* __restrict__ info) {
  if (*info != 0) return;
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 >= nev) return;
  const size_t S = (size_t)gridDim.x * blockDim.x;
  InvitView v;
  v.S = S;
  v.D = scratch + i0;
  v.DL = v.D + (size_t)n * S;
  v.DU = v.DL + (size_t)n * S;
  v.DU2 = v.DU + (size_t)n * S;
  v.X = v.DU2 + (size_t)n * S;
  v.Y = v.X + (size_t)n * S;
  v.PV = reinterpret_cast<unsigned char*>(scratch + 6 * (size_t)n * S) + i0;
  invit_cluster<0>(n, d, e, nev, w, Z, ldz, i0, v);
}

// scratch in LDS: the tridiagonal (16 n bytes) and TPW threads per workgroup,
// 49 n bytes each
constexpr int kInvitLdsBytes = 120 * 1024;
template <int TPW>
__global__ void __launch_bounds__(64) k_invit_lds(int n, const double* __restrict__ d,
                                                  const double* __restrict__ e, int nev,
                                                  const double* __restrict__ w, double* __restrict__ Z,
                                                  int ldz, const int* __restrict__ info) {
  if (*info != 0) return;
  extern __shared__ __align__(16) char smem_raw[];
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * TPW + t;
  // the tridiagonal, read once per step of every recurrence, is staged in LDS
  double* sd = reinterpret_cast<double*>(smem_raw);
  double* se = sd + n;
  for (int i = t; i < n; i += blockDim.x) {
    sd[i] = d[i];
    se[i] = (i < n - 1) ? e[i] : 0.0;
  }
  __syncthreads();
  if (t >= TPW || i0 >= nev) return;
  double* base = se + n;
  InvitView v;
  v.S = TPW;
  v.D = base + t;
  v.DL = v.D + (size_t)n * TPW;
  v.DU = v.DL + (size_t)n * TPW;
  v.DU2 = v.DU + (size_t)n * TPW;
  v.X = v.DU2 + (size_t)n * TPW;
  v.Y = v.X + (size_t)n * TPW;
  v.PV = reinterpret_cast<unsigned char*>(base + 6 * (size_t)n * TPW) + t;
  invit_cluster<TPW>(n, sd, se, nev, w, Z, ldz, i0, v);
}

// ---------------------------------------------------------------------------
// Y = Q Z, Q = H_0 H_1 ... H_{n-2}: Y <- H_k Y = Y - tau_k v_k (v_k^H Y) for
// k = n-2 down to 0.  One wave per column of Y, held in registers (row
// r = lane + 64 t in slot t); the dot product is a wave reduction, so no
// workgroup barrier is needed.
// ---------------------------------------------------------------------------
template <int NPL>
__global__ void __launch_bounds__(256) k_backtr(int n, const c128* __restrict__ A, int lda,
                                                const c128* __restrict__ tau, const double* __restrict__ Z,
                                                int ldz, int nev, c128* __restrict__ Y, int ldy,
                                                const int* __restrict__ info) {
  if (*info != 0) return;
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (col >= nev) return;
  c128 y[NPL];
#pragma unroll
  for (int t = 0; t < NPL; ++t) {
    const int r = lane + 64 * t;
    y[t] = c128{r < n ? Z[(size_t)col * ldz + r] : 0.0, 0.0};
  }
  // the reflector of the next step is loaded while the current one is applied
  auto load_v = [&](int k, c128 (&vv)[NPL]) {
    const c128* v = A + (size_t)k * lda;   // v_k at rows k+1 .. n-1
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int r = lane + 64 * t;
      vv[t] = (r > k && r < n) ? v[r] : c128{0.0, 0.0};
    }
  };
  c128 vn[NPL];
  if (n >= 2) load_v(n - 2, vn);
  for (int k = n - 2; k >= 0; --k) {
    c128 vv[NPL];
#pragma unroll
    for (int t = 0; t < NPL; ++t) vv[t] = vn[t];
    const c128 tk = tau[k];
    if (k > 0) load_v(k - 1, vn);
    if (tk.x == 0.0 && tk.y == 0.0) continue;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const c128 u = cmulc(vv[t], y[t]);   // conj(v_r) y_r
      sr += u.x;
      si += u.y;
    }
    const c128 sc = cmul(tk, c128{wave_sum(sr), wave_sum(si)});
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const c128 u = cmul(vv[t], sc);
      y[t] = c128{y[t].x - u.x, y[t].y - u.y};
    }
  }
#pragma unroll
  for (int t = 0; t < NPL; ++t) {
    const int r = lane + 64 * t;
    if (r < n) Y[(size_t)col * ldy + r] = y[t];
  }
}

// The same product for columns of up to 2048 rows with the reflectors staged
// through LDS: the four waves of a workgroup (four columns) share chunks of C
// reflectors, double-buffered; the loads of the next chunk are issued before
// the current chunk's C steps and written to LDS after them, so a step waits
// on LDS, not on memory (the one-step register prefetch above waited on
// every load).  The dot product keeps two partial sums per complex part.
template <int NPL>
__global__ void __launch_bounds__(256) k_backtr_lds(int n, const c128* __restrict__ A, int lda,
                                                    const c128* __restrict__ tau, const double* __restrict__ Z,
                                                    int ldz, int nev, c128* __restrict__ Y, int ldy,
                                                    const int* __restrict__ info) {
  constexpr int R = 64 * NPL;            // rows of a staged reflector (padded)
  constexpr int C = NPL >= 32 ? 1 : (NPL >= 16 ? 2 : (NPL >= 8 ? 4 : 8));   // 2 C R x 16 B <= 64 KB
  constexpr int PER = C * R / 256;       // chunk entries each thread stages
  __shared__ c128 buf[2][C * R];
  __shared__ c128 s_tau[2][C];
  if (*info != 0) return;
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const bool active = col < nev;   // every wave stays for the barriers
  c128 y[NPL];
#pragma unroll
  for (int t = 0; t < NPL; ++t) {
    const int r = lane + 64 * t;
    y[t] = c128{(active && r < n) ? Z[(size_t)col * ldz + r] : 0.0, 0.0};
  }
  // reflector k = n - 2 - (c C + j) is entry j of chunk c; v_k holds rows k+1 .. n-1
  c128 reg[PER], rtau = c128{0.0, 0.0};
  auto stage = [&](int c) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = threadIdx.x + 256 * e;
      const int j = idx / R, r = idx % R;
      const int k = n - 2 - c * C - j;
      reg[e] = (k >= 0 && r > k && r < n) ? A[(size_t)k * lda + r] : c128{0.0, 0.0};
    }
    if (threadIdx.x < C) {
      const int k = n - 2 - c * C - (int)threadIdx.x;
      rtau = k >= 0 ? tau[k] : c128{0.0, 0.0};
    }
  };
  auto commit = [&](int b) {
#pragma unroll
    for (int e = 0; e < PER; ++e) buf[b][threadIdx.x + 256 * e] = reg[e];
    if (threadIdx.x < C) s_tau[b][threadIdx.x] = rtau;
  };
  const int nchunks = (n - 1 + C - 1) / C;
  if (nchunks > 0) {
    stage(0);
    commit(0);
  }
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int cur = c & 1;
    if (c + 1 < nchunks) stage(c + 1);
    if (active) {
      for (int j = 0; j < C; ++j) {
        if (n - 2 - c * C - j < 0) break;
        const c128 tk = s_tau[cur][j];
        if (tk.x == 0.0 && tk.y == 0.0) continue;
        const c128* v = &buf[cur][j * R];
        // up to 8 rows a lane the reflector is held in registers for both
        // passes; beyond, it is read from LDS twice (registers hold y)
        constexpr int NV = NPL <= 8 ? NPL : 1;
        c128 vv[NV];
        if constexpr (NPL <= 8) {
#pragma unroll
          for (int t = 0; t < NPL; ++t) vv[t] = v[lane + 64 * t];
        }
        auto vat = [&](int t) -> c128 {
          if constexpr (NPL <= 8) return vv[t];
          else return v[lane + 64 * t];
        };
        double sr0 = 0.0, si0 = 0.0, sr1 = 0.0, si1 = 0.0;
#pragma unroll
        for (int t = 0; t < NPL; t += 2) {
          const c128 u = cmulc(vat(t), y[t]);   // conj(v_r) y_r
          sr0 += u.x;
          si0 += u.y;
          if (t + 1 < NPL) {
            const c128 u1 = cmulc(vat(t + 1), y[t + 1]);
            sr1 += u1.x;
            si1 += u1.y;
          }
        }
        const c128 sc = cmul(tk, c128{wave_sum(sr0 + sr1), wave_sum(si0 + si1)});
#pragma unroll
        for (int t = 0; t < NPL; ++t) {
          const c128 u = cmul(vat(t), sc);
          y[t] = c128{y[t].x - u.x, y[t].y - u.y};
        }
      }
    }
    if (c + 1 < nchunks) commit(cur ^ 1);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int t = 0; t < NPL; ++t) {
    const int r = lane + 64 * t;
    if (r < n) Y[(size_t)col * ldy + r] = y[t];
  }
}

}  // namespace

int pw::coop_workgroups(int n, bool wide) { return ceil_div(n, (n <= kCoopSmallN && !wide) ? 8 : CR); }

namespace {
size_t coop_bytes() { return sizeof(c128) * (4 * kCoopMaxN + 2 * kCoopMaxP) + 2 * 256 + kGoLines * 128; }
CoopBuf coop_buf(const pw::HeigWork& hw) {
  char* p = static_cast<char*>(hw.coop);
  CoopBuf cb;
  cb.p = reinterpret_cast<c128*>(p);
  cb.row = cb.p + 2 * kCoopMaxN;
  cb.s = cb.row + 2 * kCoopMaxN;
  cb.count = reinterpret_cast<unsigned*>(p + sizeof(c128) * (4 * kCoopMaxN + 2 * kCoopMaxP));
  cb.fail = reinterpret_cast<unsigned*>(p + sizeof(c128) * (4 * kCoopMaxN + 2 * kCoopMaxP) + 256);
  cb.go = reinterpret_cast<unsigned*>(p + sizeof(c128) * (4 * kCoopMaxN + 2 * kCoopMaxP) + 512);
  return cb;
}
}  // namespace

size_t pw::heig_work_bytes(int nmax) {
  const size_t n = (size_t)std::max(nmax, 1);
  return sizeof(c128) * (5 * n * n + 2 * n + 2 * n * PANEL) + sizeof(double) * (3 * n + n * n + 7 * n * (n + 64)) +
         sizeof(int) * n + 25 * 256 + coop_bytes();
}

pw_status pw::heig_setup(HeigWork& hw, void* base, int nmax) {
  const size_t n = (size_t)std::max(nmax, 1);
  {
    // 0 if the query fails: the large 8-row form is then not taken
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      hw.cus = cus;
    else
      hw.cus = 0;
    (void)hipGetLastError();
  }
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) / 256 * 256;
    return q;
  };
  hw.nmax = nmax;
  hw.L = reinterpret_cast<c128*>(take(sizeof(c128) * n * n));
  hw.X = reinterpret_cast<c128*>(take(sizeof(c128) * n * n));
  hw.T1 = reinterpret_cast<c128*>(take(sizeof(c128) * n * n));
  hw.A = reinterpret_cast<c128*>(take(sizeof(c128) * n * n));
  hw.Y = reinterpret_cast<c128*>(take(sizeof(c128) * n * n));
  hw.tau = reinterpret_cast<c128*>(take(sizeof(c128) * n));
  hw.d = reinterpret_cast<double*>(take(sizeof(double) * n));
  hw.e = reinterpret_cast<double*>(take(sizeof(double) * n));
  hw.w = reinterpret_cast<double*>(take(sizeof(double) * n));
  hw.Z = reinterpret_cast<double*>(take(sizeof(double) * n * n));
  hw.scratch = reinterpret_cast<double*>(take(sizeof(double) * 7 * n * (n + 64)));
  hw.info = reinterpret_cast<int*>(take(256));
  hw.gamma = reinterpret_cast<double*>(take(256));
  hw.drop = reinterpret_cast<int*>(take(sizeof(int) * n));
  hw.PV = reinterpret_cast<c128*>(take(sizeof(c128) * n * PANEL));
  hw.PW = reinterpret_cast<c128*>(take(sizeof(c128) * n * PANEL));
  hw.coop = take(coop_bytes());
  hw.cflags = reinterpret_cast<int*>(take(256));
  return PW_OK;
}

// Generalized eigenproblem of the n x n Hermitian pair (H, S) (col-major, ld):
// lowest nev eigenvalues -> w (device), eigenvectors -> C (n x nev, ldc).
// When n0 > 0 the factor L of S[0:n0, 0:n0] and X = L^-H from the previous
// call (or heig_reset) are still valid, and only the new block rows are
// factored:  U12 = X11^H S12,  L22 L22^H = S22 - U12^H U12,  X22 = L22^-H,
// X12 = -X11 U12 X22.
pw_status pw::heig_solve(HeigWork& hw, int n0, int n, int nev, const c128* H, const c128* S, int ld,
                         double* w, c128* C, int ldc, void* part, size_t part_bytes, hipStream_t st) {
  PW_CHECK(n <= hw.nmax && nev <= n && nev > 0 && n0 >= 0 && n0 < n, PW_EINVAL,
           "reduced problem larger than its workspace");
  const int ldw = hw.nmax;
  const int m = n - n0;
  // split-K workspace for the small products; none when solves run
  // concurrently (they fill the device already, and splitting K would only
  // add partial-sum traffic and launches)
  const size_t skb = hw.coop_wide ? 0 : part_bytes;
  c128* L22 = hw.L + (size_t)n0 * ldw + n0;
  c128* X22 = hw.X + (size_t)n0 * ldw + n0;
  if (n0 > 0) {
    PW_TRY((pw::zgemm_cn<double, double, double>(n0, m, n0, hw.X, ldw, S + (size_t)n0 * ld, ld, hw.T1, ldw,
                                                 part, part_bytes, st)));
  }
  if (n0 > 0) {
    // L22 = S22 - U12^H U12, reading S22 in place of a copy
    PW_TRY((pw::zgemm_cn<double, double, double>(m, m, n0, hw.T1, ldw, hw.T1, ldw, L22, ldw, part, part_bytes,
                                                 st, -1.0, 1.0, S + (size_t)n0 * ld + n0, ld)));
  } else {
    PW_HIP(hipMemcpy2DAsync(L22, sizeof(c128) * ldw, S + (size_t)n0 * ld + n0, sizeof(c128) * ld,
                            sizeof(c128) * m, m, hipMemcpyDeviceToDevice, st));
  }
  {
    pw::ProfScope ps(pw::PK_CHOL, st, 4.0 / 3.0 * m * m * (double)m);
    if (m <= kChRegN) {
      k_chol_reg<<<1, 1024, 0, st>>>(m, 0, hw.drop_tol, L22, ldw, hw.drop + n0, hw.info, hw.drop, n, nev);
    } else if (m < kChBlockedMinN) {
      k_chol<<<1, NTL, (sizeof(c128) + sizeof(double)) * m, st>>>(m, 0, hw.drop_tol, L22, ldw, hw.drop + n0, hw.info);
    } else {
      double* diag0 = hw.scratch;   // free until the eigenvector step
      c128* PT = hw.Y;              // free until X12 is formed
      k_chol_init<<<std::min(64, ceil_div(m, 256)), 256, 0, st>>>(m, L22, ldw, diag0, hw.cflags);
      for (int j0 = 0; j0 < m; j0 += kChPanel) {
        const int bb = std::min(kChPanel, m - j0);
        const int mt = m - j0 - bb;
        k_chol_diag<<<1, 256, 0, st>>>(j0, bb, hw.drop_tol, L22, ldw, diag0, hw.drop + n0, hw.cflags);
        if (mt > 0) k_chol_trsm<<<ceil_div(mt, 256), 256, 0, st>>>(m, j0, bb, L22, ldw, hw.drop + n0, hw.cflags, PT);
        if (mt > 0) {
          // trailing L22 -= L21 L21^H (full square; the upper triangle is cleared at the end)
          c128* L21 = L22 + (size_t)j0 * ldw + j0 + bb;
          c128* T22 = L22 + (size_t)(j0 + bb) * ldw + j0 + bb;
          PW_TRY((pw::zgemm_nn<double, double, double>(mt, mt, bb, -1.0, L21, ldw, PT, kChPanel, 1.0, T22, ldw,
                                                       st, hw.cflags)));
        }
      }
      k_chol_finish<<<std::min(1024, ceil_div((size_t)m * m, 256)), 256, 0, st>>>(m, L22, ldw, hw.cflags,
                                                                                hw.info);
    }
  }
  if (m > kChRegN) k_rank_check<<<1, 256, 0, st>>>(n, nev, hw.drop, hw.info);   // else done by k_chol_reg
  {
    pw::ProfScope ps(pw::PK_TRINV, st, 8.0 / 3.0 * m * m * (double)m);
    k_trinv<<<m, 256, sizeof(c128) * m, st>>>(m, L22, ldw, X22, ldw, hw.info);
  }
  if (n0 > 0) {
    // X12 = -X11 (U12 X22)
    PW_TRY(pw::zgemm_nn_sk(n0, m, m, 1.0, hw.T1, ldw, X22, ldw, 0.0, hw.Y, ldw, part, skb, st));
    PW_TRY(pw::zgemm_nn_sk(n0, m, n0, -1.0, hw.X, ldw, hw.Y, ldw, 0.0, hw.X + (size_t)n0 * ldw, ldw, part,
                           skb, st));
    k_zero_block<<<std::min(1024, ceil_div(m * n0, 256)), 256, 0, st>>>(n0, n, n0, hw.X, ldw);
  }
  // A = X^H (H X)
  PW_TRY(pw::zgemm_nn_sk(n, n, n, 1.0, H, ld, hw.X, ldw, 0.0, hw.T1, ldw, part, skb, st));
  PW_TRY((pw::zgemm_cn<double, double, double>(n, n, n, hw.X, ldw, hw.T1, ldw, hw.A, ldw, part,
                                               part_bytes, st)));
  const bool coop_tri = hw.coop_ok && n >= kCoopMinN && n <= kCoopMaxN;
  k_isolate<<<std::min(1024, ceil_div(n * n, 256)), 256, 0, st>>>(
      n, hw.A, ldw, hw.drop, hw.info, coop_tri ? coop_buf(hw).count : nullptr, coop_tri ? coop_buf(hw).fail : nullptr,
      coop_tri ? coop_buf(hw).go : nullptr, hw.gamma);
  // tridiagonalize, eigenvalues, eigenvectors of T, back-transform
  {
    pw::ProfScope ps(pw::PK_TRIDIAG, st, 16.0 / 3.0 * n * n * (double)n);
    if (coop_tri) {
      const CoopBuf cb = coop_buf(hw);   // counter and flag cleared by k_isolate
      const bool wide = hw.coop_wide;
      // beyond 512 rows a solve that runs alone keeps 8 rows per workgroup,
      // in passes of 512 columns (up to one workgroup per CU at 2048 rows):
      // 16 rows per workgroup do not fit the registers there (at 2048 rows
      // they spilled 885 registers a thread, and the update ran from scratch
      // memory)
      const bool big8 = !wide && n > 2 * CB && hw.cus >= ceil_div(n, 8);
      const int P = big8 ? ceil_div(n, 8) : pw::coop_workgroups(n, wide);
      // up to 512 rows: 8 rows per workgroup (twice the workgroups, half the
      // update work per step on each) unless the wide form is asked for; beyond, 16
      if (big8 && n <= 4 * CB)
        k_tridiag_coop<2, 8, 2 * CB><<<P, CT, 0, st>>>(n, hw.A, ldw, hw.d, hw.e, hw.tau, hw.info, cb);
      else if (big8)
        k_tridiag_coop<4, 8, 2 * CB><<<P, CT, 0, st>>>(n, hw.A, ldw, hw.d, hw.e, hw.tau, hw.info, cb);
      else if (n <= CB && !wide) k_tridiag_coop<1, 8><<<P, CT, 0, st>>>(n, hw.A, ldw, hw.d, hw.e, hw.tau, hw.info, cb);
      else if (n <= CB) k_tridiag_coop<1, CR><<<P, CT, 0, st>>>(n, hw.A, ldw, hw.d, hw.e, hw.tau, hw.info, cb);
      else if (n <= 2 * CB && !wide)
        k_tridiag_coop<2, 8><<<P, CT, 0, st>>>(n, hw.A, ldw, hw.d, hw.e, hw.tau, hw.info, cb);
      else if (n <= 2 * CB) k_tridiag_coop<2, CR><<<P, CT, 0, st>>>(n, hw.A, ldw, hw.d, hw.e, hw.tau, hw.info, cb);
      else if (n <= 4 * CB) k_tridiag_coop<4, CR><<<P, CT, 0, st>>>(n, hw.A, ldw, hw.d, hw.e, hw.tau, hw.info, cb);
      else k_tridiag_coop<8, CR><<<P, CT, 0, st>>>(n, hw.A, ldw, hw.d, hw.e, hw.tau, hw.info, cb);
    } else if (n <= kPanelMinN) {
      k_tridiag<<<1, NTL, sizeof(c128) * (2 * n + std::max(n, NTL)), st>>>(n, hw.A, ldw, hw.d, hw.e, hw.tau,
                                                                          hw.info);
    } else {
      const size_t lds = sizeof(c128) * (2 * (size_t)n + std::max(n, NTL));
      for (int k0 = 0; k0 < n - 1; k0 += PANEL) {
        const int bb = std::min(PANEL, n - 1 - k0);
        k_tridiag_panel<<<1, NTL, lds, st>>>(n, k0, bb, hw.A, ldw, hw.PV, hw.PW, hw.d, hw.e, hw.tau, hw.info);
        const int r = k0 + bb, mm = n - r;
        if (mm > 0) {
          c128* C = hw.A + (size_t)r * ldw + r;
          PW_TRY((pw::zgemm_cn<double, double, double>(mm, mm, bb, hw.PV + (size_t)r * PANEL, PANEL,
                                                       hw.PW + (size_t)r * PANEL, PANEL, C, ldw, part,
                                                       part_bytes, st, -1.0, 1.0)));
          PW_TRY((pw::zgemm_cn<double, double, double>(mm, mm, bb, hw.PW + (size_t)r * PANEL, PANEL,
                                                       hw.PV + (size_t)r * PANEL, PANEL, C, ldw, part,
                                                       part_bytes, st, -1.0, 1.0)));
        }
      }
      k_tridiag_last<<<1, 64, 0, st>>>(n, hw.A, ldw, hw.d, hw.info);
    }
  }
  {
    pw::ProfScope ps(pw::PK_BISECT, st);
    // four waves per eigenvalue while they find a SIMD each (up to 256
    // eigenvalues); beyond, one wave each (more waves would share SIMDs and
    // the Sturm steps are issue-bound there)
    k_bisect<<<nev, nev <= 256 ? 256 : 64, sizeof(double) * 2 * n, st>>>(n, hw.d, hw.e, nev, w, hw.info);
  }
  {
    pw::ProfScope ps(pw::PK_INVIT, st);
    const size_t per_thread = 49 * (size_t)n, shared = 16 * (size_t)n;
    if (8 * per_thread + shared <= (size_t)kInvitLdsBytes)
      k_invit_lds<8><<<ceil_div(nev, 8), 64, 8 * per_thread + shared, st>>>(n, hw.d, hw.e, nev, w, hw.Z, ldw,
                                                                          hw.info);
    else if (4 * per_thread + shared <= (size_t)kInvitLdsBytes)
      k_invit_lds<4><<<ceil_div(nev, 4), 64, 4 * per_thread + shared, st>>>(n, hw.d, hw.e, nev, w, hw.Z, ldw,
                                                                          hw.info);
    else
      k_invit<<<ceil_div(nev, 64), 64, 0, st>>>(n, hw.d, hw.e, nev, w, hw.Z, ldw, hw.scratch, hw.info);
  }
  {
    pw::ProfScope ps(pw::PK_BACKTR, st, 8.0 * n * n * (double)nev);
    const dim3 g(ceil_div(nev, 4)), b(256);
    const int npl = ceil_div(n, 64);
    if (npl <= 2) k_backtr_lds<2><<<g, b, 0, st>>>(n, hw.A, ldw, hw.tau, hw.Z, ldw, nev, hw.Y, ldw, hw.info);
    else if (npl <= 4) k_backtr_lds<4><<<g, b, 0, st>>>(n, hw.A, ldw, hw.tau, hw.Z, ldw, nev, hw.Y, ldw, hw.info);
    else if (npl <= 8) k_backtr_lds<8><<<g, b, 0, st>>>(n, hw.A, ldw, hw.tau, hw.Z, ldw, nev, hw.Y, ldw, hw.info);
    else if (npl <= 16) k_backtr_lds<16><<<g, b, 0, st>>>(n, hw.A, ldw, hw.tau, hw.Z, ldw, nev, hw.Y, ldw, hw.info);
    else if (npl <= 32) k_backtr_lds<32><<<g, b, 0, st>>>(n, hw.A, ldw, hw.tau, hw.Z, ldw, nev, hw.Y, ldw, hw.info);
    else if (npl <= 64) k_backtr<64><<<g, b, 0, st>>>(n, hw.A, ldw, hw.tau, hw.Z, ldw, nev, hw.Y, ldw, hw.info);
    else return pw::fail(PW_EINVAL, "reduced problem larger than 4096");
  }
  // C = X Y
  PW_TRY(pw::zgemm_nn_sk(n, nev, n, 1.0, hw.X, ldw, hw.Y, ldw, 0.0, C, ldc, part, skb, st));
  // hw.Z (eigenvectors of T) is free once the back-transform has run
  k_colnorms<<<ceil_div(nev, 4), 256, 0, st>>>(n, nev, C, ldc, hw.gamma, hw.info);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw::heig_reset(HeigWork& hw, int n, hipStream_t st) {
  k_identity<<<std::min(1024, ceil_div(n * n, 256)), 256, 0, st>>>(n, hw.L, hw.X, hw.nmax, hw.drop);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw::heig_set_limits() {
  static bool done = false;
  if (done) return PW_OK;
  // only the tridiagonalization can need more than the default 64 KB of
  // dynamic LDS (n > 1365); allow what is left next to its static LDS
  for (const void* fn : {(const void*)k_tridiag, (const void*)k_tridiag_panel, (const void*)k_invit_lds<8>,
                         (const void*)k_invit_lds<4>}) {
    hipFuncAttributes at;
    PW_HIP(hipFuncGetAttributes(&at, fn));
    const int lim = 160 * 1024 - (int)at.sharedSizeBytes;
    PW_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  }
  done = true;
  return PW_OK;
}

extern "C" pw_status pw_reduced_eigh(pw_ctx ctx, int32_t n, int32_t nev, const pw_c128* H, const pw_c128* S,
                                     int32_t ld, double* w, pw_c128* C, int32_t ldc, double* debug,
                                     void* stream) {
  PW_CHECK(ctx != nullptr, PW_EINVAL, "NULL context");
  PW_CHECK(n >= 1 && nev >= 1 && nev <= n && ld >= n && ldc >= n, PW_EINVAL, "bad sizes");
  PW_CHECK(H && S && w && C, PW_EINVAL, "NULL pointer");
  PW_HIP(hipSetDevice(ctx->device));
  PW_TRY(pw::heig_set_limits());
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t hb = pw::heig_work_bytes(n);
  const size_t pb = pw::splitk_part_bytes(n, n, n, sizeof(c128));
  void *base = nullptr, *part = nullptr;
  if (hipMalloc(&base, hb) != hipSuccess || hipMalloc(&part, pb) != hipSuccess) {
    (void)hipGetLastError();
    if (base) (void)hipFree(base);
    return pw::fail(PW_ENOMEM, "workspace allocation failed");
  }
  pw::HeigWork hw;
  pw::heig_setup(hw, base, n);
  pw_status stt = pw::heig_solve(hw, 0, n, nev, reinterpret_cast<const c128*>(H), reinterpret_cast<const c128*>(S),
                                 ld, w, reinterpret_cast<c128*>(C), ldc, part, pb, st);
  int info = 0;
  if (stt == PW_OK && debug) {
    if (hipMemcpyAsync(debug, hw.d, sizeof(double) * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        (n > 1 && hipMemcpyAsync(debug + n, hw.e, sizeof(double) * (n - 1), hipMemcpyDeviceToDevice, st) != hipSuccess))
      stt = pw::fail(PW_EDEVICE, "copy of the tridiagonal failed");
  }
  if (stt == PW_OK) {
    if (hipMemcpyAsync(&info, hw.info, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      stt = pw::fail(PW_EDEVICE, "reduced eigensolver failed");
    else if (info == 2)
      stt = pw::fail(PW_EDEVICE, "workgroups of the cooperative tridiagonalization were not co-resident");
    else if (info != 0)
      stt = pw::fail(PW_EBREAKDOWN, "S is not positive definite or has rank < nev");
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(base);
  (void)hipFree(part);
  return stt;
}

// ---------------------------------------------------------------------------
// Allocation-free variant of pw_reduced_eigh: the workspace is a file-scope
// device array (one copy per GPU, held until the process ends) instead of
// hipMalloc'd memory.  Host code never passes the array's name to a kernel:
// it uses the device address hipGetSymbolAddress returns for each device.
// ---------------------------------------------------------------------------
namespace {
constexpr int kNoAllocMaxN = 256;
constexpr size_t kNoAllocBytes = (size_t)48 << 20;   // 48 MiB per device
constexpr int kMaxDevices = 64;
__device__ __align__(256) char scratch[kNoAllocBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Looks up this device's copy of the array; `device` must be current.
pw_status pw::noalloc_scratch_init(int device) {
  PW_CHECK(device >= 0 && device < kMaxDevices, PW_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return PW_OK;
  const size_t need = (heig_work_bytes(kNoAllocMaxN) + 255) / 256 * 256 +
                      splitk_part_bytes(kNoAllocMaxN, kNoAllocMaxN, kNoAllocMaxN, sizeof(c128));
  PW_CHECK(need <= kNoAllocBytes, PW_EDEVICE, "static scratch array smaller than its stated capacity");
  void* ptr = nullptr;
  PW_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  PW_CHECK(ptr != nullptr, PW_EDEVICE, "no device address for the static scratch array");
  g_scratch_ptr[device] = ptr;
  return PW_OK;
}

extern "C" pw_status pw_reduced_eigh_noalloc(pw_ctx ctx, int32_t n, int32_t nev, const pw_c128* H,
                                             const pw_c128* S, int32_t ld, double* w, pw_c128* C, int32_t ldc,
                                             double* debug, void* stream) {
  PW_CHECK(ctx != nullptr, PW_EINVAL, "NULL context");
  PW_CHECK(n >= 1 && nev >= 1 && nev <= n && ld >= n && ldc >= n, PW_EINVAL, "bad sizes");
  PW_CHECK(n <= kNoAllocMaxN, PW_EINVAL,
           "n = " + std::to_string(n) + " exceeds the static workspace (n <= " + std::to_string(kNoAllocMaxN) + ")");
  PW_CHECK(H && S && w && C, PW_EINVAL, "NULL pointer");
  PW_HIP(hipSetDevice(ctx->device));
  PW_TRY(pw::heig_set_limits());
  PW_TRY(pw::noalloc_scratch_init(ctx->device));   // set at context creation; a no-op here
  void* base = g_scratch_ptr[ctx->device];
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t hb = (pw::heig_work_bytes(n) + 255) / 256 * 256;
  const size_t pb = pw::splitk_part_bytes(n, n, n, sizeof(c128));
  void* part = static_cast<char*>(base) + hb;
  pw::HeigWork hw;
  pw::heig_setup(hw, base, n);
  pw_status stt = pw::heig_solve(hw, 0, n, nev, reinterpret_cast<const c128*>(H), reinterpret_cast<const c128*>(S),
                                 ld, w, reinterpret_cast<c128*>(C), ldc, part, pb, st);
  if (stt == PW_OK && debug) {
    if (hipMemcpyAsync(debug, hw.d, sizeof(double) * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        (n > 1 && hipMemcpyAsync(debug + n, hw.e, sizeof(double) * (n - 1), hipMemcpyDeviceToDevice, st) != hipSuccess))
      stt = pw::fail(PW_EDEVICE, "copy of the tridiagonal failed");
  }
  int info = 0;
  if (stt == PW_OK) {
    if (hipMemcpyAsync(&info, hw.info, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      stt = pw::fail(PW_EDEVICE, "reduced eigensolver failed");
    else if (info == 2)
      stt = pw::fail(PW_EDEVICE, "workgroups of the cooperative tridiagonalization were not co-resident");
    else if (info != 0)
      stt = pw::fail(PW_EBREAKDOWN, "S is not positive definite or has rank < nev");
  }
  (void)hipStreamSynchronize(st);
  return stt;
}
