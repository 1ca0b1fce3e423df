// H.psi on the plane-wave sphere: plan construction (sphere -> FFT box maps,
// kinetic and preconditioner diagonals, twiddles, operator copies) and the
// three transform passes of the local potential term:
//
//   k_zinv  : gather psi(G) onto z sticks, inverse z transform      (sphere -> sticks)
//   k_plane : per z plane, inverse y (x columns that hold sticks), inverse x,
//             multiply by V(r), forward x, forward y; only stick positions
//             are written back                                        (sticks -> sticks)
//   k_zfwd  : forward z transform, 1/N, gather to the sphere, add the
//             kinetic term 1/2 |k+G|^2 psi(G)                        (sticks -> sphere)
//
// followed by the projector term (calbec, D blocks, add back), see zgemm.hip.
// The product equals sum_G' Vt((m_G - m_G') mod n) psi(G') exactly (up to
// rounding), Vt being the discrete Fourier coefficients of V(r) on the grid;
// with n_d >= 4 max|m_d| + 1 no wrapped term reaches the sphere.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "fft_reg.h"
#include "plan.h"
#include "profile.h"

namespace {

constexpr int ZSB = 16;        // sticks per workgroup in the z passes
constexpr int ZTHREADS = 128;
constexpr int PTHREADS = 256;

template <typename T>
__device__ __forceinline__ cpx<T> to_t(c128 v) { return cpx<T>{(T)v.x, (T)v.y}; }

// Workgroup -> (stick chunk, band) of the z passes.  Workgroups go to the 8
// XCDs round-robin by linear id, so all chunks of one band get ids of one
// residue mod 8: each band's scattered sphere reads then meet one L2.  The
// grid has gz * roundup(nb, 8) workgroups; those past the last band exit.
constexpr int kXcds = 8;
__device__ __forceinline__ bool z_tile(int gz, int nb, int& chunk, int& band) {
  const int id = blockIdx.x;
  const int slot = id / kXcds;
  band = (slot / gz) * kXcds + id % kXcds;
  chunk = slot % gz;
  return band < nb;
}

// ---------------------------------------------------------------------------
// pass 1: sphere -> sticks, inverse z transform
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(ZTHREADS)
k_zinv(SphereMap m, const c128* __restrict__ psi, int ldpsi,
       cpx<T>* __restrict__ sticks, const cpx<T>* __restrict__ twg, int gz, int nb) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n3 = m.n3;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = tw + n3;
  cpx<T>* B = A + ZSB * n3;
  int chunk, band;
  if (!z_tile(gz, nb, chunk, band)) return;
  const int s0 = chunk * ZSB;
  const int ns = min(ZSB, m.nst - s0);
  const c128* pb = psi + (size_t)band * ldpsi;
  for (int i = threadIdx.x; i < n3; i += blockDim.x) tw[i] = twg[i];
  for (int i = threadIdx.x; i < ZSB * n3; i += blockDim.x) B[i] = cpx<T>{T(0), T(0)};
  __syncthreads();
  const int e0 = m.st_ptr[s0], e1 = m.st_ptr[s0 + ns];
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x)
    B[(m.ent_s[e] - s0) * n3 + m.ent_z[e]] = to_t<T>(pb[m.ent_g[e]]);
  __syncthreads();
  cpx<T>* out = sticks + (size_t)band * n3 * m.ldst + s0;
  const int ldst = m.ldst;
  fft_run<T>(
      m.f3, ns, T(1), tw, A, B, n3, false, true,
      [&](int b, int i) { return B[b * n3 + i]; },
      [&](int b, int i, cpx<T> v) { out[(size_t)i * ldst + b] = v; });
}

// ---------------------------------------------------------------------------
// pass 2: one z plane of one band
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(PTHREADS)
k_plane(SphereMap m, cpx<T>* __restrict__ sticks, const T* __restrict__ vr,
        const cpx<T>* __restrict__ tw1g, const cpx<T>* __restrict__ tw2g, int cbatch) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n1 = m.n1, n2 = m.n2, nxr = m.nxr, nst = m.nst;
  const int lmax = max(n1, n2);
  cpx<T>* tw1 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw2 = tw1 + n1;
  cpx<T>* Y = tw2 + n2;              // [nxr][n2]
  cpx<T>* A = Y + nxr * n2;          // [cbatch][lmax]
  cpx<T>* B = A + cbatch * lmax;     // [cbatch][lmax]
  int* hx_of = reinterpret_cast<int*>(B + cbatch * lmax);   // [n1]

  // band fastest in the launch order: the workgroups in flight share z
  // planes, so each plane of V(r) is read from HBM about once per XCD
  const int band = blockIdx.x;
  const int z = blockIdx.y;
  cpx<T>* st = sticks + ((size_t)band * m.n3 + z) * m.ldst;
  const T* vz = vr + (size_t)z * n1 * n2;

  for (int i = threadIdx.x; i < n1; i += blockDim.x) { tw1[i] = tw1g[i]; hx_of[i] = m.i1_hx[i]; }
  for (int i = threadIdx.x; i < n2; i += blockDim.x) tw2[i] = tw2g[i];
  for (int i = threadIdx.x; i < nxr * n2; i += blockDim.x) Y[i] = cpx<T>{T(0), T(0)};
  __syncthreads();
  for (int s = threadIdx.x; s < nst; s += blockDim.x) Y[m.st_hx[s] * n2 + m.st_i2[s]] = st[s];
  __syncthreads();

  // inverse y on the x columns that hold sticks
  for (int c0 = 0; c0 < nxr; c0 += cbatch) {
    const int nc = min(cbatch, nxr - c0);
    cpx<T>* Yc = Y + c0 * n2;
    fft_run<T>(
        m.f2, nc, T(1), tw2, A, B, lmax, false, false,
        [&](int b, int i) { return Yc[b * n2 + i]; },
        [&](int b, int i, cpx<T> v) { Yc[b * n2 + i] = v; });
  }

  // rows: inverse x (x_r nonzero inputs), times V(r), forward x (x_r outputs kept)
  const int lr = fft_last_read(m.f1);
  cpx<T>* X = (lr == 0) ? B : A;
  cpx<T>* P0 = (X == A) ? B : A;
  for (int r0 = 0; r0 < n2; r0 += cbatch) {
    const int nr = min(cbatch, n2 - r0);
    fft_run<T>(
        m.f1, nr, T(1), tw1, A, B, lmax, false, false,
        [&](int b, int i) {
          const int hx = hx_of[i];
          return hx >= 0 ? Y[hx * n2 + r0 + b] : cpx<T>{T(0), T(0)};
        },
        [&](int b, int i, cpx<T> v) { X[b * lmax + i] = v * vz[(r0 + b) * n1 + i]; });
    fft_run<T>(
        m.f1, nr, T(-1), tw1, P0, X, lmax, false, false,
        [&](int b, int i) { return X[b * lmax + i]; },
        [&](int b, int i, cpx<T> v) {
          const int hx = hx_of[i];
          if (hx >= 0) Y[hx * n2 + r0 + b] = v;
        });
  }

  // forward y on the x columns
  for (int c0 = 0; c0 < nxr; c0 += cbatch) {
    const int nc = min(cbatch, nxr - c0);
    cpx<T>* Yc = Y + c0 * n2;
    fft_run<T>(
        m.f2, nc, T(-1), tw2, A, B, lmax, false, false,
        [&](int b, int i) { return Yc[b * n2 + i]; },
        [&](int b, int i, cpx<T> v) { Yc[b * n2 + i] = v; });
  }
  for (int s = threadIdx.x; s < nst; s += blockDim.x) st[s] = Y[m.st_hx[s] * n2 + m.st_i2[s]];
}


// ---------------------------------------------------------------------------
// pass 2, register-resident variant for n1 = n2 = 4 LS: one workgroup per
// (PP consecutive z planes, band); each 1D transform runs on one quad of lanes
// in VGPRs (see fft_reg.h); LDS only holds the planes' x columns
// Y[PP][nxr][n2 + 1] as the transpose between the y and x transforms.  The
// columns (rows) of the PP planes form one index space per phase, so a
// workgroup's last pass over them is fuller than with one plane.
// ---------------------------------------------------------------------------
template <typename T, int LS, int PP>
__global__ void __launch_bounds__(512)
k_plane_reg(SphereMap m, cpx<T>* __restrict__ sticks, const T* __restrict__ vr,
            const cpx<T>* __restrict__ tw1g, const cpx<T>* __restrict__ tw2g) {
  constexpr int N = 4 * LS;     // n1 = n2 = N
  constexpr int YS = N + 1;     // padded column stride
  extern __shared__ __align__(16) char smem_raw[];
  const int nxr = m.nxr, nst = m.nst;
  cpx<T>* tw1 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw2 = tw1 + N;
  cpx<T>* Y = tw2 + N;                                        // [PP][nxr][YS]
  int* hx_of = reinterpret_cast<int*>(Y + PP * nxr * YS);     // [N]
  const int z0 = blockIdx.y * PP, band = blockIdx.x;   // band fastest (see k_plane)
  const int np = min(PP, m.n3 - z0);                          // planes of this workgroup
  cpx<T>* st = sticks + ((size_t)band * m.n3 + z0) * m.ldst;   // plane pz at st + pz ldst
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    tw1[i] = tw1g[i];
    tw2[i] = tw2g[i];
    hx_of[i] = m.i1_hx[i];
  }
  for (int i = threadIdx.x; i < np * nxr * YS; i += blockDim.x) Y[i] = cpx<T>{T(0), T(0)};
  __syncthreads();
  for (int e = threadIdx.x; e < np * nst; e += blockDim.x) {
    const int pz = e / nst, s = e - pz * nst;
    Y[(pz * nxr + m.st_hx[s]) * YS + m.st_i2[s]] = st[(size_t)pz * m.ldst + s];
  }
  __syncthreads();
  const int q = threadIdx.x & 3, nquads = blockDim.x >> 2;
  const int pb = regfft::quad_block(q);   // block of the transform held after inv_dit
  const regfft::QuadLane<T> ql = regfft::quad_lane<T>(q);
  // inverse y transforms of the x columns (column c = pz nxr + x)
  for (int c = threadIdx.x >> 2; c < np * nxr; c += nquads) {
    cpx<T> x[LS];
    cpx<T>* col = Y + c * YS;
#pragma unroll
    for (int j = 0; j < LS; ++j) x[j] = col[q + 4 * j];
    regfft::inv_dit<LS, T>(x, q, ql, tw2);
#pragma unroll
    for (int k = 0; k < LS; ++k) col[k + LS * pb] = x[k];
  }
  __syncthreads();
  // rows (row index pz N + r): inverse x, V(r), forward x; only the x columns
  // of the sphere are read and written
  for (int rr = threadIdx.x >> 2; rr < np * N; rr += nquads) {
    const int pz = rr / N, r = rr - pz * N;
    const cpx<T>* Yp = Y + pz * nxr * YS;
    cpx<T> x[LS];
#pragma unroll
    for (int j = 0; j < LS; ++j) {
      const int hx = hx_of[q + 4 * j];
      x[j] = hx >= 0 ? Yp[hx * YS + r] : cpx<T>{T(0), T(0)};
    }
    regfft::inv_dit<LS, T>(x, q, ql, tw1);
    const T* vrow = vr + ((size_t)(z0 + pz) * N + r) * N + LS * pb;
#pragma unroll
    for (int k = 0; k < LS; ++k) x[k] = x[k] * vrow[k];
    regfft::fwd_dif<LS, T>(x, q, ql, tw1);
    cpx<T>* Yw = Y + pz * nxr * YS;
#pragma unroll
    for (int j = 0; j < LS; ++j) {
      const int hx = hx_of[q + 4 * j];
      if (hx >= 0) Yw[hx * YS + r] = x[j];
    }
  }
  __syncthreads();
  // forward y transforms
  for (int c = threadIdx.x >> 2; c < np * nxr; c += nquads) {
    cpx<T> x[LS];
    cpx<T>* col = Y + c * YS;
#pragma unroll
    for (int k = 0; k < LS; ++k) x[k] = col[k + LS * pb];
    regfft::fwd_dif<LS, T>(x, q, ql, tw2);
#pragma unroll
    for (int j = 0; j < LS; ++j) col[q + 4 * j] = x[j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < np * nst; e += blockDim.x) {
    const int pz = e / nst, s = e - pz * nst;
    st[(size_t)pz * m.ldst + s] = Y[(pz * nxr + m.st_hx[s]) * YS + m.st_i2[s]];
  }
}

// ---------------------------------------------------------------------------
// pass 2, lane-group variant for n1 = n2 = G LS (G = 16 lanes per 1D
// transform): one workgroup per (z plane, band) holds the plane's x columns
// Y[nxr][N] in LDS with no padding -- a float64 144 x 71 plane (163,584
// bytes) fits in the 160 KB of a CU -- and each 1D transform runs on a group
// of G lanes in VGPRs (fft_reg.h).  The y transforms read their sticks
// straight from HBM and write them back through the (column, y) -> stick
// map; twiddles, the x map and V(r) come from global memory (L1/L2), so the
// plane is the kernel's only LDS.
// ---------------------------------------------------------------------------
constexpr int OCT_G = 16;          // lanes per 1D transform
// 512 threads (32 groups of 16 lanes).  float64: one workgroup per CU (the
// plane fills the LDS), two waves per SIMD with up to 256 registers;
// float32: at most 128 registers, so that two workgroups (two 82 KB planes)
// share a CU.
template <typename T>
struct OctCfg {
  static constexpr int threads = 512;
  static constexpr int waves = sizeof(T) == 8 ? 2 : 4;
};

// LDS position of (x column c, y): y ^ 2 sigma(c mod 8), sigma rotating the
// three bits of c mod 8 right, so bit 3 of the mask is bit 0 of c.  Column
// accesses (consecutive y of one or two columns per 16 lanes) and row
// accesses (neighbouring columns at one y) then spread over the banks.  The
// mask stays below 16 and N is a multiple of 16: a bijection of each column.
template <int N>
__device__ __forceinline__ int oct_pos(int c, int y) {
  const int sg = ((c & 1) << 2) | ((c >> 1) & 3);
  return c * N + (y ^ (sg << 1));
}

template <typename T, int LS>
__global__ void __launch_bounds__(OctCfg<T>::threads) __attribute__((amdgpu_waves_per_eu(OctCfg<T>::waves)))
k_plane_oct(SphereMap m, cpx<T>* __restrict__ sticks, const T* __restrict__ vr, const cpx<T>* __restrict__ tw) {
  constexpr int G = OCT_G;
  constexpr int N = G * LS;
  static_assert(N % 16 == 0, "the LDS swizzle permutes within aligned blocks of 16");
  extern __shared__ __align__(16) char smem_raw[];
  cpx<T>* Y = reinterpret_cast<cpx<T>*>(smem_raw);   // [nxr][N], swizzled
  const int nxr = m.nxr;
  const int z = blockIdx.y, band = blockIdx.x;   // band fastest (see k_plane)
  cpx<T>* st = sticks + ((size_t)band * m.n3 + z) * m.ldst;
  const int g = threadIdx.x & (G - 1), grp = threadIdx.x / G, ngrp = blockDim.x / G;
  const int pb = regfft::g_block<G>(g);   // block of the transform held after ginv
  const regfft::GLane<T> gl = regfft::glane<T>(g);
  // inverse y transforms: the sticks of column c -> Y[c][*]
#pragma unroll 1
  for (int c = grp; c < nxr; c += ngrp) {
    const int* cs = m.cy_st + (size_t)c * N;
    cpx<T> x[LS];
#pragma unroll
    for (int j = 0; j < LS; ++j) {
      const int sidx = cs[g + G * j];
      x[j] = sidx >= 0 ? st[sidx] : cpx<T>{T(0), T(0)};
    }
    regfft::ginv<G, LS, T>(x, g, gl, tw);
#pragma unroll
    for (int k = 0; k < LS; ++k) Y[oct_pos<N>(c, k + LS * pb)] = x[k];
  }
  __syncthreads();
  // rows: inverse x, V(r), forward x; only the x columns of the sphere are
  // read and written
  int hx[LS];
#pragma unroll
  for (int j = 0; j < LS; ++j) hx[j] = m.i1_hx[g + G * j];
#pragma unroll 1
  for (int r = grp; r < N; r += ngrp) {
    const T* vrow = vr + ((size_t)z * N + r) * N + LS * pb;
    cpx<T> x[LS];
#pragma unroll
    for (int j = 0; j < LS; ++j) x[j] = hx[j] >= 0 ? Y[oct_pos<N>(hx[j], r)] : cpx<T>{T(0), T(0)};
    regfft::ginv<G, LS, T>(x, g, gl, tw);
    // keep the V(r) loads after the transform: hoisted above it they would
    // hold LS more registers through it
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < LS; ++k) x[k] = x[k] * vrow[k];
    regfft::gfwd<G, LS, T>(x, g, gl, tw);
#pragma unroll
    for (int j = 0; j < LS; ++j)
      if (hx[j] >= 0) Y[oct_pos<N>(hx[j], r)] = x[j];
  }
  __syncthreads();
  // forward y transforms: Y[c][*] -> the sticks of column c
#pragma unroll 1
  for (int c = grp; c < nxr; c += ngrp) {
    cpx<T> x[LS];
#pragma unroll
    for (int k = 0; k < LS; ++k) x[k] = Y[oct_pos<N>(c, k + LS * pb)];
    regfft::gfwd<G, LS, T>(x, g, gl, tw);
    const int* cs = m.cy_st + (size_t)c * N;
#pragma unroll
    for (int j = 0; j < LS; ++j) {
      const int sidx = cs[g + G * j];
      if (sidx >= 0) st[sidx] = x[j];
    }
  }
}

template <typename T>
using PlaneOctFn = void (*)(SphereMap, cpx<T>*, const T*, const cpx<T>*);

// lane-group plane kernel for n1 = n2 = 16 LS, or nullptr
template <typename T>
PlaneOctFn<T> plane_oct_kernel(int n1, int n2) {
  if (n1 != n2) return nullptr;
  switch (n1) {
    case 80: return k_plane_oct<T, 5>;
    case 96: return k_plane_oct<T, 6>;
    case 128: return k_plane_oct<T, 8>;
    case 144: return k_plane_oct<T, 9>;
    default: return nullptr;
  }
}

// the plane is the lane-group kernel's only LDS; a workgroup may take all 160 KB of a CU
constexpr size_t kPlaneOctMaxLds = 160 * 1024;
template <typename T>
size_t plane_oct_lds_bytes(int n, int nxr) { return sizeof(cpx<T>) * (size_t)n * nxr; }
template <typename T>
bool plane_oct_fits(int n1, int n2, int nxr) {
  return plane_oct_kernel<T>(n1, n2) != nullptr && plane_oct_lds_bytes<T>(n1, nxr) <= kPlaneOctMaxLds;
}

// ---------------------------------------------------------------------------
// pass 2, three-kernel form for planes whose x columns do not fit in LDS
// (float64 at 144^2 and above): the y transforms and the x transforms of a
// plane run in separate kernels and meet in an HBM copy of the plane's x
// columns, rows[band][z][n2][nxr] (y major, the x columns of one row
// contiguous).  Each workgroup holds only CB columns or CB rows.
// ---------------------------------------------------------------------------
constexpr int SPLIT_CB = 16;        // columns / rows per workgroup
constexpr int SPLIT_THREADS = 256;

template <typename T>
size_t split_lds_bytes(int n1, int n2) {
  const int lmax = std::max(n1, n2);
  return 2 * sizeof(cpx<T>) * (size_t)SPLIT_CB * lmax + sizeof(int) * (size_t)SPLIT_CB * n2 +
         sizeof(int) * (size_t)n1;
}

// sticks of x columns [c0, c0+CB) -> inverse y -> rows
template <typename T>
__global__ void __launch_bounds__(SPLIT_THREADS)
k_plane_yinv(SphereMap m, const cpx<T>* __restrict__ sticks, cpx<T>* __restrict__ rows,
             const cpx<T>* __restrict__ tw2) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n2 = m.n2, nxr = m.nxr, lmax = max(m.n1, n2);
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* B = A + SPLIT_CB * lmax;
  int* sidx = reinterpret_cast<int*>(B + SPLIT_CB * lmax);   // [CB][n2] stick at (column, y) or -1
  const int z = blockIdx.x, band = blockIdx.y, c0 = blockIdx.z * SPLIT_CB;
  const int nc = min(SPLIT_CB, nxr - c0);
  for (int i = threadIdx.x; i < SPLIT_CB * n2; i += blockDim.x) sidx[i] = -1;
  __syncthreads();
  for (int s = m.col_ptr[c0] + threadIdx.x; s < m.col_ptr[c0 + nc]; s += blockDim.x)
    sidx[(m.st_hx[s] - c0) * n2 + m.st_i2[s]] = s;
  __syncthreads();
  const cpx<T>* st = sticks + ((size_t)band * m.n3 + z) * m.ldst;
  cpx<T>* out = rows + ((size_t)band * m.n3 + z) * n2 * nxr + c0;
  fft_run<T>(
      m.f2, nc, T(1), tw2, A, B, lmax, false, true,
      [&](int b, int i) {
        const int s = sidx[b * n2 + i];
        return s >= 0 ? st[s] : cpx<T>{T(0), T(0)};
      },
      [&](int b, int i, cpx<T> v) { out[(size_t)i * nxr + b] = v; });
}

// rows [r0, r0+CB) of one plane: inverse x, times V(r), forward x; the x
// columns of the sphere are read and written back in place
template <typename T>
__global__ void __launch_bounds__(SPLIT_THREADS)
k_plane_x(SphereMap m, cpx<T>* __restrict__ rows, const T* __restrict__ vr, const cpx<T>* __restrict__ tw1) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n1 = m.n1, n2 = m.n2, nxr = m.nxr, lmax = max(n1, n2);
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* B = A + SPLIT_CB * lmax;
  int* hx_of = reinterpret_cast<int*>(B + SPLIT_CB * lmax) + SPLIT_CB * n2;   // [n1]
  const int z = blockIdx.x, band = blockIdx.y, r0 = blockIdx.z * SPLIT_CB;
  const int nr = min(SPLIT_CB, n2 - r0);
  for (int i = threadIdx.x; i < n1; i += blockDim.x) hx_of[i] = m.i1_hx[i];
  __syncthreads();
  cpx<T>* rw = rows + (((size_t)band * m.n3 + z) * n2 + r0) * nxr;
  const T* vz = vr + ((size_t)z * n2 + r0) * n1;
  const int lr = fft_last_read(m.f1);
  cpx<T>* X = (lr == 0) ? B : A;
  cpx<T>* P0 = (X == A) ? B : A;
  fft_run<T>(
      m.f1, nr, T(1), tw1, A, B, lmax, false, false,
      [&](int b, int i) {
        const int hx = hx_of[i];
        return hx >= 0 ? rw[(size_t)b * nxr + hx] : cpx<T>{T(0), T(0)};
      },
      [&](int b, int i, cpx<T> v) { X[b * lmax + i] = v * vz[(size_t)b * n1 + i]; });
  fft_run<T>(
      m.f1, nr, T(-1), tw1, P0, X, lmax, false, false,
      [&](int b, int i) { return X[b * lmax + i]; },
      [&](int b, int i, cpx<T> v) {
        const int hx = hx_of[i];
        if (hx >= 0) rw[(size_t)b * nxr + hx] = v;
      });
}

// rows -> forward y of x columns [c0, c0+CB) -> stick positions only
template <typename T>
__global__ void __launch_bounds__(SPLIT_THREADS)
k_plane_yfwd(SphereMap m, cpx<T>* __restrict__ sticks, const cpx<T>* __restrict__ rows,
             const cpx<T>* __restrict__ tw2) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n2 = m.n2, nxr = m.nxr, lmax = max(m.n1, n2);
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* B = A + SPLIT_CB * lmax;
  int* sidx = reinterpret_cast<int*>(B + SPLIT_CB * lmax);
  const int z = blockIdx.x, band = blockIdx.y, c0 = blockIdx.z * SPLIT_CB;
  const int nc = min(SPLIT_CB, nxr - c0);
  for (int i = threadIdx.x; i < SPLIT_CB * n2; i += blockDim.x) sidx[i] = -1;
  __syncthreads();
  for (int s = m.col_ptr[c0] + threadIdx.x; s < m.col_ptr[c0 + nc]; s += blockDim.x)
    sidx[(m.st_hx[s] - c0) * n2 + m.st_i2[s]] = s;
  __syncthreads();
  cpx<T>* st = sticks + ((size_t)band * m.n3 + z) * m.ldst;
  const cpx<T>* in = rows + ((size_t)band * m.n3 + z) * n2 * nxr + c0;
  fft_run<T>(
      m.f2, nc, T(-1), tw2, A, B, lmax, true, false,
      [&](int b, int i) { return in[(size_t)i * nxr + b]; },
      [&](int b, int i, cpx<T> v) {
        const int s = sidx[b * n2 + i];
        if (s >= 0) st[s] = v;
      });
}

template <typename T>
using PlaneRegFn = void (*)(SphereMap, cpx<T>*, const T*, const cpx<T>*, const cpx<T>*);

// register-resident plane kernel for n1 = n2 = 4 LS with PP z planes per
// workgroup, or nullptr
template <typename T, int PP>
PlaneRegFn<T> plane_reg_kernel(int n1, int n2) {
  if (n1 != n2 || n1 % 4 != 0) return nullptr;
  const int ls = n1 / 4;
  const bool f64 = sizeof(T) == 8;
  switch (ls) {
    case 8: return k_plane_reg<T, 8, PP>;
    case 9: return k_plane_reg<T, 9, PP>;
    case 10: return k_plane_reg<T, 10, PP>;
    case 12: return k_plane_reg<T, 12, PP>;
    case 15: return k_plane_reg<T, 15, PP>;
    case 16: return k_plane_reg<T, 16, PP>;
    case 18: return k_plane_reg<T, 18, PP>;
    case 20: return f64 ? nullptr : k_plane_reg<T, 20, PP>;
    case 24: return f64 ? nullptr : k_plane_reg<T, 24, PP>;
    case 25: return f64 ? nullptr : k_plane_reg<T, 25, PP>;
    case 27: return f64 ? nullptr : k_plane_reg<T, 27, PP>;
    case 30: return f64 ? nullptr : k_plane_reg<T, 30, PP>;
    case 32: return f64 ? nullptr : k_plane_reg<T, 32, PP>;
    case 36: return f64 ? nullptr : k_plane_reg<T, 36, PP>;
    default: return nullptr;
  }
}

// largest LDS of the two-plane register kernel: two workgroups per CU (160 KB)
constexpr size_t kPlaneRegMaxLds = 80 * 1024;
// largest LDS of the one-plane register kernel (static LDS of the kernel is nil)
constexpr size_t kPlaneRegMaxLds1 = 156 * 1024;

// raise a kernel's dynamic LDS limit (above the default 64 KB) once per kernel
pw_status raise_lds_limit(const void* fn, int bytes) {
  static std::mutex mu;
  static std::map<const void*, int> raised;
  std::lock_guard<std::mutex> lk(mu);
  auto it = raised.find(fn);
  if (it != raised.end() && it->second >= bytes) return PW_OK;
  PW_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  raised[fn] = bytes;
  return PW_OK;
}

template <typename T>
size_t plane_reg_lds_bytes(int n, int nxr, int pp) {
  return sizeof(cpx<T>) * (2 * (size_t)n + (size_t)pp * nxr * (n + 1)) + sizeof(int) * (size_t)n;
}

// float64 transforms use ~240 VGPRs (2 waves per SIMD): 256-thread groups
// keep two planes in flight per CU; float32 ones use up to a full quad per row
template <typename T>
int plane_reg_threads(int n, int nxr) {
  const int need = 4 * std::max(n, nxr);
  const int cap = sizeof(T) == 8 ? 256 : 512;
  return std::min(cap, (need + 63) / 64 * 64);
}

// the register (quad) plane kernel exists for this grid and its LDS fits
template <typename T>
bool plane_quad_fits(int n1, int n2, int nxr) {
  if (plane_reg_kernel<T, 2>(n1, n2) != nullptr && plane_reg_lds_bytes<T>(n1, nxr, 2) <= kPlaneRegMaxLds) return true;
  return plane_reg_kernel<T, 1>(n1, n2) != nullptr && plane_reg_lds_bytes<T>(n1, nxr, 1) <= kPlaneRegMaxLds1;
}

// ---------------------------------------------------------------------------
// pass 3: forward z transform, gather to the sphere, kinetic term
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(ZTHREADS)
k_zfwd(SphereMap m, const cpx<T>* __restrict__ sticks,
       const c128* __restrict__ psi, int ldpsi, c128* __restrict__ hpsi, int ldhpsi,
       const cpx<T>* __restrict__ twg, double inv_n, int accumulate, int gz, int nb) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n3 = m.n3;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = tw + n3;
  cpx<T>* B = A + ZSB * n3;
  int chunk, band;
  if (!z_tile(gz, nb, chunk, band)) return;
  const int s0 = chunk * ZSB;
  const int ns = min(ZSB, m.nst - s0);
  for (int i = threadIdx.x; i < n3; i += blockDim.x) tw[i] = twg[i];
  __syncthreads();
  const cpx<T>* in = sticks + (size_t)band * n3 * m.ldst + s0;
  const int ldst = m.ldst;
  const int lr = fft_last_read(m.f3);
  cpx<T>* X = (lr == 0) ? B : A;
  fft_run<T>(
      m.f3, ns, T(-1), tw, A, B, n3, true, false,
      [&](int b, int i) { return in[(size_t)i * ldst + b]; },
      [&](int b, int i, cpx<T> v) { X[b * n3 + i] = v; });
  const c128* pb = psi + (size_t)band * ldpsi;
  c128* hb = hpsi + (size_t)band * ldhpsi;
  const int e0 = m.st_ptr[s0], e1 = m.st_ptr[s0 + ns];
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int g = m.ent_g[e];
    const cpx<T> v = X[(m.ent_s[e] - s0) * n3 + m.ent_z[e]];
    c128 r = c128{(double)v.x * inv_n, (double)v.y * inv_n};
    if (!(accumulate & 2)) {   // kinetic term (not yet in hpsi)
      const c128 p = pb[g];
      const double t = m.kin[g];
      r = c128{r.x + t * p.x, r.y + t * p.y};
    }
    if (accumulate & 1) {   // the projector term is already in hpsi
      const c128 o = hb[g];
      r = c128{r.x + o.x, r.y + o.y};
    }
    hb[g] = r;
  }
}

// ---------------------------------------------------------------------------
// z passes, register-resident variant for n3 = 4 LS: one quad of lanes per
// stick holds the whole column in VGPRs (see fft_reg.h); no LDS staging.
// The (z, stick) -> sphere index map gives every lane its gather and scatter
// positions directly, zero where the column leaves the sphere.
// ---------------------------------------------------------------------------
constexpr int ZRTHREADS = 128;
constexpr int ZRSTICKS = ZRTHREADS / 4;   // sticks per workgroup

template <typename T, int LS>
__global__ void __launch_bounds__(ZRTHREADS)
k_zinv_reg(SphereMap m, const c128* __restrict__ psi, int ldpsi, cpx<T>* __restrict__ sticks,
           const cpx<T>* __restrict__ twg, int gz, int nb) {
  constexpr int N3 = 4 * LS;
  __shared__ cpx<T> tw[N3];
  int chunk, band;
  if (!z_tile(gz, nb, chunk, band)) return;
  for (int i = threadIdx.x; i < N3; i += blockDim.x) tw[i] = twg[i];
  __syncthreads();
  const int s = chunk * ZRSTICKS + (threadIdx.x >> 2);
  if (s >= m.nst) return;   // the whole quad of the stick leaves together
  const int q = threadIdx.x & 3, nst = m.nst;
  const c128* pb = psi + (size_t)band * ldpsi;
  cpx<T> x[LS];
#pragma unroll
  for (int j = 0; j < LS; ++j) {
    const int g = m.zidx[(size_t)(q + 4 * j) * nst + s];
    x[j] = g >= 0 ? to_t<T>(pb[g]) : cpx<T>{T(0), T(0)};
  }
  const regfft::QuadLane<T> ql = regfft::quad_lane<T>(q);
  regfft::inv_dit<LS, T>(x, q, ql, tw);
  const int blk = regfft::quad_block(q);
  cpx<T>* out = sticks + (size_t)band * N3 * m.ldst + s;
#pragma unroll
  for (int k = 0; k < LS; ++k) out[(size_t)(k + LS * blk) * m.ldst] = x[k];
}

template <typename T, int LS>
__global__ void __launch_bounds__(ZRTHREADS)
k_zfwd_reg(SphereMap m, const cpx<T>* __restrict__ sticks, const c128* __restrict__ psi, int ldpsi,
           c128* __restrict__ hpsi, int ldhpsi, const cpx<T>* __restrict__ twg, double inv_n,
           int accumulate, int gz, int nb) {
  constexpr int N3 = 4 * LS, XS = N3 + 1;   // padded stick stride of the LDS copy
  __shared__ cpx<T> tw[N3];
  __shared__ cpx<T> X[ZRSTICKS * XS];
  int chunk, band;
  if (!z_tile(gz, nb, chunk, band)) return;
  for (int i = threadIdx.x; i < N3; i += blockDim.x) tw[i] = twg[i];
  __syncthreads();
  const int s0 = chunk * ZRSTICKS, sl = threadIdx.x >> 2, s = s0 + sl;
  const int q = threadIdx.x & 3;
  if (s < m.nst) {
    const int blk = regfft::quad_block(q);
    const cpx<T>* in = sticks + (size_t)band * N3 * m.ldst + s;
    cpx<T> x[LS];
#pragma unroll
    for (int k = 0; k < LS; ++k) x[k] = in[(size_t)(k + LS * blk) * m.ldst];
    const regfft::QuadLane<T> ql = regfft::quad_lane<T>(q);
    regfft::fwd_dif<LS, T>(x, q, ql, tw);
#pragma unroll
    for (int j = 0; j < LS; ++j) X[sl * XS + q + 4 * j] = x[j];
  }
  __syncthreads();
  // the chunk's sphere entries in stick order: coalesced index reads
  const c128* pb = psi + (size_t)band * ldpsi;
  c128* hb = hpsi + (size_t)band * ldhpsi;
  const int e0 = m.st_ptr[s0], e1 = m.st_ptr[min(s0 + ZRSTICKS, m.nst)];
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int g = m.ent_g[e];
    const cpx<T> v = X[(m.ent_s[e] - s0) * XS + m.ent_z[e]];
    c128 r = c128{(double)v.x * inv_n, (double)v.y * inv_n};
    if (!(accumulate & 2)) {   // kinetic term (not yet in hpsi)
      const c128 p = pb[g];
      const double t = m.kin[g];
      r = c128{r.x + t * p.x, r.y + t * p.y};
    }
    if (accumulate & 1) {   // the projector term is already in hpsi
      const c128 o = hb[g];
      r = c128{r.x + o.x, r.y + o.y};
    }
    hb[g] = r;
  }
}

// ---------------------------------------------------------------------------
// z passes on 16-lane groups for n3 = 16 LS (float64 columns too long for a
// quad of lanes to hold in registers, e.g. n3 = 144): one group of 16 lanes
// per stick, LS points per lane, the same transform as the lane-group plane
// kernel; twiddles from global memory.
// ---------------------------------------------------------------------------
constexpr int ZGTHREADS = 256;
constexpr int ZGSTICKS = ZGTHREADS / 16;   // sticks per workgroup

template <typename T, int LS>
__global__ void __launch_bounds__(ZGTHREADS)
k_zinv_grp(SphereMap m, const c128* __restrict__ psi, int ldpsi, cpx<T>* __restrict__ sticks,
           const cpx<T>* __restrict__ tw, int gz, int nb) {
  constexpr int G = 16, N3 = G * LS;
  int chunk, band;
  if (!z_tile(gz, nb, chunk, band)) return;
  const int s = chunk * ZGSTICKS + (threadIdx.x >> 4);
  if (s >= m.nst) return;   // the whole group of the stick leaves together
  const int g = threadIdx.x & (G - 1), nst = m.nst;
  const c128* pb = psi + (size_t)band * ldpsi;
  cpx<T> x[LS];
#pragma unroll
  for (int j = 0; j < LS; ++j) {
    const int e = m.zidx[(size_t)(g + G * j) * nst + s];
    x[j] = e >= 0 ? to_t<T>(pb[e]) : cpx<T>{T(0), T(0)};
  }
  const regfft::GLane<T> gl = regfft::glane<T>(g);
  regfft::ginv<G, LS, T>(x, g, gl, tw);
  const int blk = regfft::g_block<G>(g);
  cpx<T>* out = sticks + (size_t)band * N3 * m.ldst + s;
#pragma unroll
  for (int k = 0; k < LS; ++k) out[(size_t)(k + LS * blk) * m.ldst] = x[k];
}

template <typename T, int LS>
__global__ void __launch_bounds__(ZGTHREADS)
k_zfwd_grp(SphereMap m, const cpx<T>* __restrict__ sticks, const c128* __restrict__ psi, int ldpsi,
           c128* __restrict__ hpsi, int ldhpsi, const cpx<T>* __restrict__ tw, double inv_n,
           int accumulate, int gz, int nb) {
  constexpr int G = 16, N3 = G * LS, XS = N3 + 1;   // padded stick stride of the LDS copy
  __shared__ cpx<T> X[ZGSTICKS * XS];
  int chunk, band;
  if (!z_tile(gz, nb, chunk, band)) return;
  const int s0 = chunk * ZGSTICKS, sl = threadIdx.x >> 4, s = s0 + sl;
  const int g = threadIdx.x & (G - 1);
  if (s < m.nst) {
    const int blk = regfft::g_block<G>(g);
    const cpx<T>* in = sticks + (size_t)band * N3 * m.ldst + s;
    cpx<T> x[LS];
#pragma unroll
    for (int k = 0; k < LS; ++k) x[k] = in[(size_t)(k + LS * blk) * m.ldst];
    const regfft::GLane<T> gl = regfft::glane<T>(g);
    regfft::gfwd<G, LS, T>(x, g, gl, tw);
#pragma unroll
    for (int j = 0; j < LS; ++j) X[sl * XS + g + G * j] = x[j];
  }
  __syncthreads();
  // the chunk's sphere entries in stick order: coalesced index reads
  const c128* pb = psi + (size_t)band * ldpsi;
  c128* hb = hpsi + (size_t)band * ldhpsi;
  const int e0 = m.st_ptr[s0], e1 = m.st_ptr[min(s0 + ZGSTICKS, m.nst)];
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int gi = m.ent_g[e];
    const cpx<T> v = X[(m.ent_s[e] - s0) * XS + m.ent_z[e]];
    c128 r = c128{(double)v.x * inv_n, (double)v.y * inv_n};
    if (!(accumulate & 2)) {   // kinetic term (not yet in hpsi)
      const c128 p = pb[gi];
      const double t = m.kin[gi];
      r = c128{r.x + t * p.x, r.y + t * p.y};
    }
    if (accumulate & 1) {   // the projector and kinetic terms are already in hpsi
      const c128 o = hb[gi];
      r = c128{r.x + o.x, r.y + o.y};
    }
    hb[gi] = r;
  }
}

// ---------------------------------------------------------------------------
// Gamma point (real wavefunctions on the half sphere): bands a = 2t and
// b = 2t + 1 share transform t.  The inverse z pass packs a + i b onto the
// sticks of the whole sphere (conj(a) + i conj(b) at the mirror -G), so the
// real-space grid holds psi_a(r) + i psi_b(r); after V(r) and the forward
// transform f(G) = (V psi_a)(G) + i (V psi_b)(G), and the gather separates
// (V psi_a)(G) = (f(G) + conj f(-G)) / 2, (V psi_b)(G) = (f(G) - conj f(-G)) / 2i.
// ---------------------------------------------------------------------------
__device__ __forceinline__ c128 gamma_pack(const c128* __restrict__ pa, const c128* __restrict__ pb, int enc) {
  const int g = enc >> 1;
  c128 a = pa[g];
  c128 b = pb ? pb[g] : c128{0.0, 0.0};
  if (g == 0) { a.y = 0.0; b.y = 0.0; }   // psi(0) is real
  return (enc & 1) ? c128{a.x + b.y, b.x - a.y} : c128{a.x - b.y, a.y + b.x};
}

template <typename T, int LS>
__global__ void __launch_bounds__(ZRTHREADS)
k_zinv_reg_g(SphereMap m, const c128* __restrict__ psi, int ldpsi, cpx<T>* __restrict__ sticks,
             const cpx<T>* __restrict__ twg, int gz, int npair, int nbands) {
  constexpr int N3 = 4 * LS;
  __shared__ cpx<T> tw[N3];
  int chunk, pair;
  if (!z_tile(gz, npair, chunk, pair)) return;
  for (int i = threadIdx.x; i < N3; i += blockDim.x) tw[i] = twg[i];
  __syncthreads();
  const int s = chunk * ZRSTICKS + (threadIdx.x >> 2);
  if (s >= m.nst) return;
  const int q = threadIdx.x & 3, nst = m.nst;
  const c128* pa = psi + (size_t)(2 * pair) * ldpsi;
  const c128* pb = 2 * pair + 1 < nbands ? pa + ldpsi : nullptr;
  cpx<T> x[LS];
#pragma unroll
  for (int j = 0; j < LS; ++j) {
    const int enc = m.zidx[(size_t)(q + 4 * j) * nst + s];
    x[j] = enc >= 0 ? to_t<T>(gamma_pack(pa, pb, enc)) : cpx<T>{T(0), T(0)};
  }
  const regfft::QuadLane<T> ql = regfft::quad_lane<T>(q);
  regfft::inv_dit<LS, T>(x, q, ql, tw);
  const int blk = regfft::quad_block(q);
  cpx<T>* out = sticks + (size_t)pair * N3 * m.ldst + s;
#pragma unroll
  for (int k = 0; k < LS; ++k) out[(size_t)(k + LS * blk) * m.ldst] = x[k];
}

// forward z transform of each stick, in place (the gather follows)
template <typename T, int LS>
__global__ void __launch_bounds__(ZRTHREADS)
k_zfwd_reg_g(SphereMap m, cpx<T>* __restrict__ sticks, const cpx<T>* __restrict__ twg, int gz, int npair) {
  constexpr int N3 = 4 * LS;
  __shared__ cpx<T> tw[N3];
  int chunk, pair;
  if (!z_tile(gz, npair, chunk, pair)) return;
  for (int i = threadIdx.x; i < N3; i += blockDim.x) tw[i] = twg[i];
  __syncthreads();
  const int s = chunk * ZRSTICKS + (threadIdx.x >> 2);
  if (s >= m.nst) return;
  const int q = threadIdx.x & 3;
  const int blk = regfft::quad_block(q);
  cpx<T>* io = sticks + (size_t)pair * N3 * m.ldst + s;
  cpx<T> x[LS];
#pragma unroll
  for (int k = 0; k < LS; ++k) x[k] = io[(size_t)(k + LS * blk) * m.ldst];
  const regfft::QuadLane<T> ql = regfft::quad_lane<T>(q);
  regfft::fwd_dif<LS, T>(x, q, ql, tw);
#pragma unroll
  for (int j = 0; j < LS; ++j) io[(size_t)(q + 4 * j) * m.ldst] = x[j];
}

// LDS Stockham forms of the two Gamma z passes (other lengths)
template <typename T>
__global__ void __launch_bounds__(ZTHREADS)
k_zinv_g(SphereMap m, const c128* __restrict__ psi, int ldpsi, cpx<T>* __restrict__ sticks,
         const cpx<T>* __restrict__ twg, int gz, int npair, int nbands) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n3 = m.n3;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = tw + n3;
  cpx<T>* B = A + ZSB * n3;
  int chunk, pair;
  if (!z_tile(gz, npair, chunk, pair)) return;
  const int s0 = chunk * ZSB;
  const int ns = min(ZSB, m.nst - s0);
  const c128* pa = psi + (size_t)(2 * pair) * ldpsi;
  const c128* pb = 2 * pair + 1 < nbands ? pa + ldpsi : nullptr;
  for (int i = threadIdx.x; i < n3; i += blockDim.x) tw[i] = twg[i];
  for (int i = threadIdx.x; i < ZSB * n3; i += blockDim.x) B[i] = cpx<T>{T(0), T(0)};
  __syncthreads();
  const int e0 = m.st_ptr[s0], e1 = m.st_ptr[s0 + ns];
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x)
    B[(m.ent_s[e] - s0) * n3 + m.ent_z[e]] = to_t<T>(gamma_pack(pa, pb, m.ent_g[e]));
  __syncthreads();
  cpx<T>* out = sticks + (size_t)pair * n3 * m.ldst + s0;
  const int ldst = m.ldst;
  fft_run<T>(
      m.f3, ns, T(1), tw, A, B, n3, false, true,
      [&](int b, int i) { return B[b * n3 + i]; },
      [&](int b, int i, cpx<T> v) { out[(size_t)i * ldst + b] = v; });
}

template <typename T>
__global__ void __launch_bounds__(ZTHREADS)
k_zfwd_g(SphereMap m, cpx<T>* __restrict__ sticks, const cpx<T>* __restrict__ twg, int gz, int npair) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n3 = m.n3;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = tw + n3;
  cpx<T>* B = A + ZSB * n3;
  int chunk, pair;
  if (!z_tile(gz, npair, chunk, pair)) return;
  const int s0 = chunk * ZSB;
  const int ns = min(ZSB, m.nst - s0);
  for (int i = threadIdx.x; i < n3; i += blockDim.x) tw[i] = twg[i];
  __syncthreads();
  cpx<T>* io = sticks + (size_t)pair * n3 * m.ldst + s0;
  const int ldst = m.ldst;
  fft_run<T>(
      m.f3, ns, T(-1), tw, A, B, n3, true, true,
      [&](int b, int i) { return io[(size_t)i * ldst + b]; },
      [&](int b, int i, cpx<T> v) { io[(size_t)i * ldst + b] = v; });
}

// H psi(G) for the half sphere: kinetic + the separated local terms of the
// two bands of each transform (+ the projector term already in hpsi)
template <typename T>
__global__ void __launch_bounds__(256)
k_gamma_gather(int npw, const int* __restrict__ gpos_p, const int* __restrict__ gpos_m,
               const cpx<T>* __restrict__ sticks, size_t pair_stride, const double* __restrict__ kin,
               const c128* __restrict__ psi, int ldpsi, c128* __restrict__ hpsi, int ldhpsi, double inv_n,
               int accumulate, int nbands) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int pair = blockIdx.y;
  if (g >= npw) return;
  const cpx<T>* st = sticks + (size_t)pair * pair_stride;
  const cpx<T> fp = st[gpos_p[g]], fm = st[gpos_m[g]];
  const double f1x = (double)fp.x, f1y = (double)fp.y, f2x = (double)fm.x, f2y = -(double)fm.y;   // f(G), conj f(-G)
  // (f1 + f2) / 2 and (f1 - f2) / (2 i)
  double va_x = 0.5 * (f1x + f2x), va_y = 0.5 * (f1y + f2y);
  double vb_x = 0.5 * (f1y - f2y), vb_y = -0.5 * (f1x - f2x);
  if (g == 0) { va_y = 0.0; vb_y = 0.0; }
  const double t = kin[g];
  for (int h = 0; h < 2; ++h) {
    const int band = 2 * pair + h;
    if (band >= nbands) break;
    const c128 p = psi[(size_t)band * ldpsi + g];
    const double px = p.x, py = g == 0 ? 0.0 : p.y;
    c128 r = h == 0 ? c128{t * px + va_x * inv_n, t * py + va_y * inv_n}
                    : c128{t * px + vb_x * inv_n, t * py + vb_y * inv_n};
    c128* o = hpsi + (size_t)band * ldhpsi + g;
    if (accumulate) r = c128{r.x + o->x, r.y + o->y};
    *o = r;
  }
}

// Gamma z passes on 16-lane groups (n3 = 16 LS, float64 beyond the quad form)
template <typename T, int LS>
__global__ void __launch_bounds__(ZGTHREADS)
k_zinv_grp_g(SphereMap m, const c128* __restrict__ psi, int ldpsi, cpx<T>* __restrict__ sticks,
             const cpx<T>* __restrict__ tw, int gz, int npair, int nbands) {
  constexpr int G = 16, N3 = G * LS;
  int chunk, pair;
  if (!z_tile(gz, npair, chunk, pair)) return;
  const int s = chunk * ZGSTICKS + (threadIdx.x >> 4);
  if (s >= m.nst) return;
  const int g = threadIdx.x & (G - 1), nst = m.nst;
  const c128* pa = psi + (size_t)(2 * pair) * ldpsi;
  const c128* pb = 2 * pair + 1 < nbands ? pa + ldpsi : nullptr;
  cpx<T> x[LS];
#pragma unroll
  for (int j = 0; j < LS; ++j) {
    const int enc = m.zidx[(size_t)(g + G * j) * nst + s];
    x[j] = enc >= 0 ? to_t<T>(gamma_pack(pa, pb, enc)) : cpx<T>{T(0), T(0)};
  }
  const regfft::GLane<T> gl = regfft::glane<T>(g);
  regfft::ginv<G, LS, T>(x, g, gl, tw);
  const int blk = regfft::g_block<G>(g);
  cpx<T>* out = sticks + (size_t)pair * N3 * m.ldst + s;
#pragma unroll
  for (int k = 0; k < LS; ++k) out[(size_t)(k + LS * blk) * m.ldst] = x[k];
}

template <typename T, int LS>
__global__ void __launch_bounds__(ZGTHREADS)
k_zfwd_grp_g(SphereMap m, cpx<T>* __restrict__ sticks, const cpx<T>* __restrict__ tw, int gz, int npair) {
  constexpr int G = 16, N3 = G * LS;
  int chunk, pair;
  if (!z_tile(gz, npair, chunk, pair)) return;
  const int s = chunk * ZGSTICKS + (threadIdx.x >> 4);
  if (s >= m.nst) return;
  const int g = threadIdx.x & (G - 1);
  const int blk = regfft::g_block<G>(g);
  cpx<T>* io = sticks + (size_t)pair * N3 * m.ldst + s;
  cpx<T> x[LS];
#pragma unroll
  for (int k = 0; k < LS; ++k) x[k] = io[(size_t)(k + LS * blk) * m.ldst];
  const regfft::GLane<T> gl = regfft::glane<T>(g);
  regfft::gfwd<G, LS, T>(x, g, gl, tw);
#pragma unroll
  for (int j = 0; j < LS; ++j) io[(size_t)(g + G * j) * m.ldst] = x[j];
}

template <typename T>
struct ZGrpFns {
  void (*inv)(SphereMap, const c128*, int, cpx<T>*, const cpx<T>*, int, int) = nullptr;
  void (*fwd)(SphereMap, const cpx<T>*, const c128*, int, c128*, int, const cpx<T>*, double, int, int, int) = nullptr;
  void (*inv_g)(SphereMap, const c128*, int, cpx<T>*, const cpx<T>*, int, int, int) = nullptr;
  void (*fwd_g)(SphereMap, cpx<T>*, const cpx<T>*, int, int) = nullptr;
};
template <typename T, int LS>
ZGrpFns<T> zgrp_set() {
  ZGrpFns<T> f;
  f.inv = k_zinv_grp<T, LS>;
  f.fwd = k_zfwd_grp<T, LS>;
  f.inv_g = k_zinv_grp_g<T, LS>;
  f.fwd_g = k_zfwd_grp_g<T, LS>;
  return f;
}

// 16-lane-group z passes for n3 = 16 LS, or none
template <typename T>
ZGrpFns<T> zgrp_kernels(int n3) {
  switch (n3) {
    case 80: return zgrp_set<T, 5>();
    case 96: return zgrp_set<T, 6>();
    case 128: return zgrp_set<T, 8>();
    case 144: return zgrp_set<T, 9>();
    default: return ZGrpFns<T>{};
  }
}

template <typename T>
struct ZRegFns {
  void (*inv)(SphereMap, const c128*, int, cpx<T>*, const cpx<T>*, int, int) = nullptr;
  void (*fwd)(SphereMap, const cpx<T>*, const c128*, int, c128*, int, const cpx<T>*, double, int, int, int) = nullptr;
  void (*inv_g)(SphereMap, const c128*, int, cpx<T>*, const cpx<T>*, int, int, int) = nullptr;
  void (*fwd_g)(SphereMap, cpx<T>*, const cpx<T>*, int, int) = nullptr;
};

template <typename T, int LS>
ZRegFns<T> zreg_pair() {
  ZRegFns<T> f;
  f.inv = k_zinv_reg<T, LS>;
  f.fwd = k_zfwd_reg<T, LS>;
  f.inv_g = k_zinv_reg_g<T, LS>;
  f.fwd_g = k_zfwd_reg_g<T, LS>;
  return f;
}

// register-resident z passes for n3 = 4 LS (same lengths as the plane pass)
template <typename T>
ZRegFns<T> zreg_kernels(int n3) {
  if (n3 % 4 != 0) return {};
  const bool f64 = sizeof(T) == 8;
  switch (n3 / 4) {
    case 8: return zreg_pair<T, 8>();
    case 9: return zreg_pair<T, 9>();
    case 10: return zreg_pair<T, 10>();
    case 12: return zreg_pair<T, 12>();
    case 15: return zreg_pair<T, 15>();
    case 16: return zreg_pair<T, 16>();
    case 18: return zreg_pair<T, 18>();
    case 20: return f64 ? ZRegFns<T>{} : zreg_pair<T, 20>();
    case 24: return f64 ? ZRegFns<T>{} : zreg_pair<T, 24>();
    case 25: return f64 ? ZRegFns<T>{} : zreg_pair<T, 25>();
    case 27: return f64 ? ZRegFns<T>{} : zreg_pair<T, 27>();
    case 30: return f64 ? ZRegFns<T>{} : zreg_pair<T, 30>();
    case 32: return f64 ? ZRegFns<T>{} : zreg_pair<T, 32>();
    case 36: return f64 ? ZRegFns<T>{} : zreg_pair<T, 36>();
    default: return {};
  }
}

// ---------------------------------------------------------------------------
// plan-time helpers
// ---------------------------------------------------------------------------
__global__ void k_f64_to_f32(const double* __restrict__ a, float* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

// diag of the projector term: sum_{ij in blocks} beta_i(G) D_ij conj(beta_j(G))
__global__ void k_hdiag(int npw, int nbeta, const c128* __restrict__ beta, int ldb,
                        const int* __restrict__ dstart, const int* __restrict__ dlen,
                        const c128* __restrict__ drow, int nhmax, const double* __restrict__ kin,
                        double v0, double* __restrict__ hdiag) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  double acc = 0.0;
  for (int i = 0; i < nbeta; ++i) {
    const c128 bi = beta[(size_t)i * ldb + g];
    const int j0 = dstart[i], nh = dlen[i];
    for (int t = 0; t < nh; ++t) {
      const c128 d = drow[(size_t)i * nhmax + t];
      const c128 bj = beta[(size_t)(j0 + t) * ldb + g];
      // Re( beta_i D_ij conj(beta_j) )
      const c128 dbj = c128{d.x * bj.x + d.y * bj.y, d.y * bj.x - d.x * bj.y};  // D_ij conj(bj)
      acc += bi.x * dbj.x - bi.y * dbj.y;
    }
  }
  hdiag[g] = (kin ? kin[g] : 0.0) + v0 + acc;
}

template <typename T>
size_t plane_lds_bytes(int n1, int n2, int nxr, int cb) {
  const int lmax = std::max(n1, n2);
  return sizeof(cpx<T>) * ((size_t)n1 + n2 + (size_t)nxr * n2 + 2 * (size_t)cb * lmax) +
         sizeof(int) * (size_t)n1;
}

// largest column/row batch whose plane pass fits the LDS budget
template <typename T>
int plane_batch(int n1, int n2, int nxr) {
  const size_t budget = 156 * 1024;
  for (int cb : {16, 12, 8, 6, 4, 2, 1})
    if (plane_lds_bytes<T>(n1, n2, nxr, cb) <= budget) return cb;
  return 0;
}

// Forms of the plane pass (pw_plan_info reports them).
enum PlaneForm { kFormQuad = 0, kFormSplit = 1, kFormGroup = 2, kFormLds = 3 };

template <typename T>
bool plane_form_ok(int form, int n1, int n2, int nxr) {
  switch (form) {
    case kFormQuad: return plane_quad_fits<T>(n1, n2, nxr);
    case kFormGroup: return plane_oct_fits<T>(n1, n2, nxr);
    case kFormLds: return plane_batch<T>(n1, n2, nxr) > 0;
    default: return true;   // three kernels fit any grid the plan accepts
  }
}

// Form chosen without measurement: plane_mode 1 takes three kernels; 2 the
// lane-group kernel where it applies; 4 the register kernel where it
// applies; 0 (and 3, before its measurement, and 2 and 4 elsewhere) the
// register (quad) kernel where two planes fit a workgroup, else the
// lane-group kernel, else the register kernel with one plane per workgroup,
// else the generic LDS kernel, else three kernels.  (At 144^2 in float32 the
// lane-group kernel runs two workgroups per CU where the one-plane register
// kernel runs one: 12.5 against 18.4 ms per 1024-band H.psi.)
template <typename T>
int plane_form_for(int mode, int n1, int n2, int nxr) {
  if (mode == 1) return kFormSplit;
  if (mode == 2 && plane_form_ok<T>(kFormGroup, n1, n2, nxr)) return kFormGroup;
  if (mode == 4 && plane_form_ok<T>(kFormQuad, n1, n2, nxr)) return kFormQuad;
  if (plane_reg_kernel<T, 2>(n1, n2) != nullptr && plane_reg_lds_bytes<T>(n1, nxr, 2) <= kPlaneRegMaxLds)
    return kFormQuad;
  for (int f : {(int)kFormGroup, (int)kFormQuad, (int)kFormLds})
    if (plane_form_ok<T>(f, n1, n2, nxr)) return f;
  return kFormSplit;
}


template <typename T>
size_t z_lds_bytes(int n3) { return sizeof(cpx<T>) * ((size_t)n3 + 2 * (size_t)ZSB * n3); }

template <typename T>
pw_status set_lds_limit(const void* fn) {
  hipFuncAttributes at;
  PW_HIP(hipFuncGetAttributes(&at, fn));
  PW_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)at.sharedSizeBytes));
  return PW_OK;
}

template <typename T>
pw_status set_lds_limits() {
  static bool done = false;
  if (done) return PW_OK;
  PW_TRY(set_lds_limit<T>((const void*)k_plane<T>));
  PW_TRY(set_lds_limit<T>((const void*)k_zinv<T>));
  PW_TRY(set_lds_limit<T>((const void*)k_zfwd<T>));
  PW_TRY(set_lds_limit<T>((const void*)k_zinv_g<T>));
  PW_TRY(set_lds_limit<T>((const void*)k_zfwd_g<T>));
  PW_TRY(set_lds_limit<T>((const void*)k_plane_yinv<T>));
  PW_TRY(set_lds_limit<T>((const void*)k_plane_x<T>));
  PW_TRY(set_lds_limit<T>((const void*)k_plane_yfwd<T>));
  done = true;
  return PW_OK;
}

template <typename X>
pw_status dalloc(pw_plan p, X** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return PW_OK;
  void* q = nullptr;
  PW_TRY(pw::dev_alloc(p, count * sizeof(X), &q));
  p->allocs.push_back(q);
  *ptr = static_cast<X*>(q);
  return PW_OK;
}

template <typename X>
pw_status upload(pw_plan p, X** ptr, const std::vector<X>& v) {
  PW_TRY(dalloc(p, ptr, v.size()));
  if (v.empty()) return PW_OK;
  if (p->pool) {
    // on the plan's set-up stream only (a served plan never waits on the device)
    PW_HIP(hipMemcpyAsync(*ptr, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice, p->init_stream));
    PW_HIP(hipStreamSynchronize(p->init_stream));
  } else {
    PW_HIP(hipMemcpy(*ptr, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice));
  }
  return PW_OK;
}

void twiddles(int L, std::vector<c128>& t64, std::vector<c64>& t32) {
  t64.resize(L);
  t32.resize(L);
  for (int m = 0; m < L; ++m) {
    // exp(+2 pi i m / L) in float64 from libm
    const double a = 2.0 * M_PI * (double)m / (double)L;
    t64[m] = c128{std::cos(a), std::sin(a)};
    t32[m] = c64{(float)t64[m].x, (float)t64[m].y};
  }
}

struct Geometry {
  int n1, n2, n3, nst, nxr, ldst, nhmax;
  int form64, form32;      // plane pass form per precision (PlaneForm)
  bool split64, split32;   // three-kernel plane pass per precision (its HBM plane copies are allocated)
  bool density;            // workspace of pw_density / pw_scf_norm
  bool gamma;              // Gamma point, real wavefunctions on the half sphere
  std::vector<int> mfull;  // Miller indices of the whole sphere, [nfull][3]
  std::vector<int> enc;    // for each G of mfull: its vector index (2 g + mirror at Gamma)
};

// The whole sphere the transforms cover.  Without gamma it is the problem's
// list and enc[g] = g.  With gamma the problem lists the half sphere, G = 0
// first; G = (k, l, m) and -G fill the sphere, enc = 2 g for G and 2 g + 1
// for the mirror -G of half-sphere entry g (g >= 1).
pw_status full_sphere(const pw_problem* pr, bool gamma, Geometry* geo) {
  geo->mfull.assign(pr->miller, pr->miller + 3 * (size_t)pr->npw);
  geo->enc.resize(pr->npw);
  if (!gamma) {
    for (int g = 0; g < pr->npw; ++g) geo->enc[g] = g;
    return PW_OK;
  }
  PW_CHECK(pr->miller[0] == 0 && pr->miller[1] == 0 && pr->miller[2] == 0, PW_EINVAL,
           "a Gamma-point problem lists G = 0 first");
  PW_CHECK(pr->kpg[0] == 0.0 && pr->kpg[1] == 0.0 && pr->kpg[2] == 0.0, PW_EINVAL,
           "a Gamma-point problem needs k = 0");
  for (int g = 0; g < pr->npw; ++g) geo->enc[g] = 2 * g;
  for (int g = 1; g < pr->npw; ++g) {
    for (int d = 0; d < 3; ++d) geo->mfull.push_back(-pr->miller[3 * g + d]);
    geo->enc.push_back(2 * g + 1);
  }
  return PW_OK;
}

// transform workspace per band: the sticks, plus the plane copies of the
// three-kernel plane pass when a precision of the plan takes it
size_t fft_ws_per_band(const Geometry& g) {
  size_t b = (size_t)g.n3 * g.ldst * sizeof(c128);
  if (g.split64 || g.split32 || g.density) b += (size_t)g.n3 * g.n2 * g.nxr * sizeof(c128);
  return b;
}

// bands per transform chunk: the workspace of a chunk stays within the cap
int band_chunk_for(const pw_plan_opts& o, const Geometry& g) {
  const size_t cap_bytes = o.fft_ws_bytes ? o.fft_ws_bytes : ((size_t)2 << 30);
  size_t cap = cap_bytes / std::max<size_t>(fft_ws_per_band(g), 1);
  cap = std::max<size_t>(cap, 1);
  return (int)std::min<size_t>((size_t)std::max(o.nb_max, 1), cap);
}

pw_status check_problem(const pw_problem* pr, const pw_plan_opts* o, Geometry* geo) {
  PW_CHECK(pr != nullptr && o != nullptr, PW_EINVAL, "NULL problem or options");
  PW_CHECK(pr->npw > 0, PW_EINVAL, "npw must be positive");
  PW_CHECK(pr->miller && pr->kpg, PW_EINVAL, "miller and kpg are required (host arrays)");
  PW_CHECK(pr->vloc_r, PW_EINVAL, "vloc_r is required (device array)");
  PW_CHECK(o->precision == PW_FP64 || o->precision == PW_MIXED, PW_EINVAL, "bad precision");
  PW_CHECK(o->nb_max > 0, PW_EINVAL, "nb_max must be positive");
  PW_CHECK(o->ndim_max == 0 || (o->ndim_max >= 2 && o->ndim_max <= 8), PW_EINVAL, "ndim_max must be 0 or 2..8");
  PW_CHECK(pr->nbeta >= 0, PW_EINVAL, "nbeta < 0");
  if (pr->nbeta > 0) {
    PW_CHECK(pr->beta && pr->dmat && pr->blk_off, PW_EINVAL, "beta, dmat and blk_off are required when nbeta > 0");
    PW_CHECK(pr->ld_beta >= pr->npw, PW_EINVAL, "ld_beta < npw");
    PW_CHECK(pr->nblk > 0, PW_EINVAL, "nblk must be positive when nbeta > 0");
    PW_CHECK(pr->blk_off[0] == 0 && pr->blk_off[pr->nblk] == pr->nbeta, PW_EINVAL, "D blocks must cover [0, nbeta)");
  }
  PW_CHECK(o->gamma == 0 || o->gamma == 1, PW_EINVAL, "gamma must be 0 or 1");
  geo->gamma = o->gamma == 1;
  PW_TRY(full_sphere(pr, geo->gamma, geo));
  const int nfull = (int)geo->enc.size();
  const int* mf = geo->mfull.data();
  int hmax[3] = {0, 0, 0};
  for (int g = 0; g < nfull; ++g)
    for (int d = 0; d < 3; ++d) hmax[d] = std::max(hmax[d], std::abs(mf[3 * g + d]));
  for (int d = 0; d < 3; ++d) {
    PW_CHECK(pr->nr[d] >= 4 * hmax[d] + 1, PW_EINVAL,
             "FFT grid too small along axis " + std::to_string(d) + ": need >= " + std::to_string(4 * hmax[d] + 1));
    FftDesc f;
    PW_CHECK(fft_factor(pr->nr[d], f), PW_EINVAL, "grid size must have only prime factors 2, 3, 5");
  }
  geo->n1 = pr->nr[0];
  geo->n2 = pr->nr[1];
  geo->n3 = pr->nr[2];
  // sticks and x columns
  std::vector<char> col(geo->n1, 0);
  std::vector<char> stk((size_t)geo->n1 * geo->n2, 0);
  int nst = 0;
  for (int g = 0; g < nfull; ++g) {
    const int i1 = ((mf[3 * g] % geo->n1) + geo->n1) % geo->n1;
    const int i2 = ((mf[3 * g + 1] % geo->n2) + geo->n2) % geo->n2;
    col[i1] = 1;
    if (!stk[(size_t)i1 * geo->n2 + i2]) { stk[(size_t)i1 * geo->n2 + i2] = 1; ++nst; }
  }
  geo->nst = nst;
  geo->nxr = 0;
  for (int i = 0; i < geo->n1; ++i) geo->nxr += col[i];
  geo->ldst = (nst + 3) / 4 * 4;
  geo->nhmax = 0;
  for (int b = 0; b < pr->nblk && pr->nbeta > 0; ++b) {
    const int nh = pr->blk_off[b + 1] - pr->blk_off[b];
    PW_CHECK(nh > 0, PW_EINVAL, "empty or decreasing D block offsets");
    geo->nhmax = std::max(geo->nhmax, nh);
  }
  const bool mixed = o->precision == PW_MIXED;
  PW_CHECK(o->plane_mode >= 0 && o->plane_mode <= 4, PW_EINVAL, "plane_mode must be 0..4");
  PW_CHECK(o->nl_overlap >= 0 && o->nl_overlap <= 2, PW_EINVAL, "nl_overlap must be 0, 1 or 2");
  geo->form64 = plane_form_for<double>(o->plane_mode, geo->n1, geo->n2, geo->nxr);
  geo->form32 = mixed ? plane_form_for<float>(o->plane_mode, geo->n1, geo->n2, geo->nxr) : kFormQuad;
  geo->split64 = geo->form64 == kFormSplit;
  geo->split32 = mixed && geo->form32 == kFormSplit;
  PW_CHECK(o->density == 0 || o->density == 1, PW_EINVAL, "density must be 0 or 1");
  geo->density = o->density == 1;
  PW_CHECK(split_lds_bytes<double>(geo->n1, geo->n2) <= 160 * 1024, PW_EINVAL, "grid too large for the plane pass");
  PW_CHECK(z_lds_bytes<double>(geo->n3) <= 160 * 1024, PW_EINVAL, "n3 too large");
  return PW_OK;
}

// plane_mode 3 measurement (defined with the H.psi launch code below)
template <typename T>
pw_status tune_plane(pw_plan p, hipStream_t s);

}  // namespace

// ---------------------------------------------------------------------------
// public plan API
// ---------------------------------------------------------------------------
extern "C" size_t pw_footprint_bytes(const pw_problem* pr, const pw_plan_opts* o) {
  Geometry geo;
  if (check_problem(pr, o, &geo) != PW_OK) return 0;
  const bool mixed = o->precision == PW_MIXED;
  const size_t N = (size_t)geo.n1 * geo.n2 * geo.n3;
  const size_t ldb = ((size_t)pr->npw + 15) / 16 * 16;
  size_t b = 0;
  b += (size_t)pr->npw * (4 * sizeof(int) + 2 * sizeof(double));
  b += (size_t)geo.nst * 3 * sizeof(int) + geo.n1 * sizeof(int);
  b += (size_t)geo.nst * geo.n3 * sizeof(int);   // (z, stick) -> sphere map
  b += N * (sizeof(double) + (mixed ? sizeof(float) : 0));
  b += (size_t)pr->nbeta * ldb * (sizeof(c128) + (mixed ? sizeof(c64) : 0));
  b += (size_t)pr->nbeta * (2 * sizeof(int) + geo.nhmax * (sizeof(c128) + sizeof(c64)));
  const int chunk = band_chunk_for(*o, geo);
  b += (size_t)chunk * fft_ws_per_band(geo);
  if (geo.density) b += N * sizeof(c128) + kDensityPart * sizeof(double);
  b += 2 * (size_t)o->nb_max * std::max(pr->nbeta, 1) * sizeof(c128);
  if (pr->nbeta > 0 && pr->qmat != nullptr)
    b += (size_t)o->nb_max * pr->nbeta * sizeof(c128) + (size_t)pr->npw * sizeof(double) +
         (size_t)pr->nbeta * geo.nhmax * (sizeof(c128) + sizeof(c64));
  b += std::max(pw::splitk_part_bytes(std::max(pr->nbeta, 1), o->nb_max, pr->npw, sizeof(c128)),
                pw::dgemm_part_bytes(std::max(pr->nbeta, 1), o->nb_max));
  if (o->ndim_max > 0) b += pw::dav_bytes(pr->npw, o->nb_max, o->ndim_max) + pw::cg_bytes(pr->npw, o->nb_max);
  return b;
}

extern "C" pw_status pw_plan_create(pw_ctx ctx, const pw_problem* pr, const pw_plan_opts* o,
                                    pw_plan* out) {
  return pw::plan_create(ctx, pr, o, nullptr, nullptr, out);
}

pw_status pw::plan_create(pw_ctx ctx, const pw_problem* pr, const pw_plan_opts* o, MemPool* pool,
                          hipStream_t stream, pw_plan* out) {
  PW_CHECK(ctx != nullptr && out != nullptr, PW_EINVAL, "NULL context or output");
  *out = nullptr;
  Geometry geo;
  PW_TRY(check_problem(pr, o, &geo));
  PW_HIP(hipSetDevice(ctx->device));
  PW_TRY(set_lds_limits<double>());
  PW_TRY(set_lds_limits<float>());

  const int npw = pr->npw, n1 = geo.n1, n2 = geo.n2, n3 = geo.n3;
  const int nfull = (int)geo.enc.size();   // entries of the whole sphere (npw without gamma)
  const int* mfull = geo.mfull.data();
  // D blocks: Hermitian check
  std::vector<int> dstart, dlen;
  std::vector<c128> drow;
  if (pr->nbeta > 0) {
    dstart.resize(pr->nbeta);
    dlen.resize(pr->nbeta);
    drow.assign((size_t)pr->nbeta * geo.nhmax, c128{0, 0});
    size_t pos = 0;
    for (int b = 0; b < pr->nblk; ++b) {
      const int o0 = pr->blk_off[b], nh = pr->blk_off[b + 1] - o0;
      const pw_c128* blk = pr->dmat + pos;
      for (int i = 0; i < nh; ++i)
        for (int j = 0; j < nh; ++j) {
          const pw_c128 dij = blk[(size_t)j * nh + i], dji = blk[(size_t)i * nh + j];
          const double scale = std::max(1.0, std::hypot(dij.re, dij.im));
          PW_CHECK(std::abs(dij.re - dji.re) <= 1e-12 * scale && std::abs(dij.im + dji.im) <= 1e-12 * scale,
                   PW_EINVAL, "D block " + std::to_string(b) + " is not Hermitian");
          PW_CHECK(!geo.gamma || std::abs(dij.im) <= 1e-12 * scale, PW_EINVAL,
                   "a Gamma-point problem needs real D blocks (real-space-real projectors)");
          drow[(size_t)(o0 + i) * geo.nhmax + j] = c128{dij.re, dij.im};
        }
      for (int i = 0; i < nh; ++i) { dstart[o0 + i] = o0; dlen[o0 + i] = nh; }
      pos += (size_t)nh * nh;
    }
  }

  // q blocks (ultrasoft overlap): Hermitian check, block rows as for D
  const bool us = pr->nbeta > 0 && pr->qmat != nullptr;
  std::vector<c128> qrow;
  if (us) {
    qrow.assign((size_t)pr->nbeta * geo.nhmax, c128{0, 0});
    size_t pos = 0;
    for (int b = 0; b < pr->nblk; ++b) {
      const int o0 = pr->blk_off[b], nh = pr->blk_off[b + 1] - o0;
      const pw_c128* blk = pr->qmat + pos;
      for (int i = 0; i < nh; ++i)
        for (int j = 0; j < nh; ++j) {
          const pw_c128 qij = blk[(size_t)j * nh + i], qji = blk[(size_t)i * nh + j];
          const double scale = std::max(1.0, std::hypot(qij.re, qij.im));
          PW_CHECK(std::isfinite(qij.re) && std::isfinite(qij.im), PW_ENAN, "non-finite q block entry");
          PW_CHECK(std::abs(qij.re - qji.re) <= 1e-12 * scale && std::abs(qij.im + qji.im) <= 1e-12 * scale,
                   PW_EINVAL, "q block " + std::to_string(b) + " is not Hermitian");
          PW_CHECK(!geo.gamma || std::abs(qij.im) <= 1e-12 * scale, PW_EINVAL,
                   "a Gamma-point problem needs real q blocks (real-space-real projectors)");
          qrow[(size_t)(o0 + i) * geo.nhmax + j] = c128{qij.re, qij.im};
        }
      pos += (size_t)nh * nh;
    }
  }

  // sphere -> grid maps
  std::vector<int> i1v(nfull), i2v(nfull), i3v(nfull);
  {
    std::vector<char> seen((size_t)n1 * n2 * n3, 0);
    for (int g = 0; g < nfull; ++g) {
      i1v[g] = ((mfull[3 * g] % n1) + n1) % n1;
      i2v[g] = ((mfull[3 * g + 1] % n2) + n2) % n2;
      i3v[g] = ((mfull[3 * g + 2] % n3) + n3) % n3;
      const size_t key = ((size_t)i3v[g] * n2 + i2v[g]) * n1 + i1v[g];
      PW_CHECK(!seen[key], PW_EINVAL,
               geo.gamma ? "a Gamma-point problem lists G or -G twice (half sphere expected): index " +
                               std::to_string(g < npw ? g : g - npw + 1)
                         : "duplicate G vector at index " + std::to_string(g));
      seen[key] = 1;
    }
  }
  // x columns in ascending i1; sticks ordered by (column, i2); entries by i3
  std::vector<int> i1_hx(n1, -1);
  int nxr = 0;
  {
    std::vector<char> col(n1, 0);
    for (int g = 0; g < nfull; ++g) col[i1v[g]] = 1;
    for (int i = 0; i < n1; ++i)
      if (col[i]) i1_hx[i] = nxr++;
  }
  std::vector<int> order(nfull);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    if (i1_hx[i1v[a]] != i1_hx[i1v[b]]) return i1_hx[i1v[a]] < i1_hx[i1v[b]];
    if (i2v[a] != i2v[b]) return i2v[a] < i2v[b];
    return i3v[a] < i3v[b];
  });
  std::vector<int> st_ptr, st_hx, st_i2, ent_g(nfull), ent_z(nfull), ent_s(nfull);
  for (int e = 0; e < nfull; ++e) {
    const int g = order[e];
    if (e == 0 || i1v[g] != i1v[order[e - 1]] || i2v[g] != i2v[order[e - 1]]) {
      st_ptr.push_back(e);
      st_hx.push_back(i1_hx[i1v[g]]);
      st_i2.push_back(i2v[g]);
    }
    ent_g[e] = geo.enc[g];
    ent_z[e] = i3v[g];
    ent_s[e] = (int)st_hx.size() - 1;
  }
  st_ptr.push_back(nfull);
  std::vector<int> col_ptr(nxr + 1, 0);
  for (size_t s2 = 0; s2 < st_hx.size(); ++s2) col_ptr[st_hx[s2] + 1]++;
  for (int c = 0; c < nxr; ++c) col_ptr[c + 1] += col_ptr[c];
  std::vector<int> zidx((size_t)n3 * st_hx.size(), -1);
  for (int e = 0; e < nfull; ++e) zidx[(size_t)ent_z[e] * st_hx.size() + ent_s[e]] = ent_g[e];
  // Gamma: positions (z ldst + stick) of G and of -G for each half-sphere entry
  const int ldst_h = (int)((st_hx.size() + 3) / 4 * 4);
  std::vector<int> gpos_p, gpos_m;
  if (geo.gamma) {
    gpos_p.assign(npw, -1);
    gpos_m.assign(npw, -1);
    for (int e = 0; e < nfull; ++e) {
      const int enc = ent_g[e], pos = ent_z[e] * ldst_h + ent_s[e];
      if (enc & 1) gpos_m[enc >> 1] = pos; else gpos_p[enc >> 1] = pos;
    }
    gpos_m[0] = gpos_p[0];
  }
  std::vector<double> kin(npw);
  for (int g = 0; g < npw; ++g) {
    const double* q = pr->kpg + 3 * g;
    kin[g] = 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
  }

  pw_plan p = new pw_plan_s();
  p->pool = pool;
  p->init_stream = stream;
  p->ctx = ctx;
  p->device = ctx->device;
  p->opts = *o;
  p->npw = npw;
  p->n1 = n1; p->n2 = n2; p->n3 = n3;
  p->N = (long)n1 * n2 * n3;
  p->nst = geo.nst;
  p->nxr = nxr;
  p->ldst = geo.ldst;
  p->nbeta = pr->nbeta;
  p->nblk = pr->nbeta > 0 ? pr->nblk : 0;
  p->nhmax = geo.nhmax;
  p->ldb = (npw + 15) / 16 * 16;
  p->band_chunk = band_chunk_for(*o, geo);
  p->split64 = geo.split64;
  p->split32 = geo.split32;
  p->form64 = geo.form64;
  p->form32 = geo.form32;
  fft_factor(n1, p->f1);
  fft_factor(n2, p->f2);
  fft_factor(n3, p->f3);
  const bool mixed = o->precision == PW_MIXED;

  auto fail_cleanup = [&](pw_status st) {
    pw_plan_destroy(p);
    return st;
  };
#define PLAN_TRY(expr)                      \
  do {                                      \
    pw_status s_ = (expr);                  \
    if (s_ != PW_OK) return fail_cleanup(s_); \
  } while (0)

  PLAN_TRY(upload(p, &p->st_ptr, st_ptr));
  PLAN_TRY(upload(p, &p->st_hx, st_hx));
  PLAN_TRY(upload(p, &p->st_i2, st_i2));
  PLAN_TRY(upload(p, &p->ent_g, ent_g));
  PLAN_TRY(upload(p, &p->ent_z, ent_z));
  PLAN_TRY(upload(p, &p->ent_s, ent_s));
  PLAN_TRY(upload(p, &p->i1_hx, i1_hx));
  PLAN_TRY(upload(p, &p->zidx, zidx));
  PLAN_TRY(upload(p, &p->col_ptr, col_ptr));
  // the (column, y) -> stick map of the lane-group kernel: built for every
  // plan whose grid that kernel covers (plane_mode 3 may pick it later)
  if (plane_oct_kernel<double>(n1, n2) != nullptr) {
    std::vector<int> cy_st((size_t)nxr * n2, -1);
    for (size_t s2 = 0; s2 < st_hx.size(); ++s2) cy_st[(size_t)st_hx[s2] * n2 + st_i2[s2]] = (int)s2;
    PLAN_TRY(upload(p, &p->cy_st, cy_st));
  }
  p->gamma = geo.gamma;
  p->nfull = nfull;
  if (geo.gamma) {
    PLAN_TRY(upload(p, &p->gpos_p, gpos_p));
    PLAN_TRY(upload(p, &p->gpos_m, gpos_m));
  }
  PLAN_TRY(upload(p, &p->kin, kin));
  {
    std::vector<c128> t64;
    std::vector<c64> t32;
    twiddles(n1, t64, t32);
    PLAN_TRY(upload(p, &p->tw64_1, t64));
    PLAN_TRY(upload(p, &p->tw32_1, t32));
    twiddles(n2, t64, t32);
    PLAN_TRY(upload(p, &p->tw64_2, t64));
    PLAN_TRY(upload(p, &p->tw32_2, t32));
    twiddles(n3, t64, t32);
    PLAN_TRY(upload(p, &p->tw64_3, t64));
    PLAN_TRY(upload(p, &p->tw32_3, t32));
  }
  // V(r): copy, mean for the preconditioner diagonal, float32 copy
  PLAN_TRY(dalloc(p, &p->vr64, (size_t)p->N));
  if (hipMemcpyAsync(p->vr64, pr->vloc_r, sizeof(double) * p->N, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return fail_cleanup(pw::fail(PW_EDEVICE, "copy of vloc_r failed (is it a device pointer?)"));
  double v0 = 0.0;
  {
    std::vector<double> hv(p->N);
    if (hipMemcpyAsync(hv.data(), p->vr64, sizeof(double) * p->N, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return fail_cleanup(pw::fail(PW_EDEVICE, "readback of vloc_r failed"));
    long double acc = 0.0L;
    for (long i = 0; i < p->N; ++i) {
      if (!std::isfinite(hv[i])) return fail_cleanup(pw::fail(PW_ENAN, "non-finite value in vloc_r"));
      acc += hv[i];
    }
    v0 = (double)(acc / (long double)p->N);
  }
  if (mixed) {
    PLAN_TRY(dalloc(p, &p->vr32, (size_t)p->N));
    k_f64_to_f32<<<1024, 256, 0, stream>>>(p->vr64, p->vr32, (size_t)p->N);
  }
  // beta, D
  if (p->nbeta > 0) {
    PLAN_TRY(dalloc(p, &p->beta64, (size_t)p->nbeta * p->ldb));
    if (hipMemsetAsync(p->beta64, 0, sizeof(c128) * (size_t)p->nbeta * p->ldb, stream) != hipSuccess ||
        hipMemcpy2DAsync(p->beta64, sizeof(c128) * p->ldb, pr->beta, sizeof(c128) * pr->ld_beta,
                         sizeof(c128) * npw, p->nbeta, hipMemcpyDeviceToDevice, stream) != hipSuccess)
      return fail_cleanup(pw::fail(PW_EDEVICE, "copy of beta failed (is it a device pointer?)"));
    if (mixed) {
      PLAN_TRY(dalloc(p, &p->beta32, (size_t)p->nbeta * p->ldb));
      k_f64_to_f32<<<1024, 256, 0, stream>>>((const double*)p->beta64, (float*)p->beta32,
                                             2 * (size_t)p->nbeta * p->ldb);
    }
    PLAN_TRY(upload(p, &p->dstart, dstart));
    PLAN_TRY(upload(p, &p->dlen, dlen));
    PLAN_TRY(upload(p, &p->drow64, drow));
    std::vector<c64> d32(drow.size());
    for (size_t i = 0; i < drow.size(); ++i) d32[i] = c64{(float)drow[i].x, (float)drow[i].y};
    PLAN_TRY(upload(p, &p->drow32, d32));
  }
  PLAN_TRY(dalloc(p, &p->hdiag, (size_t)npw));
  k_hdiag<<<ceil_div(npw, 256), 256, 0, stream>>>(npw, p->nbeta, p->beta64, p->ldb, p->dstart, p->dlen,
                                       p->drow64, std::max(p->nhmax, 1), p->kin, v0, p->hdiag);
  if (us) {
    p->us = true;
    PLAN_TRY(upload(p, &p->qrow64, qrow));
    std::vector<c64> q32(qrow.size());
    for (size_t i = 0; i < qrow.size(); ++i) q32[i] = c64{(float)qrow[i].x, (float)qrow[i].y};
    PLAN_TRY(upload(p, &p->qrow32, q32));
    PLAN_TRY(dalloc(p, &p->sdiag, (size_t)npw));
    // diagonal of S: 1 + sum beta_i q_ij conj(beta_j)
    k_hdiag<<<ceil_div(npw, 256), 256, 0, stream>>>(npw, p->nbeta, p->beta64, p->ldb, p->dstart, p->dlen, p->qrow64,
                                         std::max(p->nhmax, 1), nullptr, 1.0, p->sdiag);
  }
  // workspace
  PLAN_TRY(dalloc(p, reinterpret_cast<c128**>(&p->sticks), (size_t)p->band_chunk * n3 * p->ldst));
  if (p->split64 || p->split32 || geo.density)
    PLAN_TRY(dalloc(p, reinterpret_cast<c128**>(&p->rows), (size_t)p->band_chunk * n3 * n2 * nxr));
  if (geo.density) {
    PLAN_TRY(dalloc(p, &p->dgrid, (size_t)p->N));
    PLAN_TRY(dalloc(p, &p->dpart, (size_t)kDensityPart));
  }
  const int nbeta1 = std::max(p->nbeta, 1);
  PLAN_TRY(dalloc(p, reinterpret_cast<c128**>(&p->becp), (size_t)o->nb_max * nbeta1));
  PLAN_TRY(dalloc(p, reinterpret_cast<c128**>(&p->becpd), (size_t)o->nb_max * nbeta1));
  if (us) PLAN_TRY(dalloc(p, reinterpret_cast<c128**>(&p->becpq), (size_t)o->nb_max * nbeta1));
  p->part_bytes = pw::splitk_part_bytes(nbeta1, o->nb_max, npw, sizeof(c128));
  if (geo.gamma) p->part_bytes = std::max(p->part_bytes, pw::dgemm_part_bytes(nbeta1, o->nb_max));
  PLAN_TRY(dalloc(p, reinterpret_cast<char**>(&p->part), p->part_bytes));
  if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess)
    return fail_cleanup(pw::fail(PW_EDEVICE, "stream/event creation failed"));
  if (o->ndim_max > 0) {
    PLAN_TRY(pw::dav_alloc(p));
    PLAN_TRY(pw::cg_alloc(p));
  }
  if (o->plane_mode == 3) {
    PLAN_TRY(tune_plane<double>(p, stream));
    if (mixed) PLAN_TRY(tune_plane<float>(p, stream));
  }
  if ((pool ? hipStreamSynchronize(stream) : hipDeviceSynchronize()) != hipSuccess)
    return fail_cleanup(pw::fail(PW_EDEVICE, "plan initialisation kernels failed"));
#undef PLAN_TRY
  *out = p;
  return PW_OK;
}

extern "C" pw_status pw_plan_destroy(pw_plan p) {
  pw::plan_destroy(p);
  return PW_OK;
}

// A pooled (served) plan waits only for its own streams: the caller has
// synchronized the stream its solve ran on, and the memory goes back to the
// pool.  Any other plan waits for the device, then frees its memory.
void pw::plan_destroy(pw_plan p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->pool) {
    if (p->side) (void)hipStreamSynchronize(p->side);
    (void)hipStreamSynchronize(p->init_stream);
  } else {
    (void)hipDeviceSynchronize();
  }
  pw::dav_free(p);
  pw::cg_free(p);
  for (void* q : p->allocs) pw::dev_free(p, q);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  if (p->side) (void)hipStreamDestroy(p->side);
  delete p;
  (void)hipGetLastError();   // leave no error of the teardown behind for other HIP users
}

extern "C" pw_status pw_plan_info(pw_plan p, int64_t out[8]) {
  PW_CHECK(p != nullptr && out != nullptr, PW_EINVAL, "NULL plan or output");
  out[0] = p->npw;
  out[1] = p->nst;
  out[2] = p->nxr;
  out[3] = p->N;
  out[4] = p->nbeta;
  out[5] = p->band_chunk;
  out[6] = p->form64;
  out[7] = p->opts.precision == PW_MIXED ? p->form32 : 0;
  return PW_OK;
}

// New local potential for an existing plan (the self-consistency loop: the
// geometry, sphere, projectors and workspace stay).  The new V(r) is read back
// and checked on the host before anything of the plan changes.
extern "C" pw_status pw_plan_set_potential(pw_plan p, const double* vloc_r, void* stream) {
  PW_CHECK(p != nullptr && vloc_r != nullptr, PW_EINVAL, "NULL plan or vloc_r");
  PW_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<double> hv(p->N);
  PW_CHECK(hipMemcpyAsync(hv.data(), vloc_r, sizeof(double) * p->N, hipMemcpyDeviceToHost, st) == hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess,
           PW_EDEVICE, "readback of vloc_r failed (is it a device pointer?)");
  long double acc = 0.0L;
  for (long i = 0; i < p->N; ++i) {
    PW_CHECK(std::isfinite(hv[i]), PW_ENAN, "non-finite value in vloc_r");
    acc += hv[i];
  }
  const double v0 = (double)(acc / (long double)p->N);
  PW_HIP(hipMemcpyAsync(p->vr64, vloc_r, sizeof(double) * p->N, hipMemcpyDeviceToDevice, st));
  if (p->vr32) k_f64_to_f32<<<1024, 256, 0, st>>>(p->vr64, p->vr32, (size_t)p->N);
  k_hdiag<<<ceil_div(p->npw, 256), 256, 0, st>>>(p->npw, p->nbeta, p->beta64, p->ldb, p->dstart, p->dlen,
                                               p->drow64, std::max(p->nhmax, 1), p->kin, v0, p->hdiag);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

namespace {
// The kernels and LDS sizes of one plane pass form, resolved once per call.
template <typename T>
struct PlaneLaunch {
  int form = kFormQuad;
  PlaneRegFn<T> preg = nullptr;   // register (quad) kernel and its planes per workgroup
  int ppw = 0;
  size_t plds = 0;
  PlaneOctFn<T> poct = nullptr;   // lane-group kernel
  size_t olds = 0;
  int cb = 0;                     // generic LDS kernel: transforms per batch
  size_t pl = 0;                  // its LDS (or that of the three-kernel form)
};

template <typename T>
pw_status plane_setup(pw_plan p, int form, PlaneLaunch<T>& L) {
  L = PlaneLaunch<T>{};
  L.form = form;
  const int n1 = p->n1, n2 = p->n2, nxr = p->nxr;
  switch (form) {
    case kFormQuad:
      // two z planes per workgroup where their LDS fits (the last passes over
      // columns and rows are fuller), else one; above 80 KB one workgroup
      // fills the CU's LDS (float32 at 144^2: 85 KB, 512 threads)
      if (plane_reg_lds_bytes<T>(n1, nxr, 2) <= kPlaneRegMaxLds) {
        L.preg = plane_reg_kernel<T, 2>(n1, n2);
        L.ppw = 2;
      } else if (plane_reg_lds_bytes<T>(n1, nxr, 1) <= kPlaneRegMaxLds1) {
        L.preg = plane_reg_kernel<T, 1>(n1, n2);
        L.ppw = 1;
      }
      PW_CHECK(L.preg != nullptr, PW_EINVAL, "no register plane kernel for this grid");
      L.plds = plane_reg_lds_bytes<T>(n1, nxr, L.ppw);
      if (L.plds > 64 * 1024) PW_TRY(raise_lds_limit((const void*)L.preg, (int)L.plds));
      break;
    case kFormGroup:
      L.poct = plane_oct_kernel<T>(n1, n2);
      PW_CHECK(L.poct != nullptr && p->cy_st != nullptr, PW_EINVAL, "no lane-group plane kernel for this grid");
      L.olds = plane_oct_lds_bytes<T>(n1, nxr);
      if (L.olds > 64 * 1024) PW_TRY(raise_lds_limit((const void*)L.poct, (int)L.olds));
      break;
    case kFormLds:
      L.cb = plane_batch<T>(n1, n2, nxr);
      PW_CHECK(L.cb > 0, PW_EINVAL, "grid too large for the generic plane kernel");
      L.pl = plane_lds_bytes<T>(n1, n2, nxr, L.cb);
      break;
    default:
      PW_CHECK(p->rows != nullptr, PW_EINVAL, "plan has no plane copies for the three-kernel form");
      L.pl = split_lds_bytes<T>(n1, n2);
      break;
  }
  return PW_OK;
}

// the plane pass (y, x, V(r), x, y of every z plane) of nbc bands of sticks
template <typename T>
void plane_launch(pw_plan p, const PlaneLaunch<T>& L, cpx<T>* st, const T* vr, const cpx<T>* tw1,
                  const cpx<T>* tw2, int nbc, hipStream_t s) {
  const SphereMap m = p->map();
  switch (L.form) {
    case kFormQuad:
      L.preg<<<dim3(nbc, ceil_div(p->n3, L.ppw)), plane_reg_threads<T>(p->n1, p->nxr), L.plds, s>>>(m, st, vr, tw1,
                                                                                                 tw2);
      break;
    case kFormGroup:
      L.poct<<<dim3(nbc, p->n3), OctCfg<T>::threads, L.olds, s>>>(m, st, vr, tw1);
      break;
    case kFormLds:
      k_plane<T><<<dim3(nbc, p->n3), PTHREADS, L.pl, s>>>(m, st, vr, tw1, tw2, L.cb);
      break;
    default: {
      cpx<T>* rows = static_cast<cpx<T>*>(p->rows);
      k_plane_yinv<T><<<dim3(p->n3, nbc, ceil_div(p->nxr, SPLIT_CB)), SPLIT_THREADS, L.pl, s>>>(m, st, rows, tw2);
      k_plane_x<T><<<dim3(p->n3, nbc, ceil_div(p->n2, SPLIT_CB)), SPLIT_THREADS, L.pl, s>>>(m, rows, vr, tw1);
      k_plane_yfwd<T><<<dim3(p->n3, nbc, ceil_div(p->nxr, SPLIT_CB)), SPLIT_THREADS, L.pl, s>>>(m, st, rows, tw2);
      break;
    }
  }
}

// plane_mode 3: time every form of the plane pass that fits this grid (the
// three-kernel form only when no other does) on one chunk of up to 16 bands
// of the stick workspace, and keep the fastest.  The choice is cached per
// precision and grid shape for the rest of the process, so plans of the same
// shape measure once.
template <typename T>
pw_status tune_plane(pw_plan p, hipStream_t s) {
  int& form = sizeof(T) == 8 ? p->form64 : p->form32;
  if (form == kFormSplit) return PW_OK;
  const std::array<int, 6> key{(int)sizeof(T), p->n1, p->n2, p->n3, p->nxr, p->nst};
  static std::mutex mu;
  static std::map<std::array<int, 6>, int> cache;
  {
    std::lock_guard<std::mutex> l(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      form = it->second;
      return PW_OK;
    }
  }
  std::vector<int> cand;
  for (int f : {(int)kFormQuad, (int)kFormGroup, (int)kFormLds})
    if (plane_form_ok<T>(f, p->n1, p->n2, p->nxr) && (f != kFormGroup || p->cy_st != nullptr)) cand.push_back(f);
  int best = form;
  if (cand.size() > 1) {
    const bool f64 = sizeof(T) == 8;
    const cpx<T>* tw1 = f64 ? (const cpx<T>*)p->tw64_1 : (const cpx<T>*)p->tw32_1;
    const cpx<T>* tw2 = f64 ? (const cpx<T>*)p->tw64_2 : (const cpx<T>*)p->tw32_2;
    const T* vr = f64 ? (const T*)p->vr64 : (const T*)p->vr32;
    cpx<T>* st = static_cast<cpx<T>*>(p->sticks);
    const int nbc = std::min(p->band_chunk, 16);
    PW_HIP(hipMemsetAsync(st, 0, sizeof(cpx<T>) * (size_t)nbc * p->n3 * p->ldst, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PW_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return pw::fail(PW_EDEVICE, "event creation failed");
    }
    float best_ms = 0.0f;
    pw_status st_out = PW_OK;
    for (int f : cand) {
      PlaneLaunch<T> L;
      st_out = plane_setup<T>(p, f, L);
      if (st_out != PW_OK) break;
      plane_launch<T>(p, L, st, vr, tw1, tw2, nbc, s);   // warm-up
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < 3; ++r) plane_launch<T>(p, L, st, vr, tw1, tw2, nbc, s);
      (void)hipEventRecord(e1, s);
      float ms = 0.0f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st_out = pw::fail(PW_EDEVICE, "plane pass timing failed");
        break;
      }
      if (f == cand.front() || ms < best_ms) {
        best_ms = ms;
        best = f;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    PW_TRY(st_out);
  }
  form = best;
  std::lock_guard<std::mutex> l(mu);
  cache[key] = best;
  return PW_OK;
}

template <typename T>
pw_status hpsi_fft(pw_plan p, int nb, const c128* psi, int ldpsi, c128* hpsi, int ldhpsi,
                   hipStream_t s, bool accumulate, hipEvent_t join) {
  const bool f64 = sizeof(T) == 8;
  const SphereMap m = p->map();
  const cpx<T>* tw1 = f64 ? (const cpx<T>*)p->tw64_1 : (const cpx<T>*)p->tw32_1;
  const cpx<T>* tw2 = f64 ? (const cpx<T>*)p->tw64_2 : (const cpx<T>*)p->tw32_2;
  const cpx<T>* tw3 = f64 ? (const cpx<T>*)p->tw64_3 : (const cpx<T>*)p->tw32_3;
  const T* vr = f64 ? (const T*)p->vr64 : (const T*)p->vr32;
  PW_CHECK(vr != nullptr, PW_EINVAL, "float32 H.psi needs a PW_MIXED plan");
  PlaneLaunch<T> pln;
  PW_TRY(plane_setup<T>(p, f64 ? p->form64 : p->form32, pln));
  const size_t zl = z_lds_bytes<T>(p->n3);
  cpx<T>* st = static_cast<cpx<T>*>(p->sticks);
  const int gz = ceil_div(p->nst, ZSB);
  const ZRegFns<T> zr = p->use_reg_plane ? zreg_kernels<T>(p->n3) : ZRegFns<T>{};
  const int gzr = ceil_div(p->nst, ZRSTICKS);
  // 16-lane-group z passes where no quad form exists (the complex path)
  const ZGrpFns<T> zg = (p->use_reg_plane && zr.inv == nullptr) ? zgrp_kernels<T>(p->n3) : ZGrpFns<T>{};
  const int gzg = ceil_div(p->nst, ZGSTICKS);
  // algorithmic bytes per band: sphere in/out (complex128) and one write plus
  // one read of the stick columns per transform direction; V(r) once per pass
  const double sphere_b = 16.0 * p->npw, stick_b = (double)sizeof(cpx<T>) * p->n3 * p->nst;
  // transforms: one per band, or one per pair of bands at Gamma
  const bool gam = p->gamma;
  const int nt = gam ? ceil_div(nb, 2) : nb;
  for (int c0 = 0; c0 < nt; c0 += p->band_chunk) {
    const int nbc = std::min(p->band_chunk, nt - c0);
    const int nbc8 = ceil_div(nbc, 8) * 8;
    const int zgrid = gz * nbc8, zrgrid = gzr * nbc8;
    const int b0 = gam ? 2 * c0 : c0;                    // first band of the chunk
    const int nbb = gam ? std::min(nb - b0, 2 * nbc) : nbc;
    if (gam) {
      pw::ProfScope ps(pw::PK_ZINV, s, nbb * sphere_b + nbc * stick_b);
      if (zr.inv_g)
        zr.inv_g<<<zrgrid, ZRTHREADS, 0, s>>>(m, psi + (size_t)b0 * ldpsi, ldpsi, st, tw3, gzr, nbc, nbb);
      else if (zg.inv_g)
        zg.inv_g<<<gzg * nbc8, ZGTHREADS, 0, s>>>(m, psi + (size_t)b0 * ldpsi, ldpsi, st, tw3, gzg, nbc, nbb);
      else
        k_zinv_g<T><<<zgrid, ZTHREADS, zl, s>>>(m, psi + (size_t)b0 * ldpsi, ldpsi, st, tw3, gz, nbc, nbb);
    } else {
      pw::ProfScope ps(pw::PK_ZINV, s, nbc * (sphere_b + stick_b));
      if (zr.inv)
        zr.inv<<<zrgrid, ZRTHREADS, 0, s>>>(m, psi + (size_t)c0 * ldpsi, ldpsi, st, tw3, gzr, nbc);
      else if (zg.inv)
        zg.inv<<<gzg * nbc8, ZGTHREADS, 0, s>>>(m, psi + (size_t)c0 * ldpsi, ldpsi, st, tw3, gzg, nbc);
      else
        k_zinv<T><<<zgrid, ZTHREADS, zl, s>>>(m, psi + (size_t)c0 * ldpsi, ldpsi, st, tw3, gz, nbc);
    }
    {
      pw::ProfScope ps(pw::PK_PLANE, s, nbc * 2.0 * stick_b + (double)sizeof(T) * p->N);
      plane_launch<T>(p, pln, st, vr, tw1, tw2, nbc, s);
    }
    if (gam) {
      pw::ProfScope ps(pw::PK_ZFWD, s, nbb * sphere_b + nbc * stick_b);
      if (zr.fwd_g)
        zr.fwd_g<<<zrgrid, ZRTHREADS, 0, s>>>(m, st, tw3, gzr, nbc);
      else if (zg.fwd_g)
        zg.fwd_g<<<gzg * nbc8, ZGTHREADS, 0, s>>>(m, st, tw3, gzg, nbc);
      else
        k_zfwd_g<T><<<zgrid, ZTHREADS, zl, s>>>(m, st, tw3, gz, nbc);
      if (join != nullptr && c0 == 0) PW_HIP(hipStreamWaitEvent(s, join, 0));
      k_gamma_gather<T><<<dim3(ceil_div(p->npw, 256), nbc), 256, 0, s>>>(
          p->npw, p->gpos_p, p->gpos_m, st, (size_t)p->n3 * p->ldst, p->kin, psi + (size_t)b0 * ldpsi, ldpsi,
          hpsi + (size_t)b0 * ldhpsi, ldhpsi, 1.0 / (double)p->N, accumulate ? 1 : 0, nbb);
      continue;
    }
    if (join != nullptr && c0 == 0) PW_HIP(hipStreamWaitEvent(s, join, 0));
    // with projectors, hpsi already holds the projector and kinetic terms
    // (flags 3: add to hpsi, no kinetic term here); else the pass adds the
    // kinetic term itself (flags 0)
    {
      pw::ProfScope ps(pw::PK_ZFWD, s, nbc * (sphere_b + stick_b));
      if (zr.fwd)
        zr.fwd<<<zrgrid, ZRTHREADS, 0, s>>>(m, st, psi + (size_t)c0 * ldpsi, ldpsi,
                                            hpsi + (size_t)c0 * ldhpsi, ldhpsi, tw3,
                                            1.0 / (double)p->N, accumulate ? 3 : 0, gzr, nbc);
      else if (zg.fwd)
        zg.fwd<<<gzg * nbc8, ZGTHREADS, 0, s>>>(m, st, psi + (size_t)c0 * ldpsi, ldpsi,
                                               hpsi + (size_t)c0 * ldhpsi, ldhpsi, tw3,
                                               1.0 / (double)p->N, accumulate ? 3 : 0, gzg, nbc);
      else
        k_zfwd<T><<<zgrid, ZTHREADS, zl, s>>>(m, st, psi + (size_t)c0 * ldpsi, ldpsi,
                                               hpsi + (size_t)c0 * ldhpsi, ldhpsi, tw3,
                                               1.0 / (double)p->N, accumulate ? 3 : 0, gz, nbc);
    }
  }
  PW_HIP(hipGetLastError());
  return PW_OK;
}
}  // namespace

pw_status pw::psi_to_rows(pw_plan p, int nt, int nbands, const c128* psi, int ldpsi, hipStream_t s) {
  PW_CHECK(p->rows != nullptr, PW_EINVAL, "plan has no plane-copy workspace (create it with opts.density = 1)");
  PW_CHECK(nt >= 0 && nt <= p->band_chunk, PW_EINVAL, "more transforms than one chunk");
  PW_CHECK(p->gamma ? (nbands <= 2 * nt && nbands >= 2 * nt - 1) || (nt == 0 && nbands == 0) : nbands == nt,
           PW_EINVAL, "band count does not match the transform count");
  if (nt == 0) return PW_OK;
  const SphereMap m = p->map();
  const cpx<double>* tw2 = (const cpx<double>*)p->tw64_2;
  const cpx<double>* tw3 = (const cpx<double>*)p->tw64_3;
  cpx<double>* st = static_cast<cpx<double>*>(p->sticks);
  const ZRegFns<double> zr = p->use_reg_plane ? zreg_kernels<double>(p->n3) : ZRegFns<double>{};
  const int nt8 = ceil_div(nt, 8) * 8;
  const int gzr = ceil_div(p->nst, ZRSTICKS), gz = ceil_div(p->nst, ZSB);
  const size_t zl = z_lds_bytes<double>(p->n3);
  if (p->gamma) {
    if (zr.inv_g)
      zr.inv_g<<<gzr * nt8, ZRTHREADS, 0, s>>>(m, psi, ldpsi, st, tw3, gzr, nt, nbands);
    else
      k_zinv_g<double><<<gz * nt8, ZTHREADS, zl, s>>>(m, psi, ldpsi, st, tw3, gz, nt, nbands);
  } else if (zr.inv) {
    zr.inv<<<gzr * nt8, ZRTHREADS, 0, s>>>(m, psi, ldpsi, st, tw3, gzr, nt);
  } else {
    k_zinv<double><<<gz * nt8, ZTHREADS, zl, s>>>(m, psi, ldpsi, st, tw3, gz, nt);
  }
  k_plane_yinv<double><<<dim3(p->n3, nt, ceil_div(p->nxr, SPLIT_CB)), SPLIT_THREADS,
                         split_lds_bytes<double>(p->n1, p->n2), s>>>(m, st, static_cast<cpx<double>*>(p->rows), tw2);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

// Gamma: out[n][j] = sum_{t < dlen_j} Re D[j][t] becp[n][dstart_j + t] (real D, real projections)
template <typename T>
__global__ void k_dapply_real(int nbeta, int nb, const double* __restrict__ becp, const int* __restrict__ dstart,
                              const int* __restrict__ dlen, const c128* __restrict__ drow, int nhmax,
                              T* __restrict__ out) {
  const int n = blockIdx.x;
  for (int j = threadIdx.x; j < nbeta; j += blockDim.x) {
    const int j0 = dstart[j], nh = dlen[j];
    double acc = 0.0;
    for (int t = 0; t < nh; ++t) acc += drow[(size_t)j * nhmax + t].x * becp[(size_t)n * nbeta + j0 + t];
    out[(size_t)n * nbeta + j] = (T)acc;
  }
}

// Gamma projector term, written into hpsi (overwrite): real projections
// <beta_j|psi> = 2 sum_k beta_jk psi_k - beta_j(0) psi(0) over the interleaved
// half sphere, D, then hpsi = beta (D <beta|psi>) as a real product of
// 2 npw rows
template <typename T>
pw_status nonlocal_gamma(pw_plan p, int nb, const c128* psi, int ldpsi, c128* hpsi, int ldhpsi, hipStream_t s) {
  const T* beta = sizeof(T) == 8 ? (const T*)p->beta64 : (const T*)p->beta32;
  double* becp = static_cast<double*>(p->becp);
  T* becpd = static_cast<T*>(p->becpd);
  const int K = 2 * p->npw;
  PW_TRY((pw::dgemm_tn<T, T, double>(p->nbeta, nb, K, beta, 2L * p->ldb, reinterpret_cast<const double*>(psi),
                                     2L * ldpsi, 1.0, 1.0, 0.0, becp, p->nbeta, false, p->part, p->part_bytes, s,
                                     pw::PK_CALBEC)));
  k_dapply_real<T><<<nb, 256, 0, s>>>(p->nbeta, nb, becp, p->dstart, p->dlen, p->drow64, p->nhmax, becpd);
  PW_HIP(hipGetLastError());
  PW_TRY((pw::dgemm_nn<T, T, T>(K, nb, p->nbeta, 1.0, beta, 2L * p->ldb, becpd, p->nbeta, 0.0,
                                reinterpret_cast<double*>(hpsi), 2L * ldhpsi, s, nullptr, pw::PK_ADDNL)));
  return PW_OK;
}

// Projector term on the plan's side stream, written into hpsi (overwrite):
// hpsi = beta (D <beta|psi>).  Runs concurrently with the transform passes
// (matrix cores vs vector ALUs); the final transform pass adds to it.
template <typename T>
pw_status nonlocal_side(pw_plan p, int nb, const c128* psi, int ldpsi, c128* hpsi, int ldhpsi,
                        hipStream_t side) {
  cpx<T>* bd = static_cast<cpx<T>*>(p->becpd);
  const cpx<T>* beta = sizeof(T) == 8 ? (const cpx<T>*)p->beta64 : (const cpx<T>*)p->beta32;
  PW_TRY(pw::calbec_d<T>(p, nb, psi, ldpsi, bd, side));
  pw::ProfScope ps(pw::PK_ADDNL, side, 8.0 * p->npw * nb * p->nbeta);
  // hpsi = beta becp' + 1/2 |k+G|^2 psi: the kinetic term rides on the
  // add-back's coalesced epilogue, so the forward z pass need not gather psi
  PW_TRY((pw::zgemm_nn<T, T, T>(p->npw, nb, p->nbeta, 1.0, beta, p->ldb, bd, p->nbeta, 0.0, hpsi, ldhpsi, side,
                                nullptr, p->kin, psi, ldpsi)));
  return PW_OK;
}

// Does the projector term run on the side stream, beside the transforms?  By
// default yes, unless the plane pass of this precision holds a whole CU's LDS
// with one workgroup (no room for the GEMM waves beside it: they only slow
// each other down) or takes the three-kernel form.
bool nl_beside(pw_plan p, bool f64) {
  if (p->opts.nl_overlap == 1) return true;
  if (p->opts.nl_overlap == 2) return false;
  const int form = f64 ? p->form64 : p->form32;
  switch (form) {
    case kFormSplit: return false;
    case kFormGroup:   // its workgroup holds more than 64 KB of LDS
      return (f64 ? plane_oct_lds_bytes<double>(p->n1, p->nxr) : plane_oct_lds_bytes<float>(p->n1, p->nxr)) <=
             64 * 1024;
    case kFormQuad:
      return (f64 ? plane_reg_lds_bytes<double>(p->n1, p->nxr, 1) : plane_reg_lds_bytes<float>(p->n1, p->nxr, 1)) <=
             kPlaneRegMaxLds;
    default: return true;
  }
}

pw_status pw::hpsi_launch(pw_plan p, pw_precision prec, int nb, const c128* psi, int ldpsi,
                          c128* hpsi, int ldhpsi, hipStream_t s) {
  if (nb == 0) return PW_OK;
  const bool f64 = prec == PW_FP64;
  if (!f64) PW_CHECK(p->opts.precision == PW_MIXED, PW_EINVAL, "float32 H.psi needs a PW_MIXED plan");
  hipEvent_t join = nullptr;
  auto nonlocal = [&](hipStream_t ns) -> pw_status {
    if (p->gamma) return f64 ? nonlocal_gamma<double>(p, nb, psi, ldpsi, hpsi, ldhpsi, ns)
                             : nonlocal_gamma<float>(p, nb, psi, ldpsi, hpsi, ldhpsi, ns);
    return f64 ? nonlocal_side<double>(p, nb, psi, ldpsi, hpsi, ldhpsi, ns)
               : nonlocal_side<float>(p, nb, psi, ldpsi, hpsi, ldhpsi, ns);
  };
  if (p->nbeta > 0 && !nl_beside(p, f64)) {
    // projector term first, on the caller's stream; the transforms add to it
    PW_TRY(nonlocal(s));
  } else if (p->nbeta > 0) {
    // fork: the side stream starts once psi is ready on s
    PW_HIP(hipEventRecord(p->ev_fork, s));
    PW_HIP(hipStreamWaitEvent(p->side, p->ev_fork, 0));
    PW_TRY(nonlocal(p->side));
    PW_HIP(hipEventRecord(p->ev_join, p->side));
    join = p->ev_join;
  }
  if (f64) PW_TRY(hpsi_fft<double>(p, nb, psi, ldpsi, hpsi, ldhpsi, s, p->nbeta > 0, join));
  else PW_TRY(hpsi_fft<float>(p, nb, psi, ldpsi, hpsi, ldhpsi, s, p->nbeta > 0, join));
  return PW_OK;
}

extern "C" pw_status hpsi_apply(pw_plan p, pw_precision prec, int32_t nb, const pw_c128* psi,
                                int32_t ldpsi, pw_c128* hpsi, int32_t ldhpsi, void* stream) {
  PW_CHECK(p != nullptr, PW_EINVAL, "NULL plan");
  PW_CHECK(nb >= 0 && nb <= p->opts.nb_max, PW_EINVAL,
           "nb out of range [0, nb_max=" + std::to_string(p->opts.nb_max) + "]");
  if (nb == 0) return PW_OK;
  PW_CHECK(psi != nullptr && hpsi != nullptr, PW_EINVAL, "NULL psi or hpsi");
  PW_CHECK(ldpsi >= p->npw && ldhpsi >= p->npw, PW_EINVAL, "leading dimension < npw");
  PW_CHECK(prec == PW_FP64 || prec == PW_MIXED, PW_EINVAL, "bad precision");
  const char* a0 = reinterpret_cast<const char*>(psi);
  const char* a1 = a0 + sizeof(pw_c128) * ((size_t)(nb - 1) * ldpsi + p->npw);
  const char* b0 = reinterpret_cast<const char*>(hpsi);
  const char* b1 = b0 + sizeof(pw_c128) * ((size_t)(nb - 1) * ldhpsi + p->npw);
  PW_CHECK(a1 <= b0 || b1 <= a0, PW_EINVAL, "psi and hpsi overlap");
  PW_HIP(hipSetDevice(p->device));
  return pw::hpsi_launch(p, prec, nb, reinterpret_cast<const c128*>(psi), ldpsi,
                         reinterpret_cast<c128*>(hpsi), ldhpsi, static_cast<hipStream_t>(stream));
}

namespace {
// Gamma: S psi = psi + beta (q <beta|psi>) with the real projections of the
// half sphere (2 sum - G = 0 term) and a real add-back over 2 npw rows;
// spsi already holds psi
template <typename T>
pw_status spsi_gamma(pw_plan p, int nb, const c128* psi, int ldpsi, c128* spsi, int ldspsi, hipStream_t s) {
  const T* beta = sizeof(T) == 8 ? (const T*)p->beta64 : (const T*)p->beta32;
  // the real projections, then q applied to them, both in the q workspace
  // (16 bytes per band and projector)
  double* becp = static_cast<double*>(p->becpq);
  T* becpq = reinterpret_cast<T*>(becp + (size_t)nb * p->nbeta);
  const int K = 2 * p->npw;
  PW_TRY((pw::dgemm_tn<T, T, double>(p->nbeta, nb, K, beta, 2L * p->ldb, reinterpret_cast<const double*>(psi),
                                     2L * ldpsi, 1.0, 1.0, 0.0, becp, p->nbeta, false, p->part, p->part_bytes, s,
                                     pw::PK_CALBEC)));
  k_dapply_real<T><<<nb, 256, 0, s>>>(p->nbeta, nb, becp, p->dstart, p->dlen, p->qrow64, p->nhmax, becpq);
  PW_HIP(hipGetLastError());
  PW_TRY((pw::dgemm_nn<T, T, T>(K, nb, p->nbeta, 1.0, beta, 2L * p->ldb, becpq, p->nbeta, 1.0,
                                reinterpret_cast<double*>(spsi), 2L * ldspsi, s, nullptr, pw::PK_ADDNL)));
  return PW_OK;
}
}  // namespace

pw_status pw::spsi_launch(pw_plan p, pw_precision prec, int nb, const c128* psi, int ldpsi, c128* spsi,
                          int ldspsi, hipStream_t s) {
  if (nb == 0) return PW_OK;
  const bool f64 = prec == PW_FP64;
  if (!f64) PW_CHECK(p->opts.precision == PW_MIXED, PW_EINVAL, "float32 S.psi needs a PW_MIXED plan");
  PW_HIP(hipMemcpy2DAsync(spsi, sizeof(c128) * ldspsi, psi, sizeof(c128) * ldpsi, sizeof(c128) * p->npw, nb,
                          hipMemcpyDeviceToDevice, s));
  if (!p->us) return PW_OK;
  if (p->gamma) return f64 ? spsi_gamma<double>(p, nb, psi, ldpsi, spsi, ldspsi, s)
                           : spsi_gamma<float>(p, nb, psi, ldpsi, spsi, ldspsi, s);
  if (f64) {
    c128* bq = static_cast<c128*>(p->becpq);
    PW_TRY(pw::calbec_d<double>(p, nb, psi, ldpsi, bq, s, p->qrow64));
    pw::ProfScope ps(pw::PK_ADDNL, s, 8.0 * p->npw * nb * p->nbeta);
    PW_TRY((pw::zgemm_nn<double, double, double>(p->npw, nb, p->nbeta, 1.0, p->beta64, p->ldb, bq, p->nbeta, 1.0,
                                                 spsi, ldspsi, s)));
  } else {
    c64* bq = static_cast<c64*>(p->becpq);
    PW_TRY(pw::calbec_d<float>(p, nb, psi, ldpsi, bq, s, p->qrow32));
    pw::ProfScope ps(pw::PK_ADDNL, s, 8.0 * p->npw * nb * p->nbeta);
    PW_TRY((pw::zgemm_nn<float, float, float>(p->npw, nb, p->nbeta, 1.0, p->beta32, p->ldb, bq, p->nbeta, 1.0,
                                              spsi, ldspsi, s)));
  }
  return PW_OK;
}

extern "C" pw_status spsi_apply(pw_plan p, pw_precision prec, int32_t nb, const pw_c128* psi, int32_t ldpsi,
                                pw_c128* spsi, int32_t ldspsi, void* stream) {
  PW_CHECK(p != nullptr, PW_EINVAL, "NULL plan");
  PW_CHECK(nb >= 0 && nb <= p->opts.nb_max, PW_EINVAL, "nb out of range [0, nb_max]");
  if (nb == 0) return PW_OK;
  PW_CHECK(psi != nullptr && spsi != nullptr, PW_EINVAL, "NULL psi or spsi");
  PW_CHECK(ldpsi >= p->npw && ldspsi >= p->npw, PW_EINVAL, "leading dimension < npw");
  PW_CHECK(prec == PW_FP64 || prec == PW_MIXED, PW_EINVAL, "bad precision");
  const char* a0 = reinterpret_cast<const char*>(psi);
  const char* a1 = a0 + sizeof(pw_c128) * ((size_t)(nb - 1) * ldpsi + p->npw);
  const char* b0 = reinterpret_cast<const char*>(spsi);
  const char* b1 = b0 + sizeof(pw_c128) * ((size_t)(nb - 1) * ldspsi + p->npw);
  PW_CHECK(a1 <= b0 || b1 <= a0, PW_EINVAL, "psi and spsi overlap");
  PW_HIP(hipSetDevice(p->device));
  return pw::spsi_launch(p, prec, nb, reinterpret_cast<const c128*>(psi), ldpsi, reinterpret_cast<c128*>(spsi),
                         ldspsi, static_cast<hipStream_t>(stream));
}
