// Output charge density of a block of bands and the scf norm of a density
// change (the self-consistency appendix):
//
//   rho(r_j) = (1/omega) sum_b w_b |psi_b(r_j)|^2,  psi_b(r_j) = sum_G psi_b(G) exp(+i G.r_j)
//   ||drho||^2 = 4 pi omega sum_{G != 0} |drho(G)|^2 / |G|^2,  drho(G) = (1/N) sum_j drho(r_j) exp(-i G.r_j)
//
// The density reuses the first half of the H.psi transforms: the inverse z
// pass onto the sticks and the inverse y pass of every plane into the plane
// copies ([band][z][y][x column]).  One workgroup then owns a strip of rows
// of one plane and runs the inverse x transforms of those rows for every band
// of the chunk in order, accumulating w_b |psi_b|^2 in LDS: the band sum is
// done in a fixed order, with no atomics, so the result is reproducible.
//
// The norm transforms drho on the full grid (three passes of batched 1D
// transforms along x, y and z through HBM) and sums the weighted squares in a
// fixed order (per-workgroup partial sums, then one workgroup).
#include <cmath>

#include "plan.h"
#include "profile.h"

namespace {

constexpr int DCB = 16;          // rows (or lines) per workgroup
constexpr int DTHREADS = 256;

size_t dens_lds_bytes(int n1, int n2, int n3) {
  const int lmax = std::max(n1, std::max(n2, n3));
  return 2 * sizeof(c128) * (size_t)DCB * lmax + sizeof(double) * (size_t)DCB * n1 + sizeof(int) * (size_t)n1;
}

// rows [r0, r0+DCB) of plane z: for each transform t, inverse x of the row
// (its x columns scattered to their grid positions), then
// acc += w_t |psi_t(r)|^2, or at Gamma (gamma = 1: transform t holds
// psi_2t(r) + i psi_2t+1(r), both real) acc += w_2t Re^2 + w_2t+1 Im^2
__global__ void __launch_bounds__(DTHREADS)
k_density_x(SphereMap m, const c128* __restrict__ rows, int nt, int nbands, int gamma,
            const double* __restrict__ w, const c128* __restrict__ tw1, double inv_omega, int add,
            double* __restrict__ rho) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n1 = m.n1, n2 = m.n2, nxr = m.nxr;
  const int lmax = max(n1, max(n2, m.n3));
  c128* A = reinterpret_cast<c128*>(smem_raw);
  c128* B = A + DCB * lmax;
  double* acc = reinterpret_cast<double*>(B + DCB * lmax);   // [DCB][n1]
  int* hx_of = reinterpret_cast<int*>(acc + DCB * n1);        // [n1]
  const int z = blockIdx.x, r0 = blockIdx.y * DCB;
  const int nr = min(DCB, n2 - r0);
  for (int i = threadIdx.x; i < n1; i += blockDim.x) hx_of[i] = m.i1_hx[i];
  for (int i = threadIdx.x; i < DCB * n1; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  for (int b = 0; b < nt; ++b) {
    const c128* rw = rows + (((size_t)b * m.n3 + z) * n2 + r0) * nxr;
    const double wa = gamma ? w[2 * b] : w[b];
    const double wi = gamma ? (2 * b + 1 < nbands ? w[2 * b + 1] : 0.0) : wa;
    fft_run<double>(
        m.f1, nr, 1.0, tw1, A, B, lmax, false, false,
        [&](int r, int i) {
          const int hx = hx_of[i];
          return hx >= 0 ? rw[(size_t)r * nxr + hx] : c128{0.0, 0.0};
        },
        // every (r, i) is stored by exactly one thread per transform
        [&](int r, int i, c128 v) { acc[r * n1 + i] += wa * (v.x * v.x) + wi * (v.y * v.y); });
  }
  double* out = rho + ((size_t)z * n2 + r0) * n1;
  for (int e = threadIdx.x; e < nr * n1; e += blockDim.x) {
    const double v = acc[e] * inv_omega;
    out[e] = add ? out[e] + v : v;
  }
}

// x pass of the norm: g[z][y][:] = DFT_x( rho_out - rho_in ) (sign -1), rows [r0, r0+DCB) of plane z
__global__ void __launch_bounds__(DTHREADS)
k_norm_x(SphereMap m, const double* __restrict__ ro, const double* __restrict__ ri, c128* __restrict__ g,
         const c128* __restrict__ tw1) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n1 = m.n1, n2 = m.n2, lmax = max(n1, max(n2, m.n3));
  c128* A = reinterpret_cast<c128*>(smem_raw);
  c128* B = A + DCB * lmax;
  const int z = blockIdx.x, r0 = blockIdx.y * DCB, nr = min(DCB, n2 - r0);
  const size_t base = ((size_t)z * n2 + r0) * n1;
  fft_run<double>(
      m.f1, nr, -1.0, tw1, A, B, lmax, false, false,
      [&](int r, int i) { return c128{ro[base + (size_t)r * n1 + i] - ri[base + (size_t)r * n1 + i], 0.0}; },
      [&](int r, int i, c128 v) { g[base + (size_t)r * n1 + i] = v; });
}

// y pass: lines along y at fixed (z, x), x in [x0, x0+DCB)
__global__ void __launch_bounds__(DTHREADS)
k_norm_y(SphereMap m, c128* __restrict__ g, const c128* __restrict__ tw2) {
  extern __shared__ __align__(16) char smem_raw[];
  const int n1 = m.n1, n2 = m.n2, lmax = max(n1, max(n2, m.n3));
  c128* A = reinterpret_cast<c128*>(smem_raw);
  c128* B = A + DCB * lmax;
  const int z = blockIdx.x, x0 = blockIdx.y * DCB, nx = min(DCB, n1 - x0);
  c128* pl = g + (size_t)z * n2 * n1 + x0;
  fft_run<double>(
      m.f2, nx, -1.0, tw2, A, B, lmax, true, true,
      [&](int x, int i) { return pl[(size_t)i * n1 + x]; },
      [&](int x, int i, c128 v) { pl[(size_t)i * n1 + x] = v; });
}

// z pass: lines along z at fixed (y, x), x in [x0, x0+DCB); then the weighted
// squares |g|^2 / (N^2 |G|^2) of these lines, summed per workgroup
__global__ void __launch_bounds__(DTHREADS)
k_norm_z(SphereMap m, const c128* __restrict__ g, const c128* __restrict__ tw3, double b00, double b01,
         double b02, double b10, double b11, double b12, double b20, double b21, double b22,
         double* __restrict__ part) {
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ double red[DTHREADS / 64];
  const int n1 = m.n1, n2 = m.n2, n3 = m.n3, lmax = max(n1, max(n2, n3));
  c128* A = reinterpret_cast<c128*>(smem_raw);
  c128* B = A + DCB * lmax;
  c128* X = reinterpret_cast<c128*>(smem_raw) + 2 * DCB * lmax;   // [DCB][n3] results
  const int y = blockIdx.x, x0 = blockIdx.y * DCB, nx = min(DCB, n1 - x0);
  const c128* col = g + (size_t)y * n1 + x0;
  const size_t zs = (size_t)n1 * n2;
  fft_run<double>(
      m.f3, nx, -1.0, tw3, A, B, lmax, true, true,
      [&](int x, int i) { return col[(size_t)i * zs + x]; },
      [&](int x, int i, c128 v) { X[x * n3 + i] = v; });
  // fft_run ends with a barrier: X is complete
  const double invn = 1.0 / ((double)n1 * n2 * n3);
  const int m2 = y <= n2 / 2 ? y : y - n2;
  double s = 0.0;
  for (int e = threadIdx.x; e < nx * n3; e += blockDim.x) {
    const int xl = e / n3, iz = e - xl * n3;
    const int ix = x0 + xl;
    const int m1 = ix <= n1 / 2 ? ix : ix - n1;
    const int m3 = iz <= n3 / 2 ? iz : iz - n3;
    if (m1 == 0 && m2 == 0 && m3 == 0) continue;
    const double gx = m1 * b00 + m2 * b10 + m3 * b20;
    const double gy = m1 * b01 + m2 * b11 + m3 * b21;
    const double gz = m1 * b02 + m2 * b12 + m3 * b22;
    const double g2 = gx * gx + gy * gy + gz * gz;
    const c128 v = X[e];
    const double c2 = (v.x * v.x + v.y * v.y) * invn * invn;
    s += c2 / g2;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < DTHREADS / 64; ++i) t += red[i];
    part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
  }
}

// one workgroup: total = sum of the partials in index order (each thread a
// contiguous range, then the ranges in order)
__global__ void __launch_bounds__(DTHREADS) k_norm_sum(int n, const double* __restrict__ part, double scale,
                                                       double* __restrict__ out) {
  __shared__ double v[DTHREADS];
  const int per = (n + DTHREADS - 1) / DTHREADS;
  const int a = threadIdx.x * per, b = min(n, a + per);
  double s = 0.0;
  for (int i = a; i < b; ++i) s += part[i];
  v[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < DTHREADS; ++i) t += v[i];
    *out = t * scale;
  }
}

pw_status set_limits() {
  static bool done = false;
  if (done) return PW_OK;
  for (const void* fn : {(const void*)k_density_x, (const void*)k_norm_x, (const void*)k_norm_y,
                         (const void*)k_norm_z}) {
    hipFuncAttributes at;
    PW_HIP(hipFuncGetAttributes(&at, fn));
    PW_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)at.sharedSizeBytes));
  }
  done = true;
  return PW_OK;
}

}  // namespace

extern "C" pw_status pw_density(pw_plan p, int32_t nb, const pw_c128* psi, int32_t ldpsi, const double* w,
                                double omega, int32_t accumulate, double* rho, void* stream) {
  PW_CHECK(p != nullptr, PW_EINVAL, "NULL plan");
  PW_CHECK(p->dgrid != nullptr, PW_EINVAL, "plan was created without density workspace (opts.density = 0)");
  PW_CHECK(nb >= 0 && nb <= p->opts.nb_max, PW_EINVAL, "nb out of range [0, nb_max]");
  PW_CHECK(ldpsi >= p->npw, PW_EINVAL, "ldpsi < npw");
  PW_CHECK(omega > 0.0 && std::isfinite(omega), PW_EINVAL, "omega must be positive");
  PW_CHECK(rho != nullptr && (nb == 0 || (psi != nullptr && w != nullptr)), PW_EINVAL, "NULL pointer");
  PW_CHECK(accumulate == 0 || accumulate == 1, PW_EINVAL, "accumulate must be 0 or 1");
  PW_HIP(hipSetDevice(p->device));
  PW_TRY(set_limits());
  hipStream_t s = static_cast<hipStream_t>(stream);
  const SphereMap m = p->map();
  const size_t lds = dens_lds_bytes(p->n1, p->n2, p->n3);
  const c128* psi_c = reinterpret_cast<const c128*>(psi);
  if (nb == 0) {
    if (!accumulate) PW_HIP(hipMemsetAsync(rho, 0, sizeof(double) * (size_t)p->N, s));
    return PW_OK;
  }
  pw::ProfScope ps(pw::PK_DENSITY, s, (double)nb * (16.0 * p->npw) + 8.0 * (double)p->N);
  // transforms: one per band, or one per pair of bands at Gamma
  const bool gam = p->gamma;
  const int nt = gam ? ceil_div(nb, 2) : nb;
  for (int c0 = 0; c0 < nt; c0 += p->band_chunk) {
    const int ntc = std::min(p->band_chunk, nt - c0);
    const int b0 = gam ? 2 * c0 : c0;
    const int nbb = gam ? std::min(nb - b0, 2 * ntc) : ntc;
    PW_TRY(pw::psi_to_rows(p, ntc, nbb, psi_c + (size_t)b0 * ldpsi, ldpsi, s));
    k_density_x<<<dim3(p->n3, ceil_div(p->n2, DCB)), DTHREADS, lds, s>>>(
        m, static_cast<const c128*>(p->rows), ntc, nbb, gam ? 1 : 0, w + b0, p->tw64_1, 1.0 / omega,
        (accumulate || c0 > 0) ? 1 : 0, rho);
    PW_HIP(hipGetLastError());
  }
  return PW_OK;
}

extern "C" pw_status pw_scf_norm(pw_plan p, const double* rho_out, const double* rho_in, const double* bvec,
                                 double omega, double* norm2, void* stream) {
  PW_CHECK(p != nullptr, PW_EINVAL, "NULL plan");
  PW_CHECK(p->dgrid != nullptr, PW_EINVAL, "plan was created without density workspace (opts.density = 0)");
  PW_CHECK(rho_out && rho_in && bvec && norm2, PW_EINVAL, "NULL pointer");
  PW_CHECK(omega > 0.0 && std::isfinite(omega), PW_EINVAL, "omega must be positive");
  for (int i = 0; i < 9; ++i) PW_CHECK(std::isfinite(bvec[i]), PW_EINVAL, "non-finite reciprocal vector");
  PW_HIP(hipSetDevice(p->device));
  PW_TRY(set_limits());
  hipStream_t s = static_cast<hipStream_t>(stream);
  const SphereMap m = p->map();
  const size_t lds = dens_lds_bytes(p->n1, p->n2, p->n3);
  const int lmax = std::max(p->n1, std::max(p->n2, p->n3));
  const size_t lds_z = 2 * sizeof(c128) * (size_t)DCB * lmax + sizeof(c128) * (size_t)DCB * p->n3;
  const int gy = ceil_div(p->n1, DCB);
  PW_CHECK((size_t)p->n2 * gy < (size_t)kDensityPart, PW_EINVAL, "grid too large for the norm's partial sums");
  k_norm_x<<<dim3(p->n3, ceil_div(p->n2, DCB)), DTHREADS, lds, s>>>(m, rho_out, rho_in, p->dgrid, p->tw64_1);
  k_norm_y<<<dim3(p->n3, gy), DTHREADS, lds, s>>>(m, p->dgrid, p->tw64_2);
  k_norm_z<<<dim3(p->n2, gy), DTHREADS, lds_z, s>>>(m, p->dgrid, p->tw64_3, bvec[0], bvec[1], bvec[2], bvec[3],
                                                    bvec[4], bvec[5], bvec[6], bvec[7], bvec[8], p->dpart);
  k_norm_sum<<<1, DTHREADS, 0, s>>>(p->n2 * gy, p->dpart, 4.0 * M_PI * omega, p->dpart + kDensityPart - 1);
  PW_HIP(hipGetLastError());
  double out = 0.0;
  PW_HIP(hipMemcpyAsync(&out, p->dpart + kDensityPart - 1, sizeof(double), hipMemcpyDeviceToHost, s));
  PW_HIP(hipStreamSynchronize(s));
  *norm2 = out;
  return PW_OK;
}
