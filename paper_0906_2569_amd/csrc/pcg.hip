// Band-by-band preconditioned conjugate gradient for the nb lowest
// eigenpairs (the iterative-diagonalization appendix, "Conjugate-Gradient"),
// float64, for S = 1 and for the ultrasoft overlap S = 1 + sum beta q beta^H,
// on the full sphere or, at Gamma, on the half sphere of real functions.
//
// Band i minimizes <y|H~|y> - lambda (<y|S~|y> - 1), H~ = PHP, S~ = PSP,
// y = P^-1 psi, subject to S-orthogonality to the bands already found.  The
// vectors kept are the appendix's P g and P h, in the psi variables:
//
//   lambda = Re <S psi|P^2|H psi> / <S psi|P^2|S psi>   (makes P g S-orthogonal to psi)
//   G = P g = P^2 (H psi - lambda S psi), then made S-orthogonal to psi_j, j < i
//   D = P h = G + gamma D_prev,  gamma = Re <G - G_prev|G> / <G_prev|G_prev>
//       (Polak-Ribiere), then made S-orthogonal to psi;  N = D / <D|S|D>^(1/2)
//   psi <- psi cos(theta) + N sin(theta), and H psi, S psi likewise
//   theta = (1/2) atan(a / (eps - b)), a = 2 Re <psi|H N>, b = <N|H N>,
//       eps = <psi|H psi>; of the two stationary angles theta, theta + pi/2
//       the one with the lower energy
//
// with the kinetic-only preconditioner P^2(G) = 1 / smax(T_G, tau).  One H.psi
// of a single band per iteration (and, with S != 1, one S.psi of N and one of
// G for its projection on the bands found).  The vector steps run in single
// 1024-thread workgroups (fixed-order reductions: reproducible); the host
// reads one small flag block per iteration.  A final float64 H.psi (and S.psi)
// of the whole block gives the returned eigenvalues and residual norms.
#include <cmath>

#include "plan.h"
#include "profile.h"

namespace {

constexpr int CT = 1024;

struct CgScalars {
  double lambda, eps, gg_prev, resid, deps;
  int first, conv, pad0, pad1;
};

// sums of K values over the workgroup (red: [K][16])
template <int K>
__device__ void block_sums(double (&v)[K], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) red[k * 16 + wid] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[k * 16 + w];
    v[k] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ double p2_of(double t, double tau) {
  return 1.0 / (0.5 * (t + tau + sqrt((t - tau) * (t - tau) + tau * tau)));
}

// Weight of entry g in a real inner product over the whole sphere.  At Gamma
// (GAM) the vectors hold the half sphere of real functions: every entry but
// G = 0 (index 0, real) stands for G and -G, so Re <a|b> = 2 sum - a(0) b(0);
// the imaginary part of such a product is zero.
template <bool GAM>
__device__ __forceinline__ double wt(int g) { return GAM ? (g == 0 ? 1.0 : 2.0) : 1.0; }

// eps = <psi|H psi> (psi normalized before), first iteration flag
template <bool GAM>
__global__ void __launch_bounds__(CT) k_cg_start(int npw, const c128* __restrict__ psi,
                                               const c128* __restrict__ hpsi, CgScalars* __restrict__ sc) {
  __shared__ double red[16];
  double v[1] = {0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x)
    v[0] += wt<GAM>(g) * (psi[g].x * hpsi[g].x + psi[g].y * hpsi[g].y);
  block_sums<1>(v, red);
  if (threadIdx.x == 0) {
    sc->eps = v[0];
    sc->first = 1;
    sc->conv = 0;
    sc->gg_prev = 0.0;
  }
}

// G = P^2 (H psi - lambda S psi), lambda = Re <S psi|P^2 H psi> / <S psi|P^2 S psi>;
// spsi is S psi (psi itself when S = 1)
template <bool GAM>
__global__ void __launch_bounds__(CT) k_cg_grad(int npw, const c128* __restrict__ spsi,
                                              const c128* __restrict__ hpsi, const double* __restrict__ kin,
                                              double tau, c128* __restrict__ G, CgScalars* __restrict__ sc) {
  __shared__ double red[2 * 16];
  double v[2] = {0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double p2 = wt<GAM>(g) * p2_of(kin[g], tau);
    v[0] += p2 * (spsi[g].x * hpsi[g].x + spsi[g].y * hpsi[g].y);
    v[1] += p2 * (spsi[g].x * spsi[g].x + spsi[g].y * spsi[g].y);
  }
  block_sums<2>(v, red);
  const double lam = v[0] / v[1];
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double p2 = p2_of(kin[g], tau);
    G[g] = c128{p2 * (hpsi[g].x - lam * spsi[g].x), p2 * (hpsi[g].y - lam * spsi[g].y)};
  }
  if (threadIdx.x == 0) sc->lambda = lam;
}

// D = G + gamma D (gamma = 0 on the first iteration), D -= psi <S psi|D>,
// Gp = G, gg_prev = <G|G>; N = D / ||D|| when S = 1 (US false: spsi is psi),
// N = D otherwise (normalized in the S metric once S N is known)
template <bool US, bool GAM>
__global__ void __launch_bounds__(CT) k_cg_dir(int npw, const c128* __restrict__ psi, const c128* __restrict__ spsi,
                                             const c128* __restrict__ G, c128* __restrict__ Gp,
                                             c128* __restrict__ D, c128* __restrict__ N,
                                             CgScalars* __restrict__ sc) {
  __shared__ double red[2 * 16];
  double v[2] = {0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    v[0] += wt<GAM>(g) * (G[g].x * G[g].x + G[g].y * G[g].y);    // <G|G>
    v[1] += wt<GAM>(g) * (Gp[g].x * G[g].x + Gp[g].y * G[g].y);  // Re <Gp|G>
  }
  block_sums<2>(v, red);
  const bool first = sc->first != 0;
  const double gamma = first ? 0.0 : (v[0] - v[1]) / sc->gg_prev;
  double w[2] = {0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const c128 dprev = first ? c128{0.0, 0.0} : D[g];
    const c128 d = c128{G[g].x + gamma * dprev.x, G[g].y + gamma * dprev.y};
    D[g] = d;
    Gp[g] = G[g];
    w[0] += wt<GAM>(g) * (spsi[g].x * d.x + spsi[g].y * d.y);    // Re <S psi|D>
    w[1] += spsi[g].x * d.y - spsi[g].y * d.x;                   // Im <S psi|D>
  }
  block_sums<2>(w, red);
  if (GAM) w[1] = 0.0;
  double u[1] = {0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const c128 p = psi[g];
    const c128 d = c128{D[g].x - (p.x * w[0] - p.y * w[1]), D[g].y - (p.x * w[1] + p.y * w[0])};
    D[g] = d;
    if (!US) u[0] += wt<GAM>(g) * (d.x * d.x + d.y * d.y);
  }
  if (US) {
    for (int g = threadIdx.x; g < npw; g += blockDim.x) N[g] = D[g];
  } else {
    block_sums<1>(u, red);
    const double inv = u[0] > 0.0 ? 1.0 / sqrt(u[0]) : 0.0;
    for (int g = threadIdx.x; g < npw; g += blockDim.x) N[g] = c128{D[g].x * inv, D[g].y * inv};
  }
  if (threadIdx.x == 0) {
    sc->gg_prev = v[0];
    sc->first = 0;
  }
}

// line minimization along N, update of psi, H psi (and S psi when US), new
// eps = <psi|H psi> / <psi|S psi> and residual ||H psi - eps S psi||
template <bool US, bool GAM>
__global__ void __launch_bounds__(CT) k_cg_rotate(int npw, c128* __restrict__ psi, c128* __restrict__ hpsi,
                                                c128* __restrict__ spsi, const c128* __restrict__ N,
                                                const c128* __restrict__ HN, const c128* __restrict__ SN,
                                                double tol_r, double tol_e, CgScalars* __restrict__ sc) {
  __shared__ double red[2 * 16];
  __shared__ double cs[2];
  double v[2] = {0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    v[0] += wt<GAM>(g) * (psi[g].x * HN[g].x + psi[g].y * HN[g].y);   // Re <psi|H N>
    v[1] += wt<GAM>(g) * (N[g].x * HN[g].x + N[g].y * HN[g].y);       // <N|H N>
  }
  block_sums<2>(v, red);
  if (threadIdx.x == 0) {
    const double eps = sc->eps, a = 2.0 * v[0], b = v[1];
    double th = (eps != b) ? 0.5 * atan(a / (eps - b)) : 0.25 * M_PI;
    auto energy = [&](double t) {
      const double c = cos(t), s = sin(t);
      return eps * c * c + b * s * s + a * s * c;
    };
    if (energy(th + 0.5 * M_PI) < energy(th)) th += 0.5 * M_PI;
    cs[0] = cos(th);
    cs[1] = sin(th);
  }
  __syncthreads();
  const double c = cs[0], s = cs[1];
  double w[2] = {0.0, 0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const c128 x = c128{psi[g].x * c + N[g].x * s, psi[g].y * c + N[g].y * s};
    const c128 hx = c128{hpsi[g].x * c + HN[g].x * s, hpsi[g].y * c + HN[g].y * s};
    psi[g] = x;
    hpsi[g] = hx;
    c128 sx = x;
    if (US) {
      sx = c128{spsi[g].x * c + SN[g].x * s, spsi[g].y * c + SN[g].y * s};
      spsi[g] = sx;
    }
    w[0] += wt<GAM>(g) * (x.x * hx.x + x.y * hx.y);
    w[1] += wt<GAM>(g) * (x.x * sx.x + x.y * sx.y);
  }
  block_sums<2>(w, red);
  const double e = w[0] / w[1];
  double r[1] = {0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const c128 sx = US ? spsi[g] : psi[g];
    const double re = hpsi[g].x - e * sx.x, im = hpsi[g].y - e * sx.y;
    r[0] += wt<GAM>(g) * (re * re + im * im);
  }
  block_sums<1>(r, red);
  if (threadIdx.x == 0) {
    const double rn = sqrt(r[0]);
    sc->deps = fabs(e - sc->eps);
    sc->eps = e;
    sc->resid = rn;
    sc->conv = (rn <= tol_r && sc->deps <= tol_e) ? 1 : 0;
    if (!isfinite(rn) || !isfinite(e)) sc->conv = -1;
  }
}

// x <- x / ||x||; at Gamma the imaginary part of x(G = 0) is set to zero first
template <bool GAM>
__global__ void __launch_bounds__(CT) k_cg_normalize(int npw, c128* __restrict__ x) {
  __shared__ double red[16];
  double v[1] = {0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    if (GAM && g == 0) x[0].y = 0.0;   // the thread that owns g = 0 reads it back below
    v[0] += wt<GAM>(g) * (x[g].x * x[g].x + x[g].y * x[g].y);
  }
  block_sums<1>(v, red);
  const double inv = v[0] > 0.0 ? 1.0 / sqrt(v[0]) : 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) x[g] = c128{x[g].x * inv, x[g].y * inv};
}

// x <- x / <x|S x>^(1/2) and S x likewise (at Gamma the whole-sphere product;
// x(G = 0) and S x(G = 0) are real there)
template <bool GAM>
__global__ void __launch_bounds__(CT) k_cg_snormalize(int npw, c128* __restrict__ x, c128* __restrict__ sx) {
  __shared__ double red[16];
  double v[1] = {0.0};
  for (int g = threadIdx.x; g < npw; g += blockDim.x) v[0] += wt<GAM>(g) * (x[g].x * sx[g].x + x[g].y * sx[g].y);
  block_sums<1>(v, red);
  const double inv = v[0] > 0.0 ? 1.0 / sqrt(v[0]) : 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    x[g] = c128{x[g].x * inv, x[g].y * inv};
    sx[g] = c128{sx[g].x * inv, sx[g].y * inv};
  }
}

}  // namespace

struct CgWork {
  int ld = 0;
  c128 *psi = nullptr, *hpsi = nullptr, *G = nullptr, *Gp = nullptr, *D = nullptr, *N = nullptr, *HN = nullptr;
  c128 *spsi = nullptr, *SN = nullptr, *SX = nullptr;   // S psi, S N, S x of a projection (S != 1 only)
  c128* coef = nullptr;          // [nb_max] projections on the bands already found
  CgScalars* sc = nullptr;       // device
  CgScalars* hsc = nullptr;      // pinned host
  void* part = nullptr;
  size_t part_bytes = 0;
  std::vector<void*> allocs;
};

size_t pw::cg_bytes(int npw, int nb_max) {
  const size_t ld = ((size_t)npw + 15) / 16 * 16;
  return 10 * ld * sizeof(c128) + (size_t)nb_max * sizeof(c128) + 4096 +
         std::max(pw::splitk_part_bytes(nb_max, 1, npw, sizeof(c128)), pw::dgemm_part_bytes(nb_max, 1));
}

pw_status pw::cg_alloc(pw_plan p) {
  CgWork* W = new CgWork();
  p->cg = W;
  W->ld = (p->npw + 15) / 16 * 16;
  auto get = [&](size_t bytes, void** out) -> pw_status {
    PW_TRY(pw::dev_alloc(p, std::max<size_t>(bytes, 256), out));
    W->allocs.push_back(*out);
    return PW_OK;
  };
  const size_t vb = (size_t)W->ld * sizeof(c128);
  for (c128** v : {&W->psi, &W->hpsi, &W->G, &W->Gp, &W->D, &W->N, &W->HN, &W->spsi, &W->SN, &W->SX})
    PW_TRY(get(vb, (void**)v));
  PW_TRY(get((size_t)p->opts.nb_max * sizeof(c128), (void**)&W->coef));
  PW_TRY(get(sizeof(CgScalars), (void**)&W->sc));
  W->part_bytes = std::max(pw::splitk_part_bytes(p->opts.nb_max, 1, p->npw, sizeof(c128)),
                           pw::dgemm_part_bytes(p->opts.nb_max, 1));
  PW_TRY(get(W->part_bytes, &W->part));
  void* h = nullptr;
  PW_TRY(pw::host_alloc(p, sizeof(CgScalars), &h));
  W->hsc = static_cast<CgScalars*>(h);
  return PW_OK;
}

void pw::cg_free(pw_plan p) {
  CgWork* W = p->cg;
  if (!W) return;
  for (void* q : W->allocs) pw::dev_free(p, q);
  pw::host_free(p, W->hsc);
  delete W;
  p->cg = nullptr;
}

extern "C" void pw_cg_opts_default(pw_cg_opts* o) {
  if (!o) return;
  o->max_iter = 400;
  o->tol_resid = 1e-6;
  o->tol_deig = 5e-9;
  o->precond_floor = 0.2;
}

namespace {
// x -= Psi (Psi^H S x) for the i S-orthonormal bands in Psi (column-major, ldq);
// at Gamma the projections are the real whole-sphere products 2 sum - (G = 0 term)
pw_status orth_lower(pw_plan p, CgWork& W, int i, const c128* Psi, int ldq, c128* x, hipStream_t st) {
  if (i == 0) return PW_OK;
  const c128* sx = x;
  if (p->us) {
    PW_TRY(pw::spsi_launch(p, PW_FP64, 1, x, W.ld, W.SX, W.ld, st));
    sx = W.SX;
  }
  if (p->gamma)
    PW_TRY((pw::dgemm_tn<double, double, double>(i, 1, 2 * p->npw, reinterpret_cast<const double*>(Psi), 2L * ldq,
                                                 reinterpret_cast<const double*>(sx), 2L * W.ld, 1.0, 1.0, 0.0,
                                                 reinterpret_cast<double*>(W.coef), i, true, W.part, W.part_bytes,
                                                 st)));
  else
    PW_TRY((pw::zgemm_cn<double, double, double>(i, 1, p->npw, Psi, ldq, sx, W.ld, W.coef, i, W.part,
                                                 W.part_bytes, st)));
  PW_TRY((pw::zgemm_nn<double, double, double>(p->npw, 1, i, -1.0, Psi, ldq, W.coef, i, 1.0, x, W.ld, st)));
  return PW_OK;
}

// psi normalized in the S metric; S psi in W.spsi when S != 1
pw_status normalize(pw_plan p, CgWork& W, hipStream_t st) {
  if (p->us) {
    if (p->gamma) k_cg_normalize<true><<<1, CT, 0, st>>>(p->npw, W.psi);   // real psi(0) before S psi
    PW_TRY(pw::spsi_launch(p, PW_FP64, 1, W.psi, W.ld, W.spsi, W.ld, st));
    if (p->gamma)
      k_cg_snormalize<true><<<1, CT, 0, st>>>(p->npw, W.psi, W.spsi);
    else
      k_cg_snormalize<false><<<1, CT, 0, st>>>(p->npw, W.psi, W.spsi);
  } else if (p->gamma) {
    k_cg_normalize<true><<<1, CT, 0, st>>>(p->npw, W.psi);
  } else {
    k_cg_normalize<false><<<1, CT, 0, st>>>(p->npw, W.psi);
  }
  PW_HIP(hipGetLastError());
  return PW_OK;
}

// one CG step of band i: gradient, its projection on the bands found, the
// conjugate direction, H N (and S N), the line minimization
template <bool US, bool GAM>
pw_status cg_step(pw_plan p, CgWork& W, int i, const c128* out, int ldpsi, const pw_cg_opts& o, hipStream_t st) {
  const int npw = p->npw;
  k_cg_grad<GAM><<<1, CT, 0, st>>>(npw, US ? W.spsi : W.psi, W.hpsi, p->kin, o.precond_floor, W.G, W.sc);
  PW_TRY(orth_lower(p, W, i, out, ldpsi, W.G, st));
  k_cg_dir<US, GAM><<<1, CT, 0, st>>>(npw, W.psi, US ? W.spsi : W.psi, W.G, W.Gp, W.D, W.N, W.sc);
  if (US) {
    PW_TRY(pw::spsi_launch(p, PW_FP64, 1, W.N, W.ld, W.SN, W.ld, st));
    k_cg_snormalize<GAM><<<1, CT, 0, st>>>(npw, W.N, W.SN);
  }
  PW_TRY(pw::hpsi_launch(p, PW_FP64, 1, W.N, W.ld, W.HN, W.ld, st));
  k_cg_rotate<US, GAM><<<1, CT, 0, st>>>(npw, W.psi, W.hpsi, US ? W.spsi : nullptr, W.N, W.HN,
                                         US ? W.SN : nullptr, o.tol_resid, o.tol_deig, W.sc);
  PW_HIP(hipGetLastError());
  return PW_OK;
}
}  // namespace

extern "C" pw_status pcg_solve(pw_plan p, int32_t nb, pw_c128* psi_u, int32_t ldpsi, double* eig, double* resid,
                               const pw_cg_opts* o_, pw_cg_stats* stats_out, void* stream) {
  PW_CHECK(p != nullptr, PW_EINVAL, "NULL plan");
  PW_CHECK(p->cg != nullptr, PW_EINVAL, "plan was created without solver workspace (ndim_max = 0)");
  pw_cg_opts o;
  if (o_) o = *o_; else pw_cg_opts_default(&o);
  PW_CHECK(nb >= 1 && nb <= p->opts.nb_max, PW_EINVAL, "nb out of range [1, nb_max]");
  PW_CHECK(nb <= p->npw, PW_EINVAL, "nb > npw");
  PW_CHECK(o.max_iter >= 1, PW_EINVAL, "max_iter < 1");
  PW_CHECK(o.precond_floor > 0.0, PW_EINVAL, "precond_floor must be positive");
  PW_CHECK(psi_u && eig && resid, PW_EINVAL, "NULL psi, eig or resid");
  PW_CHECK(ldpsi >= p->npw, PW_EINVAL, "ldpsi < npw");
  PW_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  CgWork& W = *p->cg;
  c128* out = reinterpret_cast<c128*>(psi_u);
  const int npw = p->npw;
  const bool us = p->us, gam = p->gamma;
  const size_t pitch = sizeof(c128) * npw;
  pw_cg_stats stats{};
  pw_status result = PW_OK;
  for (int i = 0; i < nb; ++i) {
    // trial vector: the input band, orthonormalized against the bands found
    PW_HIP(hipMemcpyAsync(W.psi, out + (size_t)i * ldpsi, pitch, hipMemcpyDeviceToDevice, st));
    PW_TRY(orth_lower(p, W, i, out, ldpsi, W.psi, st));
    PW_TRY(orth_lower(p, W, i, out, ldpsi, W.psi, st));
    PW_TRY(normalize(p, W, st));
    PW_TRY(pw::hpsi_launch(p, PW_FP64, 1, W.psi, W.ld, W.hpsi, W.ld, st));
    if (gam)
      k_cg_start<true><<<1, CT, 0, st>>>(npw, W.psi, W.hpsi, W.sc);
    else
      k_cg_start<false><<<1, CT, 0, st>>>(npw, W.psi, W.hpsi, W.sc);
    PW_HIP(hipGetLastError());
    int it = 0;
    bool conv = false;
    for (; it < o.max_iter; ) {
      auto step = us ? (gam ? cg_step<true, true> : cg_step<true, false>)
                     : (gam ? cg_step<false, true> : cg_step<false, false>);
      PW_TRY(step(p, W, i, out, ldpsi, o, st));
      ++it;
      PW_HIP(hipMemcpyAsync(W.hsc, W.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, st));
      PW_HIP(hipStreamSynchronize(st));
      if (W.hsc->conv < 0) {
        result = pw::fail(PW_ENAN, "non-finite energy or residual norm in band " + std::to_string(i));
        break;
      }
      if (W.hsc->conv == 1) { conv = true; break; }
      if (p->cancel.exchange(0)) {
        result = pw::fail(PW_ECANCELLED, "solve cancelled (pw_cancel)");
        break;
      }
    }
    if (result != PW_OK) break;
    // the band joins the found ones, S-orthogonal to them and S-normalized
    PW_TRY(orth_lower(p, W, i, out, ldpsi, W.psi, st));
    PW_TRY(normalize(p, W, st));
    PW_HIP(hipMemcpyAsync(out + (size_t)i * ldpsi, W.psi, pitch, hipMemcpyDeviceToDevice, st));
    stats.iters += it;
    stats.max_band_iters = std::max(stats.max_band_iters, it);
    stats.nconv += conv ? 1 : 0;
  }
  if (result == PW_OK) {
    // final float64 verification of the whole block
    PW_TRY(pw::final_check(p, nb, out, ldpsi, eig, resid, st));
    std::vector<double> hr(nb);
    PW_HIP(hipMemcpyAsync(hr.data(), resid, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    for (double r : hr) stats.max_resid = std::max(stats.max_resid, r);
    if (stats.nconv < nb) result = PW_ENOTCONV;
  }
  if (stats_out) *stats_out = stats;
  p->cancel.store(0);
  return result;
}
