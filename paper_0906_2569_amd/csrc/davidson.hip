// Block Davidson for the nb lowest eigenpairs of the plane-wave Hamiltonian
// (the iterative-diagonalization appendix, S = 1):
//
//   start: Rayleigh-Ritz on the trial block (orthonormalizes it and gives
//          eps_i = <psi_i|H|psi_i>);
//   loop:  residuals g_i = H psi_i - eps_i psi_i and their float64 norms;
//          bands with ||g_i|| <= tol_resid and |d eps_i| <= tol_deig are
//          converged; for the others the corrections
//          dpsi_i(G) = g_i(G) / (h_diag(G) - eps_i)   (diagonal preconditioner,
//          denominator smoothly bounded below) are normalized and appended;
//          the reduced problem H_jk c = eps S_jk c on phi (new rows and columns
//          only) is solved in float64 on the GPU, and psi = phi c, H psi = H phi c.
//          The basis grows until ndim*nb (expanding-basis variant), then
//          collapses onto the current Ritz vectors.
//   end:   a float64 H.psi of the final block recomputes eps_i and ||g_i||.
//
// In mixed precision, H.psi runs in float32 and only bands with ||g_i|| above
// ladder_switch are corrected; once every band is below it (or the largest
// residual stalls), the basis restarts from the Ritz vectors with float64
// H.psi (precision ladder).  Reduced matrices, Cholesky, the reduced
// eigenproblem and residual norms are always float64.
#include <algorithm>
#include <cmath>
#include <vector>

#include "linalg.h"

struct DavFlags {
  int n_new;
  int nan;
  int info;
  int nconv;
  double maxr;
  double gamma;   // growth factor of the last Ritz rotation
};

struct DavWork {
  int nbmax = 0, ndim = 0, nbasis = 0, ld = 0;
  c128 *phi = nullptr, *hphi = nullptr, *psi = nullptr, *hpsi = nullptr;
  c128 *sphi = nullptr, *spsi = nullptr;   // S phi, S psi (ultrasoft plans only)
  c128 *hred = nullptr, *sred = nullptr, *cvec = nullptr;
  double *eps = nullptr, *eps_prev = nullptr, *rn = nullptr;
  int* idx = nullptr;
  int* perm = nullptr;       // [nb] band order (locking, final sort)
  c128* lockc = nullptr;     // [nb][nb] overlaps of locked bands with new corrections
  double* creal = nullptr;   // Gamma: real parts of the Ritz coefficients [nb][nbasis]
  double* etmp = nullptr;    // [2 nb] staging of permuted values
  DavFlags* flags = nullptr;     // device
  DavFlags* hflags = nullptr;    // pinned host
  void* part = nullptr;
  size_t part_bytes = 0;
  pw::HeigWork hw;
  std::vector<void*> allocs;
};

namespace {

// threads per workgroup of the per-band vector kernels (one workgroup per
// band streams npw entries: more waves keep more loads in flight)
constexpr int kVecThreads = 1024;

// sum over the workgroup (any size up to 1024; red[] holds one value per wave)
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Weight of half-sphere entry g in full-sphere sums at Gamma (gam = 1): the
// entry stands for G and -G, except G = 0 at index 0
__device__ __forceinline__ double gw(int gam, int g) { return (gam && g > 0) ? 2.0 : 1.0; }

// rn[b] = || hpsi_b - eps_b spsi_b ||_2  (spsi = psi when S = 1)
__global__ void __launch_bounds__(kVecThreads) k_resid(int npw, const c128* __restrict__ psi,
                                               const c128* __restrict__ hpsi, int ld,
                                               const double* __restrict__ eps, double* __restrict__ rn, int gam = 0) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  const double e = eps[b];
  const c128* x = psi + (size_t)b * ld;
  const c128* hx = hpsi + (size_t)b * ld;
  double s = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double re = hx[g].x - e * x[g].x, im = hx[g].y - e * x[g].y;
    s += gw(gam, g) * (re * re + im * im);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) rn[b] = sqrt(s);
}

// convergence flags, compaction of the unconverged bands (band order), NaN
// guard, and the reduced-solver status, gathered for one host read.  One
// wave takes the bands 64 at a time in order; the unconverged ones of a chunk
// get consecutive idx positions from a ballot prefix count.
__global__ void __launch_bounds__(64) k_select(int nb, const double* __restrict__ rn,
                                               const double* __restrict__ eps,
                                               const double* __restrict__ eps_prev, double tol_r, double tol_e,
                                               int* __restrict__ idx, const int* __restrict__ info,
                                               const double* __restrict__ gamma, DavFlags* __restrict__ f) {
  const int lane = threadIdx.x;
  if (blockIdx.x != 0 || lane >= 64) return;
  int n = 0, nconv = 0;
  bool nan = false;
  double maxr = 0.0;
  for (int b0 = 0; b0 < nb; b0 += 64) {
    const int b = b0 + lane;
    const bool act = b < nb;
    bool conv = false, bad = false;
    if (act) {
      const double r = rn[b], de = fabs(eps[b] - eps_prev[b]);
      bad = !isfinite(r) || !isfinite(eps[b]);
      maxr = fmax(maxr, r);
      conv = r <= tol_r && de <= tol_e;
    }
    const unsigned long long open = __ballot(act && !conv);
    if (act && !conv) idx[n + __popcll(open & ((1ull << lane) - 1ull))] = b;
    n += __popcll(open);
    nconv += __popcll(__ballot(act && conv));
    nan = nan || __ballot(bad) != 0ull;
  }
  for (int o = 32; o > 0; o >>= 1) maxr = fmax(maxr, __shfl_xor(maxr, o, 64));
  if (lane == 0) {
    f->n_new = n;
    f->nan = nan ? 1 : 0;
    f->info = *info;
    f->nconv = nconv;
    f->maxr = maxr;
    f->gamma = *gamma;
  }
}

// out_t = (hpsi_b - eps_b spsi_b) / smax(h_diag - eps_b s_diag, floor), normalized; b = idx[t]
// (spsi: S psi, or psi when S = 1; sdiag: diagonal of S, or nullptr for 1)
__global__ void __launch_bounds__(kVecThreads) k_correct(int npw, const int* __restrict__ idx,
                                                 const c128* __restrict__ psi, const c128* __restrict__ hpsi,
                                                 int ld, const double* __restrict__ eps,
                                                 const double* __restrict__ hdiag, const double* __restrict__ sdiag,
                                                 double floor_, c128* __restrict__ out, int ldo, int gam = 0) {
  __shared__ double red[16];
  const int t = blockIdx.x;
  const int b = idx[t];
  const double e = eps[b];
  const c128* x = psi + (size_t)b * ld;
  const c128* hx = hpsi + (size_t)b * ld;
  c128* o = out + (size_t)t * ldo;
  double s = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    // diagonal of H - eps, replaced by its smooth maximum with floor_: equal
    // to it far above floor_, positive and >= floor_/2 everywhere
    const double dg = hdiag[g] - e * (sdiag ? sdiag[g] : 1.0);
    const double den = 0.5 * (dg + floor_ + sqrt((dg - floor_) * (dg - floor_) + floor_ * floor_));
    const double inv = 1.0 / den;
    const c128 r = c128{(hx[g].x - e * x[g].x) * inv, (hx[g].y - e * x[g].y) * inv};
    o[g] = r;
    s += gw(gam, g) * (r.x * r.x + r.y * r.y);
  }
  s = block_sum(s, red);
  const double sc = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) o[g] = c128{o[g].x * sc, o[g].y * sc};
}

// out_t = hpsi_b - eps_b psi_b, b = idx[t] (residual vectors, for projection before preconditioning)
__global__ void __launch_bounds__(kVecThreads) k_residvec(int npw, const int* __restrict__ idx,
                                                  const c128* __restrict__ psi, const c128* __restrict__ hpsi,
                                                  int ld, const double* __restrict__ eps, c128* __restrict__ out,
                                                  int ldo) {
  const int b = idx[blockIdx.x];
  const double e = eps[b];
  const c128* x = psi + (size_t)b * ld;
  const c128* hx = hpsi + (size_t)b * ld;
  c128* o = out + (size_t)blockIdx.x * ldo;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) o[g] = c128{hx[g].x - e * x[g].x, hx[g].y - e * x[g].y};
}

// column t of x <- x_t / smax(h_diag - eps_b, floor), b = idx[t], normalized (as k_correct)
__global__ void __launch_bounds__(kVecThreads) k_precond(int npw, const int* __restrict__ idx,
                                                 const double* __restrict__ eps, const double* __restrict__ hdiag,
                                                 const double* __restrict__ sdiag, double floor_,
                                                 c128* __restrict__ x, int ldx, int gam = 0) {
  __shared__ double red[16];
  const double e = eps[idx[blockIdx.x]];
  c128* o = x + (size_t)blockIdx.x * ldx;
  double s = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double dg = hdiag[g] - e * (sdiag ? sdiag[g] : 1.0);
    const double den = 0.5 * (dg + floor_ + sqrt((dg - floor_) * (dg - floor_) + floor_ * floor_));
    const double inv = 1.0 / den;
    const c128 r = c128{o[g].x * inv, o[g].y * inv};
    o[g] = r;
    s += gw(gam, g) * (r.x * r.x + r.y * r.y);
  }
  s = block_sum(s, red);
  const double sc = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) o[g] = c128{o[g].x * sc, o[g].y * sc};
}

// columns of x scaled to unit norm (a zero column stays zero)
__global__ void __launch_bounds__(kVecThreads) k_normalize(int npw, c128* __restrict__ x, int ld, int gam = 0) {
  __shared__ double red[16];
  c128* o = x + (size_t)blockIdx.x * ld;
  double s = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) s += gw(gam, g) * (o[g].x * o[g].x + o[g].y * o[g].y);
  s = block_sum(s, red);
  const double sc = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) o[g] = c128{o[g].x * sc, o[g].y * sc};
}

// reduced matrices of the collapsed basis {psi}: H = diag(eps), S = I
__global__ void k_restart(int nb, const double* __restrict__ eps, c128* __restrict__ h,
                          c128* __restrict__ s, int ldm) {
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nb * nb; idx += gridDim.x * blockDim.x) {
    const int i = idx % nb, j = idx / nb;
    h[(size_t)j * ldm + i] = c128{i == j ? eps[i] : 0.0, 0.0};
    s[(size_t)j * ldm + i] = c128{i == j ? 1.0 : 0.0, 0.0};
  }
}

// columns [c0, c1) were computed for rows [0, c1): mirror them into rows
// [c0, c1) of columns [0, c0), and make the new diagonal block exactly Hermitian
// (blockIdx.y selects the matrix: m0 or m1, one launch for H and S)
__global__ void k_herm_fill(int c0, int c1, c128* __restrict__ m0, c128* __restrict__ m1, int ldm) {
  c128* __restrict__ m = blockIdx.y ? m1 : m0;
  const int nn = c1 - c0;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nn * c1; idx += gridDim.x * blockDim.x) {
    const int i = c0 + idx % nn;   // new row
    const int j = idx / nn;        // column in [0, c1)
    if (j < c0) {
      const c128 v = m[(size_t)i * ldm + j];
      m[(size_t)j * ldm + i] = c128{v.x, -v.y};
    } else if (j < i) {
      const c128 up = m[(size_t)i * ldm + j];    // (j, i), j < i: upper
      const c128 lo = m[(size_t)j * ldm + i];    // (i, j): lower
      const c128 a = c128{0.5 * (up.x + lo.x), 0.5 * (up.y - lo.y)};   // average of up and conj(lo)
      m[(size_t)i * ldm + j] = a;
      m[(size_t)j * ldm + i] = c128{a.x, -a.y};
    } else if (j == i) {
      m[(size_t)i * ldm + i].y = 0.0;
    }
  }
}

// out[j][i] = Re c[j][i] (columns of leading dimension ld), i < n, j < m
__global__ void k_real_part(int n, int m, const c128* __restrict__ c, int ld, double* __restrict__ out) {
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * m; idx += gridDim.x * blockDim.x) {
    const int i = idx % n, j = idx / n;
    out[(size_t)j * ld + i] = c[(size_t)j * ld + i].x;
  }
}

// Im x_j(G = 0) = 0 for the n columns (Gamma: the coefficient of G = 0 is real)
__global__ void k_zero_im0(int n, c128* __restrict__ x, int ld) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) x[(size_t)j * ld].y = 0.0;
}

__global__ void k_fill(int n, double v, double* __restrict__ x) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = v;
}

// Locking: order of the active bands [nl, nb) with the converged ones first and
// the n_new unconverged ones (idx, ascending) after them, both in band order;
// eps follows that order, and idx is renumbered to the new positions.
__global__ void k_lock_order(int nl, int nb, int n_new, int* __restrict__ idx, int* __restrict__ perm,
                             double* __restrict__ eps, double* __restrict__ etmp) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int nact = nb - nl, nc = nact - n_new;
  int c = 0, u = 0;
  for (int b = nl; b < nb; ++b) {
    if (u < n_new && idx[u] == b) perm[nc + u++] = b;
    else perm[c++] = b;
  }
  for (int j = 0; j < nact; ++j) etmp[j] = eps[perm[j]];
  for (int j = 0; j < nact; ++j) eps[nl + j] = etmp[j];
  for (int t = 0; t < n_new; ++t) idx[t] = nl + nc + t;
}

// dst column j = src column perm[j], j < n (complex columns of length npw)
__global__ void k_gather_cols(int npw, int n, const int* __restrict__ perm, const c128* __restrict__ src, int lds,
                              c128* __restrict__ dst, int ldd) {
  for (int j = blockIdx.y; j < n; j += gridDim.y) {
    const c128* a = src + (size_t)perm[j] * lds;
    c128* b = dst + (size_t)j * ldd;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < npw; g += gridDim.x * blockDim.x) b[g] = a[g];
  }
}

// x[j] = x[perm[j]] for j < n (through tmp)
__global__ void k_permute_vals(int n, const int* __restrict__ perm, double* __restrict__ x,
                               double* __restrict__ tmp) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int j = 0; j < n; ++j) tmp[j] = x[perm[j]];
  for (int j = 0; j < n; ++j) x[j] = tmp[j];
}

// eig_b = Re <psi_b|H psi_b> / <psi_b|S psi_b>,  resid_b = || H psi_b - eig_b S psi_b ||
// (spsi = nullptr: S = 1)
__global__ void __launch_bounds__(256) k_final(int npw, const c128* __restrict__ psi, int ldpsi,
                                               const c128* __restrict__ hpsi, int ldh,
                                               double* __restrict__ eig, double* __restrict__ resid,
                                               const c128* __restrict__ spsi = nullptr, int gam = 0) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  const c128* x = psi + (size_t)b * ldpsi;
  const c128* hx = hpsi + (size_t)b * ldh;
  const c128* sx = spsi ? spsi + (size_t)b * ldh : x;
  double num = 0.0, den = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    num += gw(gam, g) * (x[g].x * hx[g].x + x[g].y * hx[g].y);
    den += gw(gam, g) * (x[g].x * sx[g].x + x[g].y * sx[g].y);
  }
  num = block_sum(num, red);
  den = block_sum(den, red);
  const double e = num / den;
  double s = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    const double re = hx[g].x - e * sx[g].x, im = hx[g].y - e * sx[g].y;
    s += gw(gam, g) * (re * re + im * im);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    eig[b] = e;
    resid[b] = sqrt(s);
  }
}

}  // namespace

size_t pw::dav_bytes(int npw, int nb_max, int ndim_max) {
  const size_t ld = ((size_t)npw + 15) / 16 * 16;
  const size_t nbasis = (size_t)nb_max * ndim_max;
  size_t b = 0;
  b += 2 * nbasis * ld * sizeof(c128);                  // phi, hphi
  b += 2 * (size_t)nb_max * ld * sizeof(c128);          // psi, hpsi
  b += (nbasis + nb_max) * ld * sizeof(c128);           // S phi, S psi (upper bound: ultrasoft plans)
  b += 2 * nbasis * nbasis * sizeof(c128);              // hred, sred
  b += nbasis * nb_max * sizeof(c128);                  // cvec
  b += 5 * (size_t)nb_max * sizeof(double) + 2 * nb_max * sizeof(int) + 256;
  b += (size_t)nb_max * nb_max * sizeof(c128);          // lockc
  b += nbasis * nb_max * sizeof(double);                // real Ritz coefficients (Gamma)
  b += std::max(pw::splitk_part_bytes((int)nbasis, (int)nbasis, npw, sizeof(c128)),
                pw::dgemm_part_bytes((int)nbasis, (int)nbasis));
  b += pw::heig_work_bytes((int)nbasis);
  return b + 32 * 256;
}

pw_status pw::dav_alloc(pw_plan p) {
  PW_TRY(pw::heig_set_limits());
  DavWork* W = new DavWork();
  p->dav = W;
  W->nbmax = p->opts.nb_max;
  W->ndim = p->opts.ndim_max;
  W->nbasis = W->nbmax * W->ndim;
  W->ld = (p->npw + 15) / 16 * 16;
  auto get = [&](size_t bytes, void** out) -> pw_status {
    PW_TRY(pw::dev_alloc(p, std::max<size_t>(bytes, 256), out));
    W->allocs.push_back(*out);
    return PW_OK;
  };
  const size_t nbx = W->nbasis, ld = W->ld, nb = W->nbmax;
  PW_TRY(get(nbx * ld * sizeof(c128), (void**)&W->phi));
  PW_TRY(get(nbx * ld * sizeof(c128), (void**)&W->hphi));
  PW_TRY(get(nb * ld * sizeof(c128), (void**)&W->psi));
  PW_TRY(get(nb * ld * sizeof(c128), (void**)&W->hpsi));
  if (p->us) {
    PW_TRY(get(nbx * ld * sizeof(c128), (void**)&W->sphi));
    PW_TRY(get(nb * ld * sizeof(c128), (void**)&W->spsi));
  }
  PW_TRY(get(nbx * nbx * sizeof(c128), (void**)&W->hred));
  PW_TRY(get(nbx * nbx * sizeof(c128), (void**)&W->sred));
  PW_TRY(get(nbx * nb * sizeof(c128), (void**)&W->cvec));
  PW_TRY(get(nb * sizeof(double), (void**)&W->eps));
  PW_TRY(get(nb * sizeof(double), (void**)&W->eps_prev));
  PW_TRY(get(nb * sizeof(double), (void**)&W->rn));
  PW_TRY(get(nb * sizeof(int), (void**)&W->idx));
  PW_TRY(get(nb * sizeof(int), (void**)&W->perm));
  PW_TRY(get(nb * nb * sizeof(c128), (void**)&W->lockc));
  if (p->gamma) PW_TRY(get(nbx * nb * sizeof(double), (void**)&W->creal));
  PW_TRY(get(2 * nb * sizeof(double), (void**)&W->etmp));
  PW_TRY(get(sizeof(DavFlags), (void**)&W->flags));
  W->part_bytes = std::max(pw::splitk_part_bytes((int)nbx, (int)nbx, p->npw, sizeof(c128)),
                           pw::dgemm_part_bytes((int)nbx, (int)nbx));
  PW_TRY(get(W->part_bytes, &W->part));
  void* hwb = nullptr;
  PW_TRY(get(pw::heig_work_bytes((int)nbx), &hwb));
  PW_TRY(pw::heig_setup(W->hw, hwb, (int)nbx));
  void* hf = nullptr;
  PW_TRY(pw::host_alloc(p, sizeof(DavFlags), &hf));
  W->hflags = static_cast<DavFlags*>(hf);
  return PW_OK;
}

bool pw::dav_set_coop(pw_plan p, bool ok, bool wide) {
  if (!p || !p->dav) return false;
  const bool prev = p->dav->hw.coop_ok;
  p->dav->hw.coop_ok = ok;
  p->dav->hw.coop_wide = wide;
  return prev;
}

bool pw::dav_get_coop(pw_plan p) { return p && p->dav && p->dav->hw.coop_ok; }

void pw::dav_free(pw_plan p) {
  DavWork* W = p->dav;
  if (!W) return;
  for (void* q : W->allocs) pw::dev_free(p, q);
  pw::host_free(p, W->hflags);
  delete W;
  p->dav = nullptr;
}

namespace {

// largest accumulated error growth of H phi tolerated before H is re-applied
// (float64 / float32 stage)
constexpr double kMaxAmp = 1e4;
constexpr double kMaxAmp32 = 1e2;
// float32 stage: once max ||g_i|| is within kStallZone of ladder_switch,
// kStall32 iterations without it halving end the stage (the float32 noise
// floor lies above ladder_switch)
constexpr double kStallZone = 100.0;
constexpr int kStall32 = 12;
// rotation work (16 npw nb^2 flops) from which sub32 = 1 takes float32 rotations
constexpr double kSub32MinFlops = 1e11;

struct Solver {
  pw_plan p;
  DavWork& W;
  hipStream_t st;
  pw_david_stats& stats;
  int nfact = 0;   // leading basis size whose overlap factor is current
  int nl = 0;      // locked bands: psi[0:nl), hpsi[0:nl), eps[0:nl) stay fixed
  bool sub32 = false;   // Ritz rotations in float32 arithmetic (float32 stage)

  // The projections stay float64 in every stage: an overlap matrix from
  // float32 products (entry errors of about 5e-7 at npw 191k) breaks the
  // dependence test of the incremental Cholesky, whose inverse factor
  // multiplies those errors along K-long columns (a pivot of -4e-3 where a
  // tiny positive one belonged, at the 512-atom cell).  Only the collapsed
  // block's overlap, a near-identity, is formed from float32 products (see
  // collapse); its errors then enter the pivots unamplified, and a direction
  // counts as dependent below a relative pivot of 1e-5 instead of 1e-10.
  void set_sub32(bool on) {
    sub32 = on;
    W.hw.drop_tol = on ? 1e-5 : 1e-10;
  }

  // H x and, for ultrasoft plans, S x (columns at the same offsets in sphi)
  pw_status hpsi(pw_precision prec, int n, const c128* x, c128* hx, c128* sx = nullptr) {
    PW_TRY(pw::hpsi_launch(p, prec, n, x, W.ld, hx, W.ld, st));
    if (p->us && sx) PW_TRY(pw::spsi_launch(p, prec, n, x, W.ld, sx, W.ld, st));
    if (prec == PW_FP64) stats.n_hpsi_fp64 += n; else stats.n_hpsi_fp32 += n;
    return PW_OK;
  }

  // the vector the eigenvalue multiplies in the residual: S psi, or psi when S = 1
  const c128* spsi_or_psi() const { return p->us ? W.spsi : W.psi; }

  // reduced columns [c0, c1) of H and S over the basis phi[0:c1)
  pw_status project(int c0, int c1) {
    const int npw = p->npw, ldm = W.nbasis;
    // phi^H (H phi_new) and phi^H phi_new in one launch
    const c128* sb = (p->us ? W.sphi : W.phi) + (size_t)c0 * W.ld;
    if (p->gamma) {
      // real products over the interleaved half sphere: 2 sum - (G = 0 term)
      const double* ph = reinterpret_cast<const double*>(W.phi);
      const long l2 = 2L * W.ld;
      PW_TRY((pw::dgemm_tn<double, double, double>(c1, c1 - c0, 2 * npw, ph, l2,
                                                   reinterpret_cast<const double*>(W.hphi + (size_t)c0 * W.ld), l2,
                                                   1.0, 1.0, 0.0, reinterpret_cast<double*>(W.hred + (size_t)c0 * ldm),
                                                   ldm, true, W.part, W.part_bytes, st)));
      PW_TRY((pw::dgemm_tn<double, double, double>(c1, c1 - c0, 2 * npw, ph, l2, reinterpret_cast<const double*>(sb),
                                                   l2, 1.0, 1.0, 0.0,
                                                   reinterpret_cast<double*>(W.sred + (size_t)c0 * ldm), ldm, true,
                                                   W.part, W.part_bytes, st)));
    } else {
      PW_TRY(pw::zgemm_cn_pair(c1, c1 - c0, npw, W.phi, W.ld, W.hphi + (size_t)c0 * W.ld, sb,
                               W.ld, W.hred + (size_t)c0 * ldm, W.sred + (size_t)c0 * ldm, ldm, W.part,
                               W.part_bytes, st));
    }
    const int blocks = std::min(1024, ceil_div((size_t)(c1 - c0) * c1, 256));
    k_herm_fill<<<dim3(blocks, 2), 256, 0, st>>>(c0, c1, W.hred, W.sred, ldm);
    PW_HIP(hipGetLastError());
    return PW_OK;
  }

  // reduced eigenproblem on phi[0:nbase) for the nact active bands and the
  // Ritz rotation into psi[nl:nl+nact) (skipped on device when the overlap
  // matrix is not positive definite)
  pw_status rayleigh_ritz(int nbase, int nact) {
    const int ldm = W.nbasis;
    PW_TRY(pw::heig_solve(W.hw, nfact, nbase, nact, W.hred, W.sred, ldm, W.eps + nl, W.cvec, ldm, W.part,
                          W.part_bytes, st));
    nfact = nbase;
    if (p->gamma) {
      // real Ritz coefficients: psi = phi c and H psi = (H phi) c as real products of 2 npw rows
      k_real_part<<<std::min(1024, ceil_div(nbase * nact, 256)), 256, 0, st>>>(nbase, nact, W.cvec, ldm, W.creal);
      PW_HIP(hipGetLastError());
      const long l2 = 2L * W.ld;
      auto nn = sub32 ? pw::dgemm_nn<float, double, double> : pw::dgemm_nn<double, double, double>;
      PW_TRY(nn(2 * p->npw, nact, nbase, 1.0, reinterpret_cast<const double*>(W.phi), l2, W.creal, ldm, 0.0,
                reinterpret_cast<double*>(W.psi + (size_t)nl * W.ld), l2, st, W.hw.info, -1));
      PW_TRY(nn(2 * p->npw, nact, nbase, 1.0, reinterpret_cast<const double*>(W.hphi), l2, W.creal, ldm, 0.0,
                reinterpret_cast<double*>(W.hpsi + (size_t)nl * W.ld), l2, st, W.hw.info, -1));
      if (p->us)   // S psi = (S phi) c
        PW_TRY(nn(2 * p->npw, nact, nbase, 1.0, reinterpret_cast<const double*>(W.sphi), l2, W.creal, ldm, 0.0,
                  reinterpret_cast<double*>(W.spsi + (size_t)nl * W.ld), l2, st, W.hw.info, -1));
      return PW_OK;
    }
    // psi = phi c and hpsi = (H phi) c in one launch
    auto nn = sub32 ? pw::zgemm_nn_pair<float> : pw::zgemm_nn_pair<double>;
    PW_TRY(nn(p->npw, nact, nbase, W.phi, W.hphi, W.ld, W.cvec, ldm, W.psi + (size_t)nl * W.ld,
              W.hpsi + (size_t)nl * W.ld, W.ld, st, W.hw.info));
    if (p->us) {   // S psi = (S phi) c
      auto sn = sub32 ? pw::zgemm_nn<float, double, double> : pw::zgemm_nn<double, double, double>;
      PW_TRY(sn(p->npw, nact, nbase, 1.0, W.sphi, W.ld, W.cvec, ldm, 0.0, W.spsi + (size_t)nl * W.ld, W.ld, st,
                W.hw.info, nullptr, nullptr, 0));
    }
    return PW_OK;
  }

  // basis <- current Ritz vectors of the nact active bands
  pw_status collapse(int nact) {
    const size_t pitch = sizeof(c128) * W.ld;
    PW_HIP(hipMemcpy2DAsync(W.phi, pitch, W.psi + (size_t)nl * W.ld, pitch, sizeof(c128) * p->npw, nact,
                            hipMemcpyDeviceToDevice, st));
    PW_HIP(hipMemcpy2DAsync(W.hphi, pitch, W.hpsi + (size_t)nl * W.ld, pitch, sizeof(c128) * p->npw, nact,
                            hipMemcpyDeviceToDevice, st));
    if (p->us)
      PW_HIP(hipMemcpy2DAsync(W.sphi, pitch, W.spsi + (size_t)nl * W.ld, pitch, sizeof(c128) * p->npw, nact,
                              hipMemcpyDeviceToDevice, st));
    k_restart<<<std::min(1024, ceil_div(nact * nact, 256)), 256, 0, st>>>(nact, W.eps + nl, W.hred, W.sred,
                                                                          W.nbasis);
    PW_HIP(hipGetLastError());
    PW_TRY(pw::heig_reset(W.hw, nact, st));
    nfact = nact;
    if (sub32) {
      // Ritz vectors rotated with float32 products are orthonormal only to
      // about 1e-6, and that error would add up over collapses if the block
      // were taken as orthonormal: its overlap is formed explicitly instead
      // (H stays diag(eps): its error is of the order of the float32 stage's
      // own) and factored afresh
      const int ldm = W.nbasis;
      const c128* sb = p->us ? W.sphi : W.phi;
      if (p->gamma) {
        const long l2 = 2L * W.ld;
        PW_TRY((pw::dgemm_tn<float, double, double>(nact, nact, 2 * p->npw, reinterpret_cast<const double*>(W.phi),
                                                    l2, reinterpret_cast<const double*>(sb), l2, 1.0, 1.0, 0.0,
                                                    reinterpret_cast<double*>(W.sred), ldm, true, W.part,
                                                    W.part_bytes, st)));
      } else {
        PW_TRY((pw::zgemm_cn<float, double, double>(nact, nact, p->npw, W.phi, W.ld, sb, W.ld, W.sred, ldm, W.part,
                                                    W.part_bytes, st)));
      }
      const int blocks = std::min(1024, ceil_div((size_t)nact * nact, 256));
      k_herm_fill<<<dim3(blocks, 2), 256, 0, st>>>(0, nact, W.hred, W.sred, ldm);
      PW_HIP(hipGetLastError());
      nfact = 0;
    }
    return PW_OK;
  }

  // full Rayleigh-Ritz on a block already in phi[0:nact) (start, precision switch, rebuild)
  pw_status start_block(pw_precision prec, int nact) {
    nfact = 0;
    PW_TRY(hpsi(prec, nact, W.phi, W.hphi, W.sphi));
    PW_TRY(project(0, nact));
    PW_TRY(rayleigh_ritz(nact, nact));
    return PW_OK;
  }

  // lock the nc = nact - n_new converged active bands: they move to the front
  // of the active range (band order kept) and become psi[nl:nl+nc); idx then
  // lists the unconverged bands at their new positions
  pw_status lock(int nb, int n_new) {
    const int nact = nb - nl, nc = nact - n_new;
    if (nc <= 0) return PW_OK;
    const size_t pitch = sizeof(c128) * W.ld;
    const int npw = p->npw;
    k_lock_order<<<1, 1, 0, st>>>(nl, nb, n_new, W.idx, W.perm, W.eps, W.etmp);
    const dim3 g(std::min(64, ceil_div(npw, 256)), std::min(nact, 1024));
    k_gather_cols<<<g, 256, 0, st>>>(npw, nact, W.perm, W.psi, W.ld, W.phi, W.ld);
    k_gather_cols<<<g, 256, 0, st>>>(npw, nact, W.perm, W.hpsi, W.ld, W.hphi, W.ld);
    if (p->us) k_gather_cols<<<g, 256, 0, st>>>(npw, nact, W.perm, W.spsi, W.ld, W.sphi, W.ld);
    PW_HIP(hipGetLastError());
    PW_HIP(hipMemcpy2DAsync(W.psi + (size_t)nl * W.ld, pitch, W.phi, pitch, sizeof(c128) * npw, nact,
                            hipMemcpyDeviceToDevice, st));
    PW_HIP(hipMemcpy2DAsync(W.hpsi + (size_t)nl * W.ld, pitch, W.hphi, pitch, sizeof(c128) * npw, nact,
                            hipMemcpyDeviceToDevice, st));
    if (p->us)
      PW_HIP(hipMemcpy2DAsync(W.spsi + (size_t)nl * W.ld, pitch, W.sphi, pitch, sizeof(c128) * npw, nact,
                              hipMemcpyDeviceToDevice, st));
    nl += nc;
    return PW_OK;
  }

  // phi[c0:c0+n) <- (1 - psi_L psi_L^H) phi[c0:c0+n), `passes` times, each
  // pass followed by a normalization when `normalize` is set (a vector mostly
  // inside the locked span keeps, after one pass, rounding-level components
  // along it): no locked direction re-enters the basis
  // x -= Psi_l (Psi_l^H x) over `passes` passes (classical Gram-Schmidt
  // repeated: the second pass removes what rounding left after the first; it
  // needs no normalization in between), then unit columns if `normalize`.
  // With S != 1 the projector is 1 - Psi_l (S Psi_l)^H, which leaves x
  // S-orthogonal to the locked bands, or for a residual (`dual`, a vector of
  // the form (H - eps S) psi) its adjoint 1 - (S Psi_l) Psi_l^H
  pw_status project_out_locked(int c0, int n, int passes = 2, bool normalize = true, bool dual = false) {
    if (nl == 0 || n == 0) return PW_OK;
    c128* x = W.phi + (size_t)c0 * W.ld;
    if (p->us && !p->gamma) {
      const c128* cl = dual ? W.psi : W.spsi;   // the columns the coefficients take
      const c128* ul = dual ? W.spsi : W.psi;   // the columns the update takes
      for (int pass = 0; pass < passes; ++pass) {
        PW_TRY((pw::zgemm_cn<double, double, double>(nl, n, p->npw, cl, W.ld, x, W.ld, W.lockc, nl, W.part,
                                                     W.part_bytes, st)));
        PW_TRY((pw::zgemm_nn<double, double, double>(p->npw, n, nl, -1.0, ul, W.ld, W.lockc, nl, 1.0, x, W.ld,
                                                     st)));
      }
      if (normalize) k_normalize<<<n, kVecThreads, 0, st>>>(p->npw, x, W.ld, 0);
      PW_HIP(hipGetLastError());
      return PW_OK;
    }
    for (int pass = 0; pass < passes; ++pass) {
      if (p->gamma) {   // real products, S Psi_l in the same roles as above when S != 1
        const long l2 = 2L * W.ld;
        double* lc = reinterpret_cast<double*>(W.lockc);
        const c128* cl = p->us && !dual ? W.spsi : W.psi;
        const c128* ul = p->us && dual ? W.spsi : W.psi;
        PW_TRY((pw::dgemm_tn<double, double, double>(nl, n, 2 * p->npw, reinterpret_cast<const double*>(cl), l2,
                                                     reinterpret_cast<const double*>(x), l2, 1.0, 1.0, 0.0, lc, nl,
                                                     false, W.part, W.part_bytes, st)));
        PW_TRY((pw::dgemm_nn<double, double, double>(2 * p->npw, n, nl, -1.0, reinterpret_cast<const double*>(ul),
                                                     l2, lc, nl, 1.0, reinterpret_cast<double*>(x), l2, st)));
        continue;
      }
      PW_TRY((pw::zgemm_cn<double, double, double>(nl, n, p->npw, W.psi, W.ld, x, W.ld, W.lockc, nl, W.part,
                                                   W.part_bytes, st)));
      PW_TRY((pw::zgemm_nn<double, double, double>(p->npw, n, nl, -1.0, W.psi, W.ld, W.lockc, nl, 1.0, x, W.ld,
                                                   st)));
    }
    if (normalize) k_normalize<<<n, kVecThreads, 0, st>>>(p->npw, x, W.ld, p->gamma ? 1 : 0);
    PW_HIP(hipGetLastError());
    return PW_OK;
  }

  // corrections of the bands idx[0:n) into phi[c0:c0+n).  With locked bands
  // the residual is first projected off the locked span, so that the
  // preconditioner is applied to its active part only (the locked span's part
  // of a residual is the coupling that locking drops; preconditioned, it would
  // come back as a spurious direction), and the correction is projected again.
  pw_status corrections(int c0, int n, double floor_) {
    c128* x = W.phi + (size_t)c0 * W.ld;
    if (nl == 0) {
      k_correct<<<n, kVecThreads, 0, st>>>(p->npw, W.idx, spsi_or_psi(), W.hpsi, W.ld, W.eps, p->hdiag, p->sdiag,
                                           floor_, x, W.ld, p->gamma ? 1 : 0);
      PW_HIP(hipGetLastError());
      return PW_OK;
    }
    k_residvec<<<n, kVecThreads, 0, st>>>(p->npw, W.idx, spsi_or_psi(), W.hpsi, W.ld, W.eps, x, W.ld);
    PW_TRY(project_out_locked(c0, n, 1, false, true));
    k_precond<<<n, kVecThreads, 0, st>>>(p->npw, W.idx, W.eps, p->hdiag, p->sdiag, floor_, x, W.ld, p->gamma ? 1 : 0);
    PW_HIP(hipGetLastError());
    return project_out_locked(c0, n);
  }
};

}  // namespace

pw_status pw::final_check(pw_plan p, int nb, const c128* psi, int ldpsi, double* eig, double* resid,
                          hipStream_t st) {
  PW_CHECK(p->dav != nullptr, PW_EINVAL, "plan was created without solver workspace (ndim_max = 0)");
  DavWork& W = *p->dav;
  PW_CHECK(nb <= W.nbmax, PW_EINVAL, "nb > nb_max");
  PW_TRY(pw::hpsi_launch(p, PW_FP64, nb, psi, ldpsi, W.hpsi, W.ld, st));
  if (p->us) PW_TRY(pw::spsi_launch(p, PW_FP64, nb, psi, ldpsi, W.spsi, W.ld, st));
  k_final<<<nb, 256, 0, st>>>(p->npw, psi, ldpsi, W.hpsi, W.ld, eig, resid, p->us ? W.spsi : nullptr, p->gamma ? 1 : 0);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

extern "C" pw_status davidson_solve(pw_plan p, int32_t nb, pw_c128* psi_u, int32_t ldpsi, double* eig,
                                    double* resid, const pw_david_opts* o_, pw_david_stats* stats_out,
                                    void* stream) {
  PW_CHECK(p != nullptr, PW_EINVAL, "NULL plan");
  PW_CHECK(p->dav != nullptr, PW_EINVAL, "plan was created without Davidson workspace (ndim_max = 0)");
  pw_david_opts o;
  if (o_) o = *o_; else pw_david_opts_default(&o);
  DavWork& W = *p->dav;
  PW_CHECK(nb >= 1 && nb <= W.nbmax, PW_EINVAL, "nb out of range [1, nb_max]");
  PW_CHECK(nb <= p->npw, PW_EINVAL, "nb > npw");
  PW_CHECK(o.ndim >= 2 && o.ndim <= W.ndim, PW_EINVAL, "ndim out of range [2, ndim_max]");
  PW_CHECK(o.max_iter >= 0, PW_EINVAL, "max_iter < 0");
  PW_CHECK(o.precond_floor > 0.0, PW_EINVAL, "precond_floor must be positive");
  PW_CHECK(psi_u && eig && resid, PW_EINVAL, "NULL psi, eig or resid");
  PW_CHECK(ldpsi >= p->npw, PW_EINVAL, "ldpsi < npw");
  PW_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  pw_david_stats stats{};
  Solver S{p, W, st, stats};
  const int npw = p->npw;
  pw_precision prec = (p->opts.precision == PW_MIXED) ? PW_MIXED : PW_FP64;
  c128* psi = reinterpret_cast<c128*>(psi_u);

  PW_HIP(hipMemcpy2DAsync(W.phi, sizeof(c128) * W.ld, psi, sizeof(c128) * ldpsi, sizeof(c128) * npw, nb,
                          hipMemcpyDeviceToDevice, st));
  if (p->gamma) k_zero_im0<<<1, 256, 0, st>>>(nb, W.phi, W.ld);
  // float32 rotations pay where a rotation takes milliseconds; on small blocks
  // the overlap formed at each collapse and its fresh factorization cost more
  // than they save (64-atom cell: 141 against 135 ms per mixed solve)
  const bool long_rot = 16.0 * npw * (double)nb * nb >= kSub32MinFlops;
  S.set_sub32(prec == PW_MIXED && (o.sub32 == 2 || (o.sub32 == 1 && long_rot)));
  PW_TRY(S.start_block(prec, nb));
  k_fill<<<1, 256, 0, st>>>(nb, INFINITY, W.eps_prev);
  int nbase = nb;
  double amp = 1.0;   // accumulated error growth of the carried-over H phi
  double best32 = INFINITY;   // float32 stage: smallest max ||g_i|| so far ...
  int stall32 = 0;            // ... and iterations since it last halved
  bool retried = false;
  pw_status result = PW_OK;
  DavFlags f{};
  for (;;) {
    k_resid<<<nb, kVecThreads, 0, st>>>(npw, S.spsi_or_psi(), W.hpsi, W.ld, W.eps, W.rn, p->gamma ? 1 : 0);
    // float32 stage: a band needs no more corrections once its residual is
    // below the switch threshold (its eigenvalue change is float32 noise)
    const bool fp32_stage = prec == PW_MIXED;
    k_select<<<1, 64, 0, st>>>(nb, W.rn, W.eps, W.eps_prev, fp32_stage ? o.ladder_switch : o.tol_resid,
                               fp32_stage ? INFINITY : o.tol_deig, W.idx, W.hw.info, W.hw.gamma, W.flags);
    PW_HIP(hipMemcpyAsync(W.hflags, W.flags, sizeof(DavFlags), hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    f = *W.hflags;
    if (o.history && stats.iters < o.max_iter) {
      o.history[2 * stats.iters] = f.maxr;
      o.history[2 * stats.iters + 1] = f.gamma;
    }
    if (f.info == 2) {
      result = pw::fail(PW_EDEVICE, "workgroups of the cooperative tridiagonalization were not co-resident");
      break;
    }
    if (f.info != 0) {
      // the newest corrections made the overlap singular: the Ritz vectors
      // were not replaced; collapse onto them once and try again
      if (retried || nbase == nb - S.nl) { result = pw::fail(PW_EBREAKDOWN, "reduced overlap matrix not positive definite"); break; }
      retried = true;
      PW_HIP(hipMemsetAsync(W.hw.info, 0, sizeof(int), st));
      PW_TRY(S.collapse(nb - S.nl));
      nbase = nb - S.nl;
      stats.restarts++;
      continue;
    }
    if (f.nan) { result = pw::fail(PW_ENAN, "non-finite residual norm"); break; }
    if (p->cancel.exchange(0)) { result = pw::fail(PW_ECANCELLED, "solve cancelled (pw_cancel)"); break; }
    if (fp32_stage && f.maxr < kStallZone * o.ladder_switch) {
      if (f.maxr < 0.5 * best32) { best32 = f.maxr; stall32 = 0; } else { ++stall32; }
    }
    if (fp32_stage && (f.n_new == 0 || stall32 >= kStall32)) {
      // precision ladder: continue from the Ritz vectors with float64 H.psi
      // and float64 subspace products
      prec = PW_FP64;
      S.set_sub32(false);
      S.nl = 0;
      PW_HIP(hipMemcpy2DAsync(W.phi, sizeof(c128) * W.ld, W.psi, sizeof(c128) * W.ld, sizeof(c128) * npw, nb,
                              hipMemcpyDeviceToDevice, st));
      PW_TRY(S.start_block(prec, nb));
      k_fill<<<1, 256, 0, st>>>(nb, INFINITY, W.eps_prev);
      nbase = nb;
      amp = 1.0;
      stats.restarts++;
      stats.fresh_starts++;
      continue;
    }
    if (f.n_new == 0) break;
    if (stats.iters >= o.max_iter) { result = PW_ENOTCONV; break; }
    const int n_new = f.n_new;
    // the basis cap stays ndim nb: with bands locked, the active ones keep a
    // longer history of corrections before the next collapse
    if (nbase + n_new > o.ndim * nb) {
      // The collapsed block inherits H psi = (H phi) c and is taken to be
      // orthonormal: the rounding errors of both grow by ||c|| and ||c||^2 per
      // collapse.  Once the accumulated growth is large, the block is rebuilt
      // from the Ritz vectors with a fresh H psi and explicit reduced matrices.
      amp *= std::max(1.0, f.gamma) * std::max(1.0, f.gamma);
      // float32 H.psi carries ~1e-7 relative error already: a smaller budget
      if (amp > (prec == PW_MIXED ? kMaxAmp32 : kMaxAmp)) {
        PW_HIP(hipMemcpy2DAsync(W.phi, sizeof(c128) * W.ld, W.psi + (size_t)S.nl * W.ld, sizeof(c128) * W.ld,
                                sizeof(c128) * npw, nb - S.nl, hipMemcpyDeviceToDevice, st));
        PW_TRY(S.start_block(prec, nb - S.nl));
        amp = 1.0;
        stats.fresh_starts++;
      }
      // converged bands leave the basis for good (float64 stage only: a
      // float32-stage band counts as converged at ladder_switch, and locking
      // at that accuracy was seen to leave the basis nearly degenerate)
      if (o.lock && prec == PW_FP64) PW_TRY(S.lock(nb, n_new));
      PW_TRY(S.collapse(nb - S.nl));
      nbase = nb - S.nl;
      stats.restarts++;
    }
    PW_TRY(S.corrections(nbase, n_new, o.precond_floor));
    PW_TRY(S.hpsi(prec, n_new, W.phi + (size_t)nbase * W.ld, W.hphi + (size_t)nbase * W.ld,
                  W.sphi ? W.sphi + (size_t)nbase * W.ld : nullptr));
    PW_TRY(S.project(nbase, nbase + n_new));
    nbase += n_new;
    PW_HIP(hipMemcpyAsync(W.eps_prev, W.eps, sizeof(double) * nb, hipMemcpyDeviceToDevice, st));
    PW_TRY(S.rayleigh_ritz(nbase, nb - S.nl));
    if (prec == PW_MIXED) stats.iters_fp32++;
    stats.iters++;
  }
  // final float64 verification of the output block
  PW_HIP(hipMemcpy2DAsync(psi, sizeof(c128) * ldpsi, W.psi, sizeof(c128) * W.ld, sizeof(c128) * npw, nb,
                          hipMemcpyDeviceToDevice, st));
  PW_TRY(pw::hpsi_launch(p, PW_FP64, nb, psi, ldpsi, W.hpsi, W.ld, st));
  if (p->us) PW_TRY(pw::spsi_launch(p, PW_FP64, nb, psi, ldpsi, W.spsi, W.ld, st));
  stats.n_hpsi_fp64 += nb;
  k_final<<<nb, 256, 0, st>>>(npw, psi, ldpsi, W.hpsi, W.ld, eig, resid, p->us ? W.spsi : nullptr, p->gamma ? 1 : 0);
  PW_HIP(hipGetLastError());
  std::vector<double> hr(nb), he(nb);
  PW_HIP(hipMemcpyAsync(hr.data(), resid, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  PW_HIP(hipMemcpyAsync(he.data(), eig, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  PW_HIP(hipStreamSynchronize(st));
  stats.max_resid = 0.0;
  for (double r : hr) stats.max_resid = std::max(stats.max_resid, r);
  if (S.nl > 0) {
    // locked bands sit in the order they converged: sort the output by eigenvalue
    std::vector<int> order(nb);
    for (int b = 0; b < nb; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return he[a] < he[b]; });
    bool ident = true;
    for (int b = 0; b < nb; ++b) ident = ident && order[b] == b;
    if (!ident) {
      PW_HIP(hipMemcpyAsync(W.perm, order.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
      const dim3 g(std::min(64, ceil_div(npw, 256)), std::min(nb, 1024));
      k_gather_cols<<<g, 256, 0, st>>>(npw, nb, W.perm, psi, ldpsi, W.phi, W.ld);
      PW_HIP(hipMemcpy2DAsync(psi, sizeof(c128) * ldpsi, W.phi, sizeof(c128) * W.ld, sizeof(c128) * npw, nb,
                              hipMemcpyDeviceToDevice, st));
      k_permute_vals<<<1, 1, 0, st>>>(nb, W.perm, eig, W.etmp);
      k_permute_vals<<<1, 1, 0, st>>>(nb, W.perm, resid, W.etmp);
      PW_HIP(hipGetLastError());
      PW_HIP(hipStreamSynchronize(st));   // `order` is read by the copy above
    }
  }
  stats.nconv = f.nconv;
  stats.nlocked = S.nl;
  if (stats_out) *stats_out = stats;
  p->cancel.store(0);   // a cancel asked after the last check does not carry over to the next solve
  return result;
}

extern "C" pw_status pw_cancel(pw_plan p) {
  PW_CHECK(p != nullptr, PW_EINVAL, "NULL plan");
  p->cancel.store(1);
  return PW_OK;
}
