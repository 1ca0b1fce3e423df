// Internal plan / context layout shared by the library's translation units.
#pragma once
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"
#include "fft.h"

struct pw_ctx_s {
  int device = 0;
  std::mutex mu;                       // guards the stream pool
  std::vector<hipStream_t> pool;       // worker streams of the batched calls (default priority)
  std::vector<hipEvent_t> pool_events; // one per worker stream
};

// Device-side description of the sphere <-> FFT-box maps, passed by value.
struct SphereMap {
  int npw, n1, n2, n3;
  int nst;         // number of z sticks (distinct (h,k))
  int nxr;         // number of x columns (distinct h)
  int ldst;        // stick-buffer row length (>= nst)
  const int* st_ptr;   // [nst+1]   CSR: sphere entries of stick s
  const int* ent_g;    // [npw]     sphere index of each entry (stick-major, z ascending)
  const int* ent_z;    // [npw]     z grid index (l mod n3) of each entry
  const int* ent_s;    // [npw]     stick of each entry
  const int* st_hx;    // [nst]     x-column index of stick s
  const int* st_i2;    // [nst]     y grid index (k mod n2) of stick s
  const int* i1_hx;    // [n1]      x-column index at x grid index i1, or -1
  const int* zidx;     // [n3][nst] sphere index of (z, stick), or -1
  const int* col_ptr;  // [nxr+1]   first stick of each x column (sticks are column-major)
  const int* cy_st;    // [nxr][n2] stick at (x column, y grid index), or -1 (eight-lane plane pass)
  const double* kin;   // [npw]     |k+G|^2 / 2
  FftDesc f1, f2, f3;  // transforms along x, y, z
};

struct DavWork;  // Davidson workspace (davidson.hip)
struct CgWork;   // conjugate-gradient workspace (pcg.hip)

// partial sums of pw_scf_norm (one per workgroup of its last transform pass, plus the total)
constexpr int kDensityPart = 16384;

namespace pw {
// First-fit sub-allocator over one block (device memory from hipMalloc, or
// pinned host memory from hipHostMalloc) in 256-byte granules; neighbouring
// free ranges merge on release.  Thread-safe.  The serving loop gives every
// plan it builds one of these, so that requests neither call hipMalloc nor
// hipFree (both of which synchronize with work on other streams).
class Arena {
 public:
  pw_status init(size_t bytes, bool host);
  void release();
  void* alloc(size_t bytes);        // nullptr when no free range is large enough
  bool free(void* p);               // false when p is not a live block of this arena
  size_t size() const { return size_; }
  size_t used() const;
  ~Arena() { release(); }

 private:
  mutable std::mutex mu_;
  char* base_ = nullptr;
  size_t size_ = 0;
  bool host_ = false;
  std::map<size_t, size_t> free_;   // offset -> length
  std::map<size_t, size_t> used_;   // offset -> length
};

struct MemPool {
  Arena dev, host;
  std::atomic<long> fallbacks{0};   // allocations that fell back to hipMalloc / hipHostMalloc
};
}  // namespace pw

struct pw_plan_s {
  pw_ctx ctx = nullptr;
  int device = 0;           // HIP device of the plan (kept here: the plan never reads ctx after creation)
  pw_plan_opts opts{};
  int npw = 0, n1 = 0, n2 = 0, n3 = 0;
  long N = 0;
  int nst = 0, nxr = 0, ldst = 0;
  int nbeta = 0, nblk = 0, nhmax = 0;
  int ldb = 0;              // leading dimension of the plan's beta copies
  int band_chunk = 0;       // bands per FFT pass (stick workspace capacity)
  bool use_reg_plane = true;  // register-resident z passes where the grid allows
  bool split64 = false, split32 = false;  // three-kernel plane pass (float64 / float32)
  int form64 = 0, form32 = 0;   // plane pass form per precision: 0 register (quad) kernel,
                                // 1 three kernels, 2 lane-group kernel, 3 generic LDS kernel
  bool gamma = false;       // Gamma point: bands are real functions stored on the half sphere (npw
                            // entries, G = 0 first); the transforms cover the whole sphere (nfull)
  int nfull = 0;
  int *gpos_p = nullptr, *gpos_m = nullptr;   // Gamma: [npw] stick position of G and of -G

  // maps (device)
  int *st_ptr = nullptr, *ent_g = nullptr, *ent_z = nullptr, *ent_s = nullptr, *st_hx = nullptr,
      *st_i2 = nullptr, *i1_hx = nullptr, *zidx = nullptr, *col_ptr = nullptr, *cy_st = nullptr;
  double* kin = nullptr;     // [npw]
  double* hdiag = nullptr;   // [npw] exact diagonal of H
  FftDesc f1{}, f2{}, f3{};
  c128 *tw64_1 = nullptr, *tw64_2 = nullptr, *tw64_3 = nullptr;
  c64 *tw32_1 = nullptr, *tw32_2 = nullptr, *tw32_3 = nullptr;

  // operator data (device)
  double* vr64 = nullptr;    // [N]
  float* vr32 = nullptr;     // [N]  (mixed only)
  c128* beta64 = nullptr;    // [nbeta][ldb]
  c64* beta32 = nullptr;     // [nbeta][ldb] (mixed only)
  int* dstart = nullptr;     // [nbeta] first projector of the D block of projector j
  int* dlen = nullptr;       // [nbeta] size of that block
  c128* drow64 = nullptr;    // [nbeta][nhmax] row j of D restricted to its block
  c64* drow32 = nullptr;
  bool us = false;           // ultrasoft: S = 1 + beta q beta^H
  c128* qrow64 = nullptr;    // [nbeta][nhmax] row j of q restricted to its block
  c64* qrow32 = nullptr;
  double* sdiag = nullptr;   // [npw] diagonal of S (ultrasoft plans)

  // H.psi workspace (device)
  void* sticks = nullptr;    // [band_chunk][n3][ldst] complex (FP64 size)
  void* rows = nullptr;      // [band_chunk][n3][n2][nxr] complex (FP64 size), three-kernel plane pass
                             // and density only
  c128* dgrid = nullptr;     // [N] complex grid of pw_scf_norm (density plans)
  double* dpart = nullptr;   // partial sums of pw_scf_norm
  void* part = nullptr;      // split-K partials
  size_t part_bytes = 0;
  void* becp = nullptr;      // [nb_max][nbeta] complex128 (or complex64)
  void* becpd = nullptr;     // D-applied becp
  void* becpq = nullptr;     // q-applied becp (S psi of ultrasoft plans)

  DavWork* dav = nullptr;
  CgWork* cg = nullptr;
  std::atomic<int> cancel{0};   // set by pw_cancel; read once per iteration by the running solve
  std::vector<void*> allocs;
  pw::MemPool* pool = nullptr;         // device / pinned host memory of a served plan (else hipMalloc)
  hipStream_t init_stream = nullptr;   // stream of the set-up work of a pooled plan
  hipStream_t side = nullptr;          // projector term runs here, beside the transforms
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  SphereMap map() const {
    SphereMap m;
    m.npw = npw; m.n1 = n1; m.n2 = n2; m.n3 = n3;
    m.nst = nst; m.nxr = nxr; m.ldst = ldst;
    m.st_ptr = st_ptr; m.ent_g = ent_g; m.ent_z = ent_z; m.ent_s = ent_s;
    m.st_hx = st_hx; m.st_i2 = st_i2; m.i1_hx = i1_hx; m.zidx = zidx; m.col_ptr = col_ptr; m.kin = kin;
    m.cy_st = cy_st;
    m.f1 = f1; m.f2 = f2; m.f3 = f3;
    return m;
  }
};

namespace pw {
// Device and pinned host allocations of a plan and its workspaces: from the
// plan's pool when it has one (falling back to hipMalloc / hipHostMalloc when
// the pool has no free range large enough), else hipMalloc / hipHostMalloc.
pw_status dev_alloc(pw_plan p, size_t bytes, void** out);
void dev_free(pw_plan p, void* q);
pw_status host_alloc(pw_plan p, size_t bytes, void** out);
void host_free(pw_plan p, void* q);
// pw_plan_create / pw_plan_destroy with a pool: the set-up work runs on
// `stream` and only that stream is synchronized (not the device)
pw_status plan_create(pw_ctx ctx, const pw_problem* pr, const pw_plan_opts* o, MemPool* pool,
                      hipStream_t stream, pw_plan* out);
void plan_destroy(pw_plan p);

// sphere -> sticks -> rows for nt <= band_chunk transforms in float64: inverse
// z and inverse y transforms into p->rows ([transform][z][y][x column]).  One
// transform per band (nt = nbands), or at Gamma one per pair of bands
// (nt = ceil(nbands / 2), psi_2t + i psi_2t+1)
pw_status psi_to_rows(pw_plan p, int nt, int nbands, const c128* psi, int ldpsi, hipStream_t stream);
// H.psi for nb bands (nb <= opts.nb_max) on `stream`.
pw_status hpsi_launch(pw_plan p, pw_precision prec, int nb, const c128* psi, int ldpsi,
                      c128* hpsi, int ldhpsi, hipStream_t stream);

// C[m, n] = alpha sum_k conj(A[k, m]) B[k, n] + beta Cin[m, n]  (A, B K-contiguous columns),
// C col-major ldc, complex128; Cin = C unless given (col-major, ldcin).
// Deterministic split-K.  T = compute type.
template <typename T, typename TA, typename TB>
pw_status zgemm_cn(int M, int N, int K, const cpx<TA>* A, int lda, const cpx<TB>* B, int ldb,
                   c128* C, int ldc, void* part, size_t part_bytes, hipStream_t stream,
                   double alpha = 1.0, double beta = 0.0, const c128* Cin = nullptr, int ldcin = 0);

// calbec with the D blocks applied: out[n][j] = sum_{j' in blk(j)} D_jj' sum_k conj(beta[j'][k]) psi[n][k]
// (rows: the block rows of another block-diagonal matrix in the layout of drow, e.g. q)
template <typename T>
pw_status calbec_d(pw_plan p, int nb, const c128* psi, int ldpsi, cpx<T>* out, hipStream_t stream,
                   const cpx<T>* rows = nullptr);
// spsi = S psi = psi + beta (q <beta|psi>) (a copy of psi when the plan has no q)
pw_status spsi_launch(pw_plan p, pw_precision prec, int nb, const c128* psi, int ldpsi, c128* spsi, int ldspsi,
                      hipStream_t stream);

// C[m, n] = alpha sum_k A[m, k] B[k, n] + beta C[m, n];  A M-contiguous (A[k*lda + m]),
// B K-contiguous (B[n*ldb + k]), C M-contiguous complex128 (C[n*ldc + m]).
// `guard (device int, optional): when nonzero at run time the product is skipped.
// `kin` (device, optional, M entries) adds kin[m] X[n*ldx + m] to C (the
// kinetic term of H.psi, fused into the projector add-back).
template <typename T, typename TA, typename TB>
pw_status zgemm_nn(int M, int N, int K, double alpha, const cpx<TA>* A, int lda,
                   const cpx<TB>* B, int ldb, double beta, c128* C, int ldc, hipStream_t stream,
                   const int* guard = nullptr, const double* kin = nullptr, const c128* X = nullptr,
                   int ldx = 0);

// zgemm_nn in float64 for products with few output tiles: K is split over
// workgroups and the partials summed in a fixed order (part: workspace of
// splitk_part_bytes(M, N, K, 16) bytes); plain zgemm_nn when the product has
// tiles enough or the workspace is too small
pw_status zgemm_nn_sk(int M, int N, int K, double alpha, const c128* A, int lda, const c128* B, int ldb,
                      double beta, c128* C, int ldc, void* part, size_t part_bytes, hipStream_t stream);

// C0 = A^H B0 and C1 = A^H B1 (float64, as zgemm_cn with alpha 1, beta 0) in one launch
pw_status zgemm_cn_pair(int M, int N, int K, const c128* A, int lda, const c128* B0, const c128* B1, int ldb,
                        c128* C0, c128* C1, int ldc, void* part, size_t part_bytes, hipStream_t stream);

// C0 = A0 B and C1 = A1 B (same shapes and leading dimensions) in one launch.  T is the
// arithmetic: double, or float (complex128 operands rounded to float32 as they are
// staged into LDS, float32 products and sums, complex128 result)
template <typename T = double>
pw_status zgemm_nn_pair(int M, int N, int K, const c128* A0, const c128* A1, int lda, const c128* B, int ldb,
                        c128* C0, c128* C1, int ldc, hipStream_t stream, const int* guard = nullptr);

size_t splitk_part_bytes(int M, int N, int K, int elem_bytes);

// Real products for the Gamma-point path (dgemm.hip).  Complex half-sphere
// columns are read as real columns of twice the length.
// tn: C[m, n] = alpha (2 sum_k A[m*lda + k] B[n*ldb + k] - w0 A[m*lda] B[n*ldb]) + beta C[m, n],
//     C real (ldc) or, cplx_out, the real parts of a complex matrix (imaginary parts set to 0);
//     deterministic split K (part: dgemm_part_bytes(M, N) bytes).  T = compute type.
// (prof: the profiler class the product is timed under, -1 = the generic product class)
template <typename T, typename TA, typename TB>
pw_status dgemm_tn(int M, int N, int K, const TA* A, long lda, const TB* B, long ldb, double w0, double alpha,
                   double beta, double* C, int ldc, bool cplx_out, void* part, size_t part_bytes,
                   hipStream_t stream, int prof = -1);
// nn: C[n*ldc + m] = alpha sum_k A[k*lda + m] B[n*ldb + k] + beta C[n*ldc + m] (C double; guard as zgemm_nn)
template <typename T, typename TA, typename TB>
pw_status dgemm_nn(int M, int N, int K, double alpha, const TA* A, long lda, const TB* B, long ldb, double beta,
                   double* C, long ldc, hipStream_t stream, const int* guard = nullptr, int prof = -1);
size_t dgemm_part_bytes(int M, int N);

pw_status dav_alloc(pw_plan p);
// allow or forbid the cooperative (multi-workgroup) kernels of the plan's
// reduced eigensolver; returns the previous setting
// (wide: the form with fewer workgroups per launch, for concurrent solves)
bool dav_set_coop(pw_plan p, bool ok, bool wide = false);
// workgroups that cooperative launches of concurrent solves may keep
// spinning at once (half of the device's 256 compute units): concurrent
// solves use them only while workers x (workgroups of one launch) stays within it
constexpr int kCoopWgBudget = 128;
// workgroups (all resident at once) of the cooperative tridiagonalization of n rows
// (wide: 16 rows per workgroup at every size)
int coop_workgroups(int n, bool wide = false);
bool dav_get_coop(pw_plan p);
// destroy the context's worker streams (pw_ctx_destroy)
void ctx_release_pool(pw_ctx ctx);
void dav_free(pw_plan p);
size_t dav_bytes(int npw, int nb_max, int ndim_max);
// float64 H psi of the block (into the Davidson workspace), then
// eig_b = <psi_b|H psi_b> / <psi_b|psi_b> and resid_b = ||H psi_b - eig_b psi_b||
pw_status final_check(pw_plan p, int nb, const c128* psi, int ldpsi, double* eig, double* resid, hipStream_t st);
pw_status cg_alloc(pw_plan p);
void cg_free(pw_plan p);
size_t cg_bytes(int npw, int nb_max);
}  // namespace pw
