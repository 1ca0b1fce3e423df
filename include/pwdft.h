/*
 * pwdft.h -- C ABI of the MI355X plane-wave H.psi / block-Davidson library.
 *
 * What it computes (Hartree atomic units throughout):
 *
 *   H psi (G) = 1/2 |k+G|^2 psi(G)                                  kinetic
 *             + [ (1/N) sum_r exp(-iG.r) V(r) sum_G' psi(G') exp(iG'.r) ]   local
 *             + sum_I sum_{ij in I} beta_i(G) D^I_ij <beta_j|psi>            nonlocal
 *
 * for a block of bands in a plane-wave basis (the Kohn-Sham equation of the
 * self-consistency appendix, with the separable norm-conserving projector form
 * of the pseudopotential described in Sec. 3, and the plane-wave / FFT-grid
 * data of the parallelization section), and the lowest nb solutions of
 * H psi_i = eps_i psi_i with <psi_i|psi_j> = delta_ij (the generalized problem
 * of the iterative-diagonalization appendix with S = 1), by the block Davidson
 * method stated there (residuals, diagonal preconditioner, reduced problem on
 * the enlarged basis, Ritz update, optional expanding basis).
 *
 * Conventions
 *  - Complex numbers are interleaved (re, im) pairs of double (pw_c128).
 *  - A "block" of ncol vectors of length npw is column-major: element g of
 *    column j is at  x[j*ld + g],  ld >= npw.
 *  - The FFT convention is psi(r_j) = sum_G psi_G exp(+i G.r_j) (unscaled) and
 *    f_G = (1/N) sum_j f(r_j) exp(-i G.r_j); the Bloch factor exp(ik.r)
 *    commutes with V(r) and is not applied.
 *  - Device pointers are HIP device memory (e.g. torch tensors' data_ptr());
 *    host pointers are ordinary process memory.  Arguments marked [dev] must be
 *    device pointers, [host] host pointers.
 *  - Streams are hipStream_t passed as void*; NULL is the default stream.
 *  - Every call returns pw_status (0 = PW_OK); nothing is thrown across the ABI.
 *    pw_last_error() gives a message for the last failing call of the calling
 *    host thread.  Asynchronous device faults surface as PW_EDEVICE on the
 *    next call that synchronizes.
 *  - Thread safety: a plan may be used by one host thread / stream at a time.
 */
#ifndef PWDFT_H
#define PWDFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PW_OK = 0,
  PW_ENOTCONV = 1,      /* outputs valid (best Ritz pairs) but not converged          */
  PW_EINVAL = -1,       /* bad argument (sizes, strides, grid too small, ...)         */
  PW_ENOMEM = -2,       /* device allocation failed / size beyond the plan's capacity */
  PW_EDEVICE = -3,      /* HIP runtime error                                          */
  PW_EBREAKDOWN = -4,   /* overlap matrix not positive definite after a restart       */
  PW_ENAN = -5,         /* non-finite residual norm                                   */
  PW_ECANCELLED = -6    /* solve cancelled through pw_cancel or pw_server_cancel       */
} pw_status;

typedef enum {
  PW_FP64 = 0,          /* every step in float64                                      */
  PW_MIXED = 1          /* FFT and projector GEMMs in float32 (float32 accumulation);
                           Cholesky, reduced eigenproblem, residual norms in float64  */
} pw_precision;

typedef struct { double re, im; } pw_c128;

typedef struct pw_ctx_s*  pw_ctx;
typedef struct pw_plan_s* pw_plan;

/*
 * One plane-wave problem: a cell at one k-point.  Read only during
 * pw_plan_create; the plan copies everything it needs (the caller may free
 * all of these arrays afterwards).
 */
typedef struct {
  int32_t        npw;        /* number of plane waves in the sphere (> 0)                        */
  const int32_t* miller;     /* [host] [npw][3] integer (h,k,l) of each G; any order               */
  const double*  kpg;        /* [host] [npw][3] Cartesian k+G in bohr^-1                           */
  int32_t        nr[3];      /* FFT grid (n1, n2, n3); must satisfy n_d >= 4*max|m_d| + 1         */
  const double*  vloc_r;     /* [dev]  [n3][n2][n1] real V_loc(r_j) in Ha, x fastest              */
  int32_t        nbeta;      /* number of projectors (>= 0)                                        */
  const pw_c128* beta;       /* [dev]  [nbeta][ld_beta] column-major beta_j(G) (NULL if nbeta = 0) */
  int32_t        ld_beta;    /* >= npw                                                              */
  int32_t        nblk;       /* number of D blocks (atoms)                                         */
  const int32_t* blk_off;    /* [host] [nblk+1], 0 = blk_off[0] < ... < blk_off[nblk] = nbeta       */
  const pw_c128* dmat;       /* [host] concatenated Hermitian nh x nh blocks, column-major, in Ha   */
  const pw_c128* qmat;       /* [host] ultrasoft augmentation: S = 1 + sum_I beta_I q_I beta_I^H,
                                blocks laid out as dmat; NULL: norm-conserving, S = 1             */
} pw_problem;

/* Capacity of a plan: workspace is allocated once, at plan creation.  Fields
   past ndim_max may be left zero (defaults). */
typedef struct {
  pw_precision precision;    /* PW_FP64 or PW_MIXED                                                 */
  int32_t      nb_max;       /* largest number of bands passed to hpsi_apply / davidson_solve      */
  int32_t      ndim_max;     /* largest Davidson basis factor (basis <= ndim*nb); 0 = no solver ws  */
  int32_t      plane_mode;   /* 0: the plane pass (y, x, V(r), x, y of one z plane) runs in one
                                kernel per plane where the plane fits in LDS (the register form
                                where two planes fit a workgroup, else the lane-group form, e.g.
                                144^2 in both precisions), else in
                                three kernels through an HBM copy of the plane's x columns;
                                1: always three kernels; 2: the lane-group form (16 lanes per 1D
                                transform) wherever it applies (n1 = n2 in {80, 96, 128, 144},
                                unpadded plane within 160 KB); 3: measure every form that fits the
                                grid at plan creation and keep the fastest (cached per precision
                                and grid shape for the process); 4: the register form (a quad of
                                lanes per 1D transform) wherever it applies                       */
  size_t       fft_ws_bytes; /* transform workspace cap (sticks, plus the plane copies of the
                                three-kernel pass); bands are transformed in chunks that fit it;
                                0 = 2 GiB                                                          */
  int32_t      nl_overlap;   /* projector term of H.psi: 0 = on a side stream beside the transforms
                                except where a transform workgroup fills a CU's LDS (then after
                                them on the caller's stream); 1 = always beside; 2 = always after */
  int32_t      density;      /* 1: also allocate the workspace of pw_density and pw_scf_norm
                                (the plane copies of the three-kernel pass and one complex grid)   */
  int32_t      gamma;        /* 1: Gamma point with real wavefunctions.  The problem lists the half
                                sphere: G = 0 first, then one of each pair (G, -G); k = 0; beta real
                                in real space (beta(-G) = conj(beta(G))), D real.  Band vectors hold
                                the half-sphere coefficients (the -G ones are their conjugates,
                                psi(0) real; the imaginary part of psi(0) is ignored).  H.psi packs two
                                bands into one complex transform, and the projector and subspace
                                products are real products over the interleaved half sphere.
                                q blocks (ultrasoft S) must be real as D is; S.psi is then a real
                                product over the half sphere as well.                             */
} pw_plan_opts;

typedef struct {
  int32_t ndim;              /* basis cap = ndim*nb, 2..8 (default 2: the paper's 2N form)          */
  int32_t max_iter;          /* default 200                                                          */
  double  tol_resid;         /* Ha, band converged when ||g_i||_2 <= tol_resid (default 1e-6) ...   */
  double  tol_deig;          /* ... and |eps_i - eps_i(previous)| <= tol_deig (default 5e-9 Ha)     */
  double  precond_floor;     /* Ha, tau of the preconditioner denominator
                                smax(x, tau) = (x + tau + sqrt((x - tau)^2 + tau^2)) / 2,
                                x = h_diag(G) - eps_i (default 0.2)                              */
  double  ladder_switch;     /* mixed only: float32 H.psi until every ||g_i|| <= ladder_switch (or,
                                once below 100*ladder_switch, the largest stops halving for 12
                                iterations), then float64 (default 3e-4)                          */
  double* history;           /* [host] optional (NULL by default): for iteration t < max_iter,
                                history[2t] = max_i ||g_i|| and history[2t+1] = the largest column
                                norm of the Ritz rotation that produced the block (its error
                                growth); 2*max_iter entries, entries past stats.iters untouched */
  int32_t lock;              /* 1 (default): when the basis collapses in the float64 stage, bands
                                already converged are locked: kept fixed, projected out of every
                                later correction and left out of the reduced problems, which then
                                only hold the unconverged bands; 0: every band stays in the basis */
  int32_t sub32;             /* mixed only.  2: while H.psi is float32, the Ritz rotations (phi c,
                                (H phi) c) run in float32 arithmetic on the complex128 basis, and at
                                each collapse the overlap of the rotated block is formed (float32
                                products) instead of taken as the identity; the projections
                                phi^H H phi and phi^H phi, the Cholesky factor, the reduced
                                eigenproblem and the residual norms stay float64, and so does every
                                product of the float64 stage.  1 (default): as 2 for blocks whose
                                rotation is long (16 npw nb^2 >= 1e11 flops), else as 0.
                                0: float64 rotations                                              */
} pw_david_opts;

typedef struct {
  int32_t iters;             /* Davidson iterations                                                  */
  int32_t restarts;          /* basis collapses to the Ritz vectors                                  */
  int32_t n_hpsi_fp32;       /* band-H.psi applications in float32                                   */
  int32_t n_hpsi_fp64;       /* band-H.psi applications in float64                                   */
  int32_t nconv;             /* converged bands at exit                                              */
  int32_t iters_fp32;        /* iterations done with float32 H.psi (mixed precision)                 */
  int32_t fresh_starts;      /* rebuilds of the basis with a fresh H.psi (growth budget, ladder)     */
  int32_t nlocked;           /* bands locked when the solve ended (opts.lock)                        */
  double  max_resid;         /* max_i ||g_i||_2 of the final float64 verification                    */
} pw_david_stats;

/* Last error message of the calling host thread ("" if none). */
const char* pw_last_error(void);

/* Create / destroy a context bound to HIP device `device`.  Destroy the
   context's plans and servers before the context. */
pw_status pw_ctx_create(int device, pw_ctx* out);
pw_status pw_ctx_destroy(pw_ctx ctx);

/* Fill opts with the defaults listed above. */
void pw_david_opts_default(pw_david_opts* opts);

/* Device bytes pw_plan_create would allocate for (problem, opts). */
size_t pw_footprint_bytes(const pw_problem* problem, const pw_plan_opts* opts);

/*
 * Validate the problem, build the sphere -> FFT-box maps (z sticks, x columns),
 * the kinetic and preconditioner diagonals, twiddle tables, copies of V(r),
 * beta and D (float32 copies too in PW_MIXED), and all workspace.
 * Errors: PW_EINVAL (npw <= 0, duplicate G, grid below 4*max|m|+1, ld_beta <
 * npw, blocks not covering nbeta, D not Hermitian to 1e-12), PW_ENOMEM.
 * Synchronous; allocates device memory.
 */
pw_status pw_plan_create(pw_ctx ctx, const pw_problem* problem, const pw_plan_opts* opts,
                         pw_plan* out);
pw_status pw_plan_destroy(pw_plan plan);

/* Plan sizes: out[0]=npw, out[1]=n_sticks, out[2]=x columns, out[3]=N, out[4]=nbeta,
   out[5]=bands per transform chunk, out[6]/out[7]=form of the float64/float32 plane pass:
   0 register kernel (a quad of lanes per 1D transform), 1 three kernels, 2 lane-group kernel
   (16 lanes per 1D transform, unpadded plane in LDS), 3 generic LDS kernel; out[7] is 0 for a
   PW_FP64 plan. */
pw_status pw_plan_info(pw_plan plan, int64_t out[8]);

/*
 * Replace the plan's local potential (one step of the self-consistency loop
 * of the self-consistency appendix: V_in changes, the cell does not).
 * vloc_r [dev] double[n3][n2][n1] real V_loc(r_j) in Ha, x fastest, as in
 * pw_problem; read during the call (the caller may free it afterwards).  The
 * plan's float64 copy, its float32 copy (PW_MIXED plans) and the diagonal of
 * H used by the preconditioner (which holds the mean of V) are updated on
 * `stream`; maps, projectors, D and q blocks and all workspace stay.  The new
 * values are read back and checked first (one synchronization of `stream`):
 * on PW_ENAN (a non-finite value) or PW_EDEVICE the plan is unchanged.  Work
 * of this plan on other streams must not overlap the call; H.psi graphs of
 * the plan replay with the new potential.  Errors: PW_EINVAL (NULL),
 * PW_ENAN, PW_EDEVICE.
 */
pw_status pw_plan_set_potential(pw_plan plan, const double* vloc_r, void* stream);

/*
 * hpsi = H psi for nb bands (overwrite).  psi and hpsi are [dev] blocks
 * [nb][ld] of pw_c128, ldpsi/ldhpsi >= npw, and must not overlap.  `prec`
 * selects float64 or float32 arithmetic for the FFT and projector steps (the
 * latter needs a PW_MIXED plan); input and output stay complex128.
 * Asynchronous on `stream`; no allocation, no host synchronization.
 * Errors: PW_EINVAL (nb < 0 or > nb_max, ld < npw, NULL pointers), PW_EDEVICE.
 */
pw_status hpsi_apply(pw_plan plan, pw_precision prec, int32_t nb, const pw_c128* psi,
                     int32_t ldpsi, pw_c128* hpsi, int32_t ldhpsi, void* stream);

/*
 * spsi = S psi = psi + sum_I beta_I q_I <beta_I|psi> (overwrite), the overlap
 * operator of the generalized problem H psi = eps S psi (ultrasoft form; S = 1
 * when the problem has no qmat).  Layout, precision and errors as hpsi_apply.
 */
pw_status spsi_apply(pw_plan plan, pw_precision prec, int32_t nb, const pw_c128* psi, int32_t ldpsi,
                     pw_c128* spsi, int32_t ldspsi, void* stream);

/*
 * Block Davidson for the nb lowest eigenpairs.
 *   psi   [dev] [nb][ldpsi]: in = trial vectors (any linearly independent set),
 *         out = eigenvector estimates, orthonormal in the S metric
 *         (<psi_i|S|psi_j> = delta_ij; S = 1 without qmat).
 * With an ultrasoft problem (qmat) the generalized problem H psi = eps S psi
 * is solved: residuals (H - eps_i S) psi_i, reduced overlap phi^H S phi, the
 * preconditioner's diagonal h_diag(G) - eps_i s_diag(G), and S phi carried
 * through every Ritz rotation; locked bands (opts->lock) keep S psi, and later
 * corrections are made S-orthogonal to them.
 *   eig   [dev] double[nb], ascending Rayleigh quotients of the output psi.
 *   resid [dev] double[nb], ||H psi_i - eps_i psi_i||_2 of the output psi.
 * Both are recomputed by a final float64 H.psi.  opts may be NULL (defaults);
 * stats [host] may be NULL.  The host reads one small result per iteration
 * (stream synchronization).  Returns PW_OK, PW_ENOTCONV (max_iter reached;
 * outputs valid), PW_EBREAKDOWN, PW_ENAN, PW_EINVAL, PW_EDEVICE.
 * No allocation; needs a plan with nb_max >= nb and ndim_max >= opts->ndim.
 * Reduced problems of 64 to 2048 rows are tridiagonalized by ceil(n / 16)
 * workgroups that must be resident together; run concurrent solves through
 * davidson_solve_batched or the server, which bound how many of them spin
 * at once (a launch that cannot become resident ends with PW_EDEVICE).
 */
pw_status davidson_solve(pw_plan plan, int32_t nb, pw_c128* psi, int32_t ldpsi, double* eig,
                         double* resid, const pw_david_opts* opts, pw_david_stats* stats,
                         void* stream);

/*
 * Band-by-band preconditioned conjugate gradient for the nb lowest
 * eigenpairs of H psi = eps S psi (the iterative-diagonalization appendix,
 * "Conjugate-Gradient"): band i minimizes the Rayleigh quotient
 * <psi|H|psi> / <psi|S|psi> under S-orthogonality to bands 0..i-1, along
 * Polak-Ribiere conjugate directions of the preconditioned gradient, with the
 * exact line minimization psi cos(theta) + n sin(theta), n S-normalized and
 * S-orthogonal to psi; kinetic-only preconditioner
 * P^2(G) = 1 / smax(T_G, precond_floor), smax as in pw_david_opts.  S = 1
 * unless the plan carries ultrasoft q blocks.  One single-band float64 H.psi
 * per iteration (with q blocks also two single-band S.psi).  On Gamma plans
 * the bands are half-sphere real functions and every inner product is the
 * whole-sphere real one.  Same arguments and outputs as
 * davidson_solve (psi [dev] in: trial vectors, out: S-orthonormal
 * eigenvectors; eig, resid [dev] from a final float64 H.psi and S.psi,
 * resid_i = ||H psi_i - eps_i S psi_i||_2); needs a plan with
 * ndim_max >= 2 (its workspace).  Returns PW_OK,
 * PW_ENOTCONV (a band reached max_iter; outputs valid), PW_ENAN, PW_EINVAL,
 * PW_EDEVICE.  The host reads one small result per iteration.
 */
typedef struct {
  int32_t max_iter;          /* iterations per band (default 400)                                    */
  double  tol_resid;         /* Ha, band done when ||H psi - eps psi|| <= tol_resid (default 1e-6) ... */
  double  tol_deig;          /* ... and |d eps| <= tol_deig over the last step (default 5e-9 Ha)     */
  double  precond_floor;     /* Ha, tau of the kinetic preconditioner (default 0.2)                 */
} pw_cg_opts;
typedef struct {
  int32_t iters;             /* iterations summed over bands                                          */
  int32_t max_band_iters;    /* largest iteration count of one band                                   */
  int32_t nconv;             /* bands that met the tolerances                                         */
  double  max_resid;         /* max_i ||g_i|| of the final float64 verification                       */
} pw_cg_stats;
void      pw_cg_opts_default(pw_cg_opts* opts);
pw_status pcg_solve(pw_plan plan, int32_t nb, pw_c128* psi, int32_t ldpsi, double* eig, double* resid,
                    const pw_cg_opts* opts, pw_cg_stats* stats, void* stream);

/*
 * Output charge density of a block of bands (the rho_out equation of the
 * self-consistency appendix, with occupation weights):
 *   rho(r_j) = (1/omega) sum_b w_b |psi_b(r_j)|^2,   psi_b(r_j) = sum_G psi_b(G) exp(+i G.r_j),
 * on the plan's FFT grid r_j (x fastest).  psi [dev] [nb][ldpsi] complex128
 * (at Gamma the half-sphere coefficients, psi(-G) = conj psi(G); two bands
 * share one complex transform);
 * w [dev] double[nb]; omega = cell volume in bohr^3; rho [dev]
 * double[n3][n2][n1], overwritten (accumulate = 0) or added to (accumulate = 1).
 * The grid holds the density without aliasing when n_d >= 4 max|m_d| + 1
 * (checked at plan creation).  float64, deterministic (bands are summed in
 * order); asynchronous on `stream`, no allocation.  Needs a plan created with
 * opts.density = 1.  Errors: PW_EINVAL.
 */
pw_status pw_density(pw_plan plan, int32_t nb, const pw_c128* psi, int32_t ldpsi, const double* w,
                     double omega, int32_t accumulate, double* rho, void* stream);

/*
 * Squared scf norm of the density change (the self-consistency appendix's
 * estimate of the self-consistency error, its Hartree-energy form):
 *   ||rho_out - rho_in||^2 = 4 pi omega sum_{G != 0} |drho(G)|^2 / |G|^2,
 *   drho(G) = (1/N) sum_j (rho_out - rho_in)(r_j) exp(-i G.r_j)
 * (Hartree units, e^2 = 1; with these Fourier coefficients this equals
 * the integral of drho times the Hartree potential it generates), summed
 * over every G = m1 b1 + m2 b2 + m3 b3 of the grid with grid index i_d -> m_d
 * = i_d for i_d <= n_d/2, else i_d - n_d.  rho_out, rho_in [dev]
 * double[n3][n2][n1]; bvec [host] 9 doubles, row d = b_d in bohr^-1;
 * norm2 [host].  Synchronous on `stream`.  Needs opts.density = 1.
 */
pw_status pw_scf_norm(pw_plan plan, const double* rho_out, const double* rho_in, const double* bvec,
                      double omega, double* norm2, void* stream);

/*
 * Ask the solve running on `plan` (davidson_solve or pcg_solve, from another
 * host thread) to stop: it returns PW_ECANCELLED at its next iteration check,
 * with the current Ritz vectors, eigenvalues and residuals written as for
 * PW_ENOTCONV.  With no solve running, the next solve on the plan stops at its
 * first check.  Thread-safe; returns PW_EINVAL for a NULL plan.
 */
pw_status pw_cancel(pw_plan plan);

/*
 * hpsi_apply captured into a HIP graph: the transform passes, the projector
 * products and their join, replayed by pw_graph_launch with no host work per
 * kernel.  The graph is bound to these psi / hpsi buffers (their contents may
 * change between launches) and to the plan, which must outlive it.  One
 * eager hpsi_apply runs first on a private stream; capture uses a private
 * stream too.  Synchronous.  Errors: PW_EINVAL, PW_EDEVICE.
 */
typedef struct pw_graph_s* pw_graph;
pw_status pw_hpsi_graph_create(pw_plan plan, pw_precision prec, int32_t nb, const pw_c128* psi, int32_t ldpsi,
                               pw_c128* hpsi, int32_t ldhpsi, pw_graph* out);
pw_status pw_graph_launch(pw_graph graph, void* stream);   /* asynchronous on `stream` */
pw_status pw_graph_destroy(pw_graph graph);

/*
 * Batches of independent problems (cells x k-points; the paper's pool level,
 * whose problems need no communication).  Item i uses plans[i] (all plans of
 * ctx, each at most once per call) with nb[i] bands and the [dev] blocks
 * psi[i] (ldpsi[i]), ... as in the single-problem call; the pointer arrays
 * are [host].
 *
 * hpsi_apply_batched: hpsi[i] = H_i psi[i] for every i, launched round robin
 * on nstreams (<= 0: 8) worker streams of ctx that wait for the work already
 * queued on `stream` and are joined back into it.  Asynchronous.  Results are
 * bitwise those of hpsi_apply.  Errors: PW_EINVAL, PW_EDEVICE.
 *
 * davidson_solve_batched: davidson_solve for every item, nworkers (<= 0: 8)
 * at a time, each on its own worker stream driven by its own host thread.
 * Synchronous.  stats [host, n] and status [host, n] may be NULL; status[i]
 * is item i's own return code.  Returns the first hard error (with the
 * item's message), else PW_ENOTCONV if any item did not converge, else PW_OK.
 * opts->history must be NULL.  Concurrent solves use the cooperative
 * reduced-eigensolver kernels only while nworkers x ceil(ndim nb / 16) <= 128
 * (the server applies the same rule to its workers).
 * One batched call per context at a time.
 */
pw_status hpsi_apply_batched(pw_ctx ctx, int32_t n, const pw_plan* plans, pw_precision prec,
                             const int32_t* nb, const pw_c128* const* psi, const int32_t* ldpsi,
                             pw_c128* const* hpsi, const int32_t* ldhpsi, int32_t nstreams, void* stream);
pw_status davidson_solve_batched(pw_ctx ctx, int32_t n, const pw_plan* plans, const int32_t* nb,
                                 pw_c128* const* psi, const int32_t* ldpsi, double* const* eig,
                                 double* const* resid, const pw_david_opts* opts, pw_david_stats* stats,
                                 pw_status* status, int32_t nworkers, void* stream);

/*
 * Serving loop for independent requests of different sizes (the paper's pool
 * level applied to a request stream).  Requests are admitted in arrival
 * order as soon as one of nworkers host workers is idle and the device
 * memory of the request's plan (pw_footprint_bytes) fits in mem_budget next
 * to the running ones; each runs pw_plan_create, davidson_solve on the
 * worker's stream and pw_plan_destroy.
 *   pw_server_create: opts may be NULL (4 workers, mem_budget 0 = 60% of the
 *     free device memory, PW_MIXED plans).  Allocates the whole budget at once
 *     as the pool the served plans take their memory from (PW_ENOMEM when
 *     that allocation fails); it is freed by pw_server_destroy.
 *   pw_server_submit: enqueue one request and return its ticket at once.
 *     The problem's arrays (host and device) and psi [dev, in/out], eig and
 *     resid [dev] must stay valid until the request completes, and their
 *     contents must be complete when submit is called: the worker reads them
 *     on its own stream, with no ordering against the caller's streams.  PW_ENOMEM if
 *     the request alone exceeds mem_budget; PW_EINVAL for invalid problems.
 *   pw_server_wait: block until the ticket's request is done; returns its
 *     davidson_solve status (message in pw_last_error), its stats, and
 *     times[3] = submit, start and end in seconds on the server's clock.  A
 *     ticket can be waited for once.
 *   pw_server_poll: done = 1 when the request has completed.
 *   pw_server_clock: seconds since pw_server_create.
 *   pw_server_cancel: a queued request is dropped (its wait returns
 *     PW_ECANCELLED at once); a running one stops at its solve's next
 *     iteration check (pw_cancel) and returns PW_ECANCELLED with its current
 *     Ritz pairs; a finished one is left as it is.  PW_EINVAL for an unknown
 *     ticket.
 *   pw_server_destroy: finish every submitted request, then stop.
 */
typedef struct pw_server_s* pw_server;
typedef struct {
  int32_t      nworkers;     /* concurrent requests, 1..64                                          */
  size_t       mem_budget;   /* device bytes the running requests' plans may hold (0: 60% of free)  */
  pw_precision precision;    /* precision of the requests' plans                                    */
  int32_t      gamma;        /* 1: every request is a Gamma-point problem on the half sphere (plans
                                with pw_plan_opts.gamma = 1); 0 (default): whole-sphere problems   */
} pw_server_opts;
void      pw_server_opts_default(pw_server_opts* opts);
pw_status pw_server_create(pw_ctx ctx, const pw_server_opts* opts, pw_server* out);
pw_status pw_server_submit(pw_server server, const pw_problem* problem, int32_t nb, pw_c128* psi,
                           int32_t ldpsi, double* eig, double* resid, const pw_david_opts* opts,
                           int64_t* ticket);
pw_status pw_server_wait(pw_server server, int64_t ticket, pw_david_stats* stats, double times[3]);
pw_status pw_server_poll(pw_server server, int64_t ticket, int32_t* done);
pw_status pw_server_cancel(pw_server server, int64_t ticket);
double    pw_server_clock(pw_server server);
/* Serving-loop counters: out[0] = requests whose plan was built, out[1] = bytes
   of the device memory pool (allocated once at pw_server_create: the admission
   budget), out[2] = largest pool use seen when a plan completed, out[3] =
   allocations that did not fit a free range of the pool and fell back to
   hipMalloc / hipHostMalloc (0 in a steady state).  Errors: PW_EINVAL. */
pw_status pw_server_info(pw_server server, int64_t out[4]);
pw_status pw_server_destroy(pw_server server);

/*
 * The float64 reduced-problem solver used inside davidson_solve, exposed on
 * its own: lowest nev eigenpairs of the generalized Hermitian problem
 * H c = w S c (S positive definite), as the iterative-diagonalization
 * appendix's reduced step.  H, S [dev] n x n column-major (leading dimension
 * ld, both triangles filled); w [dev] double[nev] ascending; C [dev]
 * n x nev column-major (ldc), S-orthonormal.  If debug [dev] is not NULL it
 * receives the Householder tridiagonal of L^-1 H L^-H: d (n doubles) then e
 * (n-1 doubles).  Allocates and frees its own workspace; synchronous.
 * Errors: PW_EINVAL, PW_EBREAKDOWN (S not positive definite), PW_EDEVICE.
 */
pw_status pw_reduced_eigh(pw_ctx ctx, int32_t n, int32_t nev, const pw_c128* H, const pw_c128* S,
                          int32_t ld, double* w, pw_c128* C, int32_t ldc, double* debug, void* stream);

/*
 * pw_reduced_eigh without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as pw_reduced_eigh,
 * plus PW_EINVAL for n > 256.  The workspace is a static 48 MiB device array,
 * one per GPU, set up by pw_ctx_create and held until the process ends; no
 * hipMalloc or hipFree is called.  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on the same GPU (other host threads,
 * other streams) race and must be serialized by the caller.  Synchronous.
 */
pw_status pw_reduced_eigh_noalloc(pw_ctx ctx, int32_t n, int32_t nev, const pw_c128* H, const pw_c128* S,
                                  int32_t ld, double* w, pw_c128* C, int32_t ldc, double* debug, void* stream);

/*
 * Per-kernel timing for measurement: when enabled, each library launch of a
 * timed kernel class is bracketed by HIP events on its stream.
 * pw_profile_enable(on) resets the accumulators; pw_profile_read(k, ...)
 * synchronizes on the recorded events and returns the launch count, the
 * summed elapsed milliseconds and the summed algorithmic work of class k
 * (0 <= k < pw_profile_count(); bytes for the transform passes and vector
 * kernels, flops for matrix products and factorizations); pw_profile_name(k)
 * names the class.  pw_profile_only(k) resets and enables timing of class k
 * alone (k = -1: every class), so that a measurement of one kernel adds no
 * events around the others; PW_EINVAL for k outside [-1, pw_profile_count()).
 * Process-wide; not for concurrent use from several host threads while
 * enabled.
 */
pw_status   pw_profile_enable(int on);
pw_status   pw_profile_only(int32_t k);
int32_t     pw_profile_count(void);
const char* pw_profile_name(int32_t k);
pw_status   pw_profile_read(int32_t k, int64_t* launches, double* total_ms, double* units);

#ifdef __cplusplus
}
#endif
#endif /* PWDFT_H */
