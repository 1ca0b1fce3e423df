// Float64 reduced-problem solver (generalized Hermitian eigenproblem) on the GPU.
#pragma once
#include <algorithm>
#include <cfloat>

#include "plan.h"

namespace pw {

struct HeigWork {
  int nmax = 0;
  c128 *L = nullptr, *X = nullptr, *T1 = nullptr, *A = nullptr, *Y = nullptr, *tau = nullptr;
  double *d = nullptr, *e = nullptr, *w = nullptr, *Z = nullptr, *scratch = nullptr;
  int* info = nullptr;     // 0; 1 when fewer than nev independent directions remain; 2 when the
                           // workgroups of a cooperative kernel were not all resident
  int* drop = nullptr;     // [n] 1 for basis directions dropped as dependent
  double* gamma = nullptr; // max column norm of the last eigenvector block C
  c128 *PV = nullptr, *PW = nullptr;   // tridiagonalization panel vectors (conjugated, row-major)
  void* coop = nullptr;    // exchange buffers of the cooperative tridiagonalization
  int* cflags = nullptr;   // blocked Cholesky: [0] = not positive definite
  bool coop_ok = true;     // cooperative (multi-workgroup) kernels allowed: every workgroup of a
                           // launch must be resident at once, so callers that run several
                           // solves concurrently on one device switch them off
  bool coop_wide = false;  // cooperative tridiagonalization with 16 rows per workgroup at every
                           // size (half the workgroups of the 8-row form used up to 512 rows):
                           // the form for solves that run concurrently
  int cus = 0;             // compute units of the device (set by heig_setup)
  double drop_tol = 1e-10; // Cholesky pivot, relative to the original diagonal entry, below which
                           // a basis direction counts as dependent (lies, to the accuracy of S,
                           // in the span of the earlier ones); callers whose S comes from float32
                           // products raise it above that accuracy
};

size_t heig_work_bytes(int nmax);
pw_status heig_setup(HeigWork& hw, void* base, int nmax);
pw_status heig_set_limits();
// lowest nev eigenpairs of H c = w S c (n x n, col-major, leading dimension ld);
// the Cholesky factor of S[0:n0, 0:n0] from the previous call is reused
pw_status heig_solve(HeigWork& hw, int n0, int n, int nev, const c128* H, const c128* S, int ld, double* w,
                     c128* C, int ldc, void* part, size_t part_bytes, hipStream_t st);
// device address of this device's static workspace of pw_reduced_eigh_noalloc,
// looked up once per device (the device must be current)
pw_status noalloc_scratch_init(int device);
// factor of an orthonormal leading block of size n: L = X = I
pw_status heig_reset(HeigWork& hw, int n, hipStream_t st);

}  // namespace pw
