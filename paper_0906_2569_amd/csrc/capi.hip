// Context, error reporting and option defaults of the C ABI.
#include <string>

#include "linalg.h"

namespace {
thread_local std::string g_last_error;
}

void pw::set_error(const std::string& msg) { g_last_error = msg; }

pw_status pw::fail(pw_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

extern "C" const char* pw_last_error(void) { return g_last_error.c_str(); }

extern "C" pw_status pw_ctx_create(int device, pw_ctx* out) {
  PW_CHECK(out != nullptr, PW_EINVAL, "NULL output");
  *out = nullptr;
  int n = 0;
  PW_HIP(hipGetDeviceCount(&n));
  PW_CHECK(device >= 0 && device < n, PW_EINVAL, "no such HIP device");
  PW_HIP(hipSetDevice(device));
  // this device's copy of the static workspace of the allocation-free entry point
  PW_TRY(pw::noalloc_scratch_init(device));
  pw_ctx c = new pw_ctx_s();
  c->device = device;
  *out = c;
  return PW_OK;
}

extern "C" pw_status pw_ctx_destroy(pw_ctx c) {
  if (!c) return PW_OK;
  (void)hipSetDevice(c->device);
  pw::ctx_release_pool(c);
  delete c;
  (void)hipGetLastError();
  return PW_OK;
}

extern "C" void pw_david_opts_default(pw_david_opts* o) {
  if (!o) return;
  o->ndim = 2;
  o->max_iter = 200;
  o->tol_resid = 1e-6;
  o->tol_deig = 5e-9;
  o->precond_floor = 0.2;
  o->ladder_switch = 3e-4;
  o->history = nullptr;
  o->lock = 1;
  o->sub32 = 1;
}
