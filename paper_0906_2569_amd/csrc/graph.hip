// hpsi_apply captured into a HIP graph behind the C ABI: the transform
// passes, the projector products (on the plan's side stream when they run
// beside the transforms) and their join become one executable graph that is
// relaunched with no host work per kernel.  The capture runs on a private
// stream; the graph holds the pointers it was captured with.
#include "plan.h"

struct pw_graph_s {
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" pw_status pw_hpsi_graph_create(pw_plan p, pw_precision prec, int32_t nb, const pw_c128* psi,
                                          int32_t ldpsi, pw_c128* hpsi, int32_t ldhpsi, pw_graph* out) {
  PW_CHECK(out != nullptr, PW_EINVAL, "NULL output");
  *out = nullptr;
  PW_CHECK(p != nullptr, PW_EINVAL, "NULL plan");
  PW_CHECK(nb >= 1 && nb <= p->opts.nb_max, PW_EINVAL, "nb out of range [1, nb_max]");
  PW_CHECK(psi != nullptr && hpsi != nullptr, PW_EINVAL, "NULL psi or hpsi");
  PW_CHECK(ldpsi >= p->npw && ldhpsi >= p->npw, PW_EINVAL, "leading dimension < npw");
  PW_CHECK(prec == PW_FP64 || prec == PW_MIXED, PW_EINVAL, "bad precision");
  PW_HIP(hipSetDevice(p->device));
  hipStream_t cs = nullptr;
  PW_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  const c128* x = reinterpret_cast<const c128*>(psi);
  c128* y = reinterpret_cast<c128*>(hpsi);
  // one eager product first: one-time kernel set-up (LDS limits) stays out of the capture
  pw_status st = pw::hpsi_launch(p, prec, nb, x, ldpsi, y, ldhpsi, cs);
  if (st == PW_OK && hipStreamSynchronize(cs) != hipSuccess) st = pw::fail(PW_EDEVICE, "eager H.psi failed");
  pw_graph g = nullptr;
  if (st == PW_OK) {
    g = new pw_graph_s();
    g->device = p->device;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      st = pw::fail(PW_EDEVICE, "stream capture could not begin");
    } else {
      const pw_status cap = pw::hpsi_launch(p, prec, nb, x, ldpsi, y, ldhpsi, cs);
      const hipError_t e = hipStreamEndCapture(cs, &g->graph);
      if (cap != PW_OK) st = cap;
      else if (e != hipSuccess) st = pw::fail(PW_EDEVICE, std::string("stream capture failed: ") + hipGetErrorString(e));
      else if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        st = pw::fail(PW_EDEVICE, "graph instantiation failed");
    }
  }
  (void)hipGetLastError();
  (void)hipStreamDestroy(cs);
  if (st != PW_OK) {
    if (g) {
      if (g->exec) (void)hipGraphExecDestroy(g->exec);
      if (g->graph) (void)hipGraphDestroy(g->graph);
      delete g;
    }
    return st;
  }
  *out = g;
  return PW_OK;
}

extern "C" pw_status pw_graph_launch(pw_graph g, void* stream) {
  PW_CHECK(g != nullptr && g->exec != nullptr, PW_EINVAL, "NULL graph");
  PW_HIP(hipSetDevice(g->device));
  PW_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
  return PW_OK;
}

extern "C" pw_status pw_graph_destroy(pw_graph g) {
  if (!g) return PW_OK;
  (void)hipSetDevice(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  (void)hipGetLastError();
  return PW_OK;
}
