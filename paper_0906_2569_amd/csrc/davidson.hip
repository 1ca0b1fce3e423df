// Block Davidson (placeholder until the solver lands).
#include "plan.h"

struct DavWork {};

pw_status pw::dav_alloc(pw_plan) { return PW_OK; }
void pw::dav_free(pw_plan) {}
size_t pw::dav_bytes(int, int, int) { return 0; }

extern "C" pw_status davidson_solve(pw_plan p, int32_t, pw_c128*, int32_t, double*, double*,
                                    const pw_david_opts*, pw_david_stats*, void*) {
  PW_CHECK(p != nullptr, PW_EINVAL, "NULL plan");
  return pw::fail(PW_EINVAL, "davidson_solve: not built yet");
}
