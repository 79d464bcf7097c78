// rtc.h -- the DoSample kernel for a caller's device integrand, compiled at
// run time.
#pragma once
#include <map>
#include <string>

#include "context.h"

namespace ccuba {

// Modules compiled for one context, by source and kernel class, and the
// last compiler log.
struct RtcCache {
  std::map<std::string, std::pair<hipModule_t, hipFunction_t>> mods;
  std::string log;
};

// The DoSample kernel of the class (precision, histogram type, points per
// lane, Philox blocks per point, power-of-two bins, d = 4 nb) with the
// caller's `source', which defines
//   __device__ double ccuba_user(const double *x, int ndim, const double *a,
//                                const double *u)
// and, for FP32 evaluation, the same with float.  Compiled for ctx's GPU on
// first use and kept in ctx->rtc.  CCUBA_EINVAL when the source does not
// compile (the log is kept for ccuba_rtc_log), CCUBA_EHIP otherwise.
int rtc_dosample(ccuba_ctx *ctx, const char *source, int prec, int hist64, int ilp, int nb,
                 bool pow2, bool full, hipFunction_t *out);
// Unload every module of ctx (at shutdown).
void rtc_release(ccuba_ctx *ctx);

}  // namespace ccuba
