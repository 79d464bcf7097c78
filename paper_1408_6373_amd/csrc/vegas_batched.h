// vegas_batched.h -- Vegas with a caller-evaluated integrand.
#pragma once
#include "ccuba.h"
#include "context.h"

namespace ccuba {

struct BatchedSpec {
  int ndim = 1, ncomp = 1, nbins = 128, prec = FP64, flags = 0;
  int nvec = 1000;  // points per integrand call (the last of an iteration may be fewer)
  int where = CCUBA_POINTS_HOST;
  unsigned long long seed = 0;
  uint32_t sid = 0;
  long long nstart = 1000, nincrease = 0, mineval = 0, maxeval = 0;
  double epsrel = 0, epsabs = 0;
};

// Runs the whole integration on ctx's stream (the caller holds ctx->lock).
// fail: 0 accuracy reached, 1 maxeval reached first, -99 the integrand
// returned -999 (neval then counts every point handed to it).
int vegas_batched(ccuba_ctx *ctx, const BatchedSpec &sp, ccuba_batch_integrand fn,
                  void *userdata, long long *neval, int *fail, double integral[],
                  double error[], double prob[]);

}  // namespace ccuba
