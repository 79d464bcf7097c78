// suave_engine.h -- host driver of Suave: one integral's regions, grids and
// samples resident on the device, advanced one step per round trip.
#pragma once
#include "context.h"
#include "suave.h"

namespace ccuba {

struct SuaveSpec {
  int ndim = 1, nbins = 128, family = 0, flags = 0;
  double a[kMaxDim] = {0}, u[kMaxDim] = {0};
  unsigned long long seed = 0;
  uint32_t sid = 0;
  double epsrel = 0, epsabs = 0;
  long long mineval = 0, maxeval = 0, nnew = 1000;
  double flatness = 25.0;
  int nsplit = 1;
};

int validate_suave(const SuaveSpec &s);

struct SuaveResult {
  double integral = 0, error = 0, prob = 0, chi2 = 0;
  int dof = 0, fail = 1, nregions = 0;
  long long neval = 0, nsplits = 0;
};

// Host arrays the final regions are copied to (any pointer may be null).
struct SuaveTraceOut {
  int max_regions = 0, max_splits = 0;
  double *lo = nullptr, *hi = nullptr, *I = nullptr, *var = nullptr, *grid = nullptr;
  int *cut = nullptr;
};

int run_suave(ccuba_ctx *ctx, const SuaveSpec &spec, SuaveResult &res, const SuaveTraceOut *tr,
              hipStream_t s);

}  // namespace ccuba
