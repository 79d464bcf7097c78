// divonne_engine.h -- host driver of Divonne's partitioning phase.
#pragma once
#include "context.h"
#include "divonne.h"

namespace ccuba {

struct PartitionSpec {
  int ndim = 1, family = 0;
  double a[kMaxDim] = {0}, u[kMaxDim] = {0};
  unsigned long long seed = 0;
  uint32_t sid = 0;
  int nsearch = 256, niter = 32, maxregions = 64, nsplit = 1;
  double spread_tol = 0.0;
};

struct PartitionResult {
  int nregions = 0, fail = 1;
  long long neval = 0, nsplits = 0;
  double total_spread = 0.0, max_spread = 0.0;
};

// Host arrays the final regions are copied to (any pointer may be null).
struct PartitionTraceOut {
  int max_regions = 0, max_splits = 0;
  double *lo = nullptr, *hi = nullptr, *xmin = nullptr, *xmax = nullptr;
  double *fmin = nullptr, *fmax = nullptr, *spread = nullptr;
  int *cut = nullptr;
};

int validate_partition(const PartitionSpec &s);
int run_partition(ccuba_ctx *ctx, const PartitionSpec &spec, PartitionResult &res,
                  const PartitionTraceOut *tr, hipStream_t s);

}  // namespace ccuba
