// tune.h -- launch-geometry autotuner of the DoSample kernel.
#pragma once
#include <vector>

#include "context.h"

namespace ccuba {

// Pick block size, persistent blocks per CU and (FP32) histogram precision
// for precision `prec' by timing DoSample on a fixed synthetic integral, once
// per context; the choice is cached in the file named by CCUBA_TUNE_CACHE.
void maybe_autotune(ccuba_ctx *ctx, int prec);

// The same for a batch, timed on the batch itself: a few full iterations
// over the jobs of each precision for every candidate (persistent blocks per
// CU, points per lane per trip, smallest tile, histogram type, and for 2+
// jobs one stream or two halves on two), run as the batch call runs them,
// once per context and precision; the choice is cached in the file named by
// CCUBA_TUNE_CACHE under a signature of the jobs' shapes.
struct VegasSpec;
void autotune_batch(ccuba_ctx *ctx, const std::vector<VegasSpec> &specs);

}  // namespace ccuba
