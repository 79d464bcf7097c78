// tune.h -- launch-geometry autotuner of the DoSample kernel.
#pragma once
#include "context.h"

namespace ccuba {

// Pick block size, persistent blocks per CU and (FP32) histogram precision
// for precision `prec' by timing DoSample on a fixed synthetic integral, once
// per context; the choice is cached in the file named by CCUBA_TUNE_CACHE.
void maybe_autotune(ccuba_ctx *ctx, int prec);

}  // namespace ccuba
