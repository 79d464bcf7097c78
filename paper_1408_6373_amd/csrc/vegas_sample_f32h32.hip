// vegas_sample_f32h32.hip -- DoSample instances with FP32 evaluation, FP32 LDS histogram.
#include "vegas_sample.h"

namespace ccuba {

hipError_t launch_dosample_f32h32(const VegasArgs &A, int nb, bool pow2, bool full, int grid,
                              int block, size_t lds, hipStream_t s) {
  return launch_dosample_t<float, float>(A, nb, pow2, full, grid, block, lds, s);
}

void dosample_fns_f32h32(std::vector<const void *> &fns) { dosample_fns_t<float, float>(fns); }

}  // namespace ccuba
