// vegas_sample_f32hfx.hip -- DoSample instances with FP32 evaluation and a
// 64-bit fixed-point LDS histogram.
#include "vegas_sample.h"

namespace ccuba {

hipError_t launch_dosample_f32hfx(const VegasArgs &A, int nb, bool pow2, bool full, int grid,
                                  int block, size_t lds, hipStream_t s) {
  return launch_dosample_t<float, unsigned long long>(A, nb, pow2, full, grid, block, lds, s);
}

void dosample_fns_f32hfx(std::vector<const void *> &fns) {
  dosample_fns_t<float, unsigned long long>(fns);
}

}  // namespace ccuba
