// vegas_sample_f64hfx.hip -- DoSample instances with FP64 evaluation and an
// exact 64-bit fixed-point LDS histogram (two integer sums per bin).
#include "vegas_sample.h"

namespace ccuba {

hipError_t launch_dosample_f64hfx(const VegasArgs &A, int nb, bool pow2, bool full, int grid,
                                  int block, size_t lds, hipStream_t s) {
  return launch_dosample_t<double, unsigned long long>(A, nb, pow2, full, grid, block, lds, s);
}

void dosample_fns_f64hfx(std::vector<const void *> &fns) {
  dosample_fns_t<double, unsigned long long>(fns);
}

}  // namespace ccuba
