// vegas_sample_f64.hip -- DoSample instances with FP64 evaluation, FP64 LDS histogram
// (the grids whose fixed-point histogram would not fit the LDS, and the
// hist64 setting).
#include "vegas_sample.h"

namespace ccuba {

hipError_t launch_dosample_f64(const VegasArgs &A, int nb, bool pow2, bool full, int grid,
                              int block, size_t lds, hipStream_t s) {
  return launch_dosample_t<double, double>(A, nb, pow2, full, grid, block, lds, s);
}

void dosample_fns_f64(std::vector<const void *> &fns) { dosample_fns_t<double, double>(fns); }

}  // namespace ccuba
