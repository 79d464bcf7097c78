// vegas.h -- kernel arguments and launchers of the Vegas DoSample engine.
#pragma once
#include "engine.h"

namespace ccuba {

// Everything a DoSample / refine launch touches: the job table (device
// memory) and the launch's tile list.
struct VegasArgs {
  const VJob *jobs;
  const int *tile_job;  // job of each tile
  int ntiles;
  int hist64;           // FP32 path: FP64 LDS histogram
  long long lds_hist_byte_off;
};

struct PointsArgs {
  int ndim, nbins, prec, iteration;
  uint32_t key0, key1, sid;
  long long i0, npts;
  const double *grid;  // ndim * (nbins + 1)
  uint32_t *words;     // npts * 4 * ceil(ndim/4)
  double *x;           // npts * ndim
  double *w;           // npts
  int *bin;            // npts * ndim
};

hipError_t launch_dosample(const VegasArgs &A, int prec, int grid, int block, size_t lds,
                           hipStream_t s);
hipError_t launch_refine(const VegasArgs &A, int njobs, size_t lds, hipStream_t s);
hipError_t launch_collect(const VegasArgs &A, int njobs, double *sums, double *hist,
                          hipStream_t s);
hipError_t launch_points(const PointsArgs &P, hipStream_t s);
hipError_t set_kernel_limits();

}  // namespace ccuba
