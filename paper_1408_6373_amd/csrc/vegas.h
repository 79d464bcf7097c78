// vegas.h -- kernel arguments and launchers of the Vegas DoSample engine.
#pragma once
#include "engine.h"

namespace ccuba {

// Everything a DoSample / refine launch touches: the job table (device
// memory) and the launch's tile list.
struct VegasArgs {
  const VJob *jobs;
  const int *tile_job;  // job of each tile
  int tile_first;       // the launch's slice of the tile list
  int tile_count;
  int hist64;           // FP32 path: FP64 LDS histogram
  int ilp;              // points per lane per trip (1 or 2)
  long long lds_hist_byte_off;
};

// The fold launch: task_end[j] = inclusive prefix over jobs of
// ngroups(ntiles_j) * ceil(ndim_j * nbins_j / 64) wavefront tasks.
struct FoldArgs {
  const VJob *jobs;
  const long long *task_end;   // level 1 tasks
  int njobs;
  long long total;
  const long long *task_end2;  // level 2: ceil(ndim * nbins / 64) per job
  long long total2;
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

// Launch the DoSample instance of precision `prec', `nb' Philox blocks per
// point and power-of-two bin count or not over the slice of the tile list in A.
hipError_t launch_dosample(const VegasArgs &A, int prec, int nb, bool pow2, int grid, int block,
                           size_t lds, hipStream_t s);
hipError_t launch_fold(const FoldArgs &F, hipStream_t s);
hipError_t launch_refine(const VegasArgs &A, int njobs, size_t lds, hipStream_t s);
hipError_t launch_collect(const VegasArgs &A, int njobs, double *sums, double *hist,
                          hipStream_t s);
hipError_t launch_points(const PointsArgs &P, hipStream_t s);
hipError_t set_kernel_limits();

}  // namespace ccuba
