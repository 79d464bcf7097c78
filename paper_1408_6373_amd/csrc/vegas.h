// vegas.h -- kernel arguments and launchers of the Vegas DoSample engine.
#pragma once
#include "engine.h"

namespace ccuba {

// Everything a DoSample / refine launch touches; all pointers are device
// memory owned by a VegasEngine.
struct VegasArgs {
  const VJob *jobs;
  VState *state;
  const int *tile_job;  // job of each tile
  int ntiles;
  int hist64;           // FP32 path: FP64 LDS histogram
  long long lds_hist_byte_off;
  double *grids;        // two copies per job (ping-pong by iteration parity)
  const double *p64;    // [job][2][kParamRow]
  const float *p32;     // [job][2][kParamRow]
  double *tile_sums;    // [tile][2]
  double *tile_hist;    // per job: [ntiles][d*N]
  double *group_sums;   // [group][2]
  double *group_hist;   // per job: [ngroups][d*N]
  unsigned *group_cnt;  // [group], zero between launches
  double *iter_I;       // per job: [hist_cap]
  double *iter_var;
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
