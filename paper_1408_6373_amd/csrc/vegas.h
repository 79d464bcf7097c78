// vegas.h -- kernel arguments and launchers of the Vegas DoSample engine.
#pragma once
#ifndef CCUBA_RTC
#include <vector>
#endif

#include "engine.h"

namespace ccuba {

// Everything a DoSample / refine launch touches: the job table (device
// memory) and the launch's tile list.
struct VegasArgs {
  const VJob *jobs;
  const int *tile_job;  // job of each tile
  int tile_first;       // the launch's slice of the tile list
  int tile_count;
  int hist64;           // FP64 LDS histogram (else the exact 64-bit fixed-point one)
  int ilp;              // points per lane per trip (1 or 2)
  long long lds_hist_byte_off;
  int njobs;  // jobs in the table (1: every tile is job 0's)
  int pad;
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

// Caller-evaluated integrands (points in batches; see vegas_batched.cpp).
constexpr int kMaxComp = 16;  // integrand components
struct BatchedArgs {
  int ndim, nbins, ncomp, prec;
  long long npts;       // points of this batch
  int tile_pts;         // points per tile row
  int tile_base;        // row of the batch's first tile
  const double *w;      // [npts]
  const double *f;      // [npts][ncomp]
  const int *bin;       // [npts][ndim]
  double *rows;         // [tiles][2 ncomp + ndim nbins]: S1, S2 per component, H
  const VState *state;  // [ncomp]: the shift of each component's sums
};
struct BatchedFinishArgs {
  int ndim, nbins, ncomp, flags;
  int ngroups;               // group rows of the iteration
  const double *ghist;       // [ngroups][2 ncomp + ndim nbins]
  double *grid;              // ndim (nbins + 1) edges, refined in place
  VState *state;             // [ncomp]
  double *iter_I, *iter_var; // [ncomp][hist_cap]
  int hist_cap;
  int pad;
  long long nstart, nincrease, mineval, maxeval;
  double epsrel, epsabs;
};
#ifndef CCUBA_RTC  // host launchers (not part of a run-time compiled kernel)
// One tile row per block of tile_pts points of the batch.
hipError_t launch_batched_accumulate(const BatchedArgs &B, hipStream_t s);
// The last fold level, every component's statistics, the joint stop rule and
// the refinement of the grid from component 0's histogram (one workgroup).
hipError_t launch_batched_finish(const BatchedFinishArgs &F, hipStream_t s);

// Launch the DoSample instance of precision `prec', `nb' Philox blocks per
// point, power-of-two bin count or not and d = 4 nb or not over the slice of
// the tile list in A.
hipError_t launch_dosample(const VegasArgs &A, int prec, int nb, bool pow2, bool full,
                           int grid, int block, size_t lds, hipStream_t s);
// the same per (precision, histogram type), one translation unit each
hipError_t launch_dosample_f64(const VegasArgs &A, int nb, bool pow2, bool full, int grid,
                               int block, size_t lds, hipStream_t s);
hipError_t launch_dosample_f32h64(const VegasArgs &A, int nb, bool pow2, bool full, int grid,
                                  int block, size_t lds, hipStream_t s);
hipError_t launch_dosample_f64hfx(const VegasArgs &A, int nb, bool pow2, bool full, int grid,
                                  int block, size_t lds, hipStream_t s);
hipError_t launch_dosample_f32hfx(const VegasArgs &A, int nb, bool pow2, bool full, int grid,
                                  int block, size_t lds, hipStream_t s);
// every DoSample instance of a translation unit (for launch attributes)
void dosample_fns_f64(std::vector<const void *> &fns);
void dosample_fns_f32h64(std::vector<const void *> &fns);
void dosample_fns_f32hfx(std::vector<const void *> &fns);
void dosample_fns_f64hfx(std::vector<const void *> &fns);
// First fold level (tile rows -> group rows); with level2 also the second
// (group rows -> hsum), which only the raw DoSample entry point needs.
hipError_t launch_fold(const FoldArgs &F, bool level2, hipStream_t s);
// The refine kernel over njobs integrals, one workgroup per (integral,
// dimension); dmax: the largest dimension among them.
hipError_t launch_refine(const VegasArgs &A, int njobs, int dmax, hipStream_t s);
// Uniform starting grids of jobs[0, njobs) (device table).
hipError_t launch_init_grids(const VJob *jobs, int njobs, hipStream_t s);
// The same for one grid of ndim rows of nbins + 1 edges.
hipError_t launch_init_grid(double *grid, int ndim, int nbins, hipStream_t s);
hipError_t launch_collect(const VegasArgs &A, int njobs, double *sums, double *hist,
                          hipStream_t s);
hipError_t launch_points(const PointsArgs &P, hipStream_t s);
hipError_t set_kernel_limits();
#endif

}  // namespace ccuba
