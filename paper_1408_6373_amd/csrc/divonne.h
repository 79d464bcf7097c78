// divonne.h -- Divonne's partitioning phase on the device (Sect. 2.2): the
// regions of one integral with their extrema and spreads, and the launchers.
//
// The paper hands every worker an entire region to search and subdivide
// instead of a list of points; here every region's search is one workgroup,
// and all the regions of a step are searched by one launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.h"

namespace ccuba {

constexpr int kDivBlock = 128;  // two wavefronts: the maximum's search and the minimum's

struct DRegions {
  double *lo, *hi;          // [R][d] bounds
  double *xmin, *xmax;      // [R][d] the extrema's points
  double *fmin, *fmax;      // [R]
  double *spread;           // [R] 1/2 Vol (fmax - fmin)
};

struct DState {
  double max_spread, total_spread;
};

struct DivArgs {
  DRegions R;
  int d, family;
  uint32_t key0, key1, sid;
  int nsearch, niter;
  const double *p64;      // [2][kParamRow] integrand constants
  int *sel;               // [K] selected positions
  int *chpos, *chser;     // [2K] children's positions and search serials
  int *cut;               // [splits] dimension of every split, in order
  DState *state;
};

hipError_t launch_div_root(const DivArgs &A, hipStream_t s);
hipError_t launch_div_search(const DivArgs &A, int nchild, hipStream_t s);
hipError_t launch_div_split(const DivArgs &A, int R, long long Q, int K, hipStream_t s);
hipError_t launch_div_totals(const DivArgs &A, int R, hipStream_t s);

}  // namespace ccuba
