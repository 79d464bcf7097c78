// engine.h -- structures shared by the device kernels and the host drivers.
#pragma once
#ifndef CCUBA_RTC  // (hiprtc provides the HIP runtime and its integer types)
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#ifndef CCUBA_RTC  // (absent when the kernels are compiled at run time)
#include <vector>
#endif

namespace ccuba {

constexpr int kMaxDim = 16;
constexpr int kMaxBins = 256;  // bin indices are packed 4 per 32-bit word
constexpr int kGroupTiles = 32;  // tiles folded by one wavefront of the fold kernel
constexpr int kParamRow = kMaxDim;

enum Precision { FP64 = 0, FP32 = 1 };
enum Family { GAUSSIAN = 0, OSCILLATORY = 1, PRODUCT_PEAK = 2, CORNER_PEAK = 3, C0 = 4,
              // a caller's device function, compiled at run time with the kernel
              USER = 5 };

struct VState;

// One Vegas integral, device resident: its settings and the device buffers it
// owns (or that an engine carved out of its pools for it).
struct VJob {
  int ndim, nbins, family, prec;
  int flags;
  uint32_t key0, key1, sid;
  long long nstart, nincrease, mineval, maxeval;
  double epsrel, epsabs;
  int tile0, ntiles;      // tiles [tile0, tile0 + ntiles) of the launch's tile list
  long long tile_pts;     // points per tile
  int hist_cap;           // capacity of the per-iteration history
  int pad;
  VState *state;
  // the state as the iteration's fold found it (null: no refine follows):
  // the refine kernel's workgroups read it, so that none of them reads a
  // state that another one has already advanced
  VState *snap;
  double *grid;           // ndim * (nbins + 1) edges, refined in place
  double *tsums;          // [ntiles][2]
  double *thist;          // [ntiles][ndim * nbins]
  double *gsums;          // [ngroups][2]
  double *ghist;          // [ngroups][ndim * nbins]
  double *hsum;           // [2 + ndim * nbins]: S1, S2 and the folded histogram
  double *iter_I;         // [hist_cap]
  double *iter_var;       // [hist_cap]
  const double *p64;      // [2][kParamRow]
  const float *p32;       // [2][kParamRow]
};

// Per-integral iteration state, written by the refine kernel.
struct VState {
  long long neval;
  int T;      // iterations completed
  int done;   // 1 once converged or out of budget
  int fail;   // 0 converged, 1 maxeval reached
  int dof;
  double integral, error, prob, chi2;
  // running sums of the combination over iterations t < T, in order
  double sum_w, sum_wI;  // sum 1/sigma_t^2, sum I_t/sigma_t^2
  double sum_zI;         // sum of I_t over iterations with sigma_t = 0
  int nzero;             // number of such iterations
  int pad;
  // cap on v^2 for the next iteration's fixed-point histogram (FP32
  // evaluation): 1024 times the mean v^2 of the last iteration, 0 before the
  // first
  float hcap;
  int pad2;
  // the value the next iteration's sums are taken about: its lanes sum
  // v - shift and (v - shift)^2, and shift is the last iteration's estimate
  // (0 before the first), so that the variance S2/n - (S1/n)^2 does not lose
  // the digits that the plain sums of v and v^2 lose to cancellation when
  // the variance is small against I^2
  double shift;
};

__host__ __device__ inline int ngroups_of(int ntiles) { return (ntiles + kGroupTiles - 1) / kGroupTiles; }

// Flags understood by the device code.
enum { FLAG_FREEZE_GRID = 1 << 4 };

// Launch geometry of the DoSample kernel.
struct VegasTune {
  int block = 256;        // threads per block
  int blocks_per_cu = 3;  // persistent blocks per compute unit
  int hist64 = 0;         // 1 = FP64 LDS histogram, 0 = the exact 64-bit fixed-point one
  int ilp = 1;            // points per lane per trip (1 or 2)
  int tiles_per_job = 0;  // 0 = automatic (one tile per persistent block)
  long long min_tile = 4096;
  int streams = 2;        // a batch of 2+ integrals: 2 = two halves on two streams
};

}  // namespace ccuba
