// engine.h -- structures shared by the device kernels and the host drivers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace ccuba {

constexpr int kMaxDim = 16;
constexpr int kMaxBins = 256;  // bin indices are packed 4 per 32-bit word
constexpr int kGroupTiles = 32;  // tiles folded by one "last block" reduction
constexpr int kParamRow = kMaxDim;

enum Precision { FP64 = 0, FP32 = 1 };
enum Family { GAUSSIAN = 0, OSCILLATORY = 1, PRODUCT_PEAK = 2, CORNER_PEAK = 3, C0 = 4 };

// One Vegas integral, device resident.  Offsets index the engine's pools.
struct VJob {
  int ndim, nbins, family, prec;
  int flags;
  uint32_t key0, key1, sid;
  long long nstart, nincrease, mineval, maxeval;
  double epsrel, epsabs;
  int tile0, ntiles;      // tiles [tile0, tile0 + ntiles) of the tile list
  long long tile_pts;     // points per tile
  int group0;             // first reduction group
  int hist_cap;           // capacity of the per-iteration history
  long long grid_off;     // doubles: ndim * (nbins + 1)
  long long thist_off;    // doubles: ntiles * ndim * nbins
  long long ghist_off;    // doubles: ngroups * ndim * nbins
  long long iter_off;     // doubles: hist_cap
  int param_off;          // job index into the parameter pools
  int pad;
};

// Per-integral iteration state, written by the refine kernel.
struct VState {
  long long neval;
  int T;      // iterations completed
  int done;   // 1 once converged or out of budget
  int fail;   // 0 converged, 1 maxeval reached
  int dof;
  double integral, error, prob, chi2;
};

__host__ __device__ inline int ngroups_of(int ntiles) { return (ntiles + kGroupTiles - 1) / kGroupTiles; }

// Flags understood by the device code.
enum { FLAG_FREEZE_GRID = 1 << 4 };

// Launch geometry of the DoSample kernel.
struct VegasTune {
  int block = 256;        // threads per block
  int blocks_per_cu = 4;  // persistent blocks per compute unit
  int hist64 = 1;         // FP32 path: 1 = FP64 LDS histogram, 0 = FP32
  int tiles_per_job = 0;  // 0 = automatic (one tile per persistent block)
  long long min_tile = 4096;
};

}  // namespace ccuba
