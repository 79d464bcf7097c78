// suave.h -- Suave (subregion-adaptive Vegas) on the device: the regions of
// one integral, the per-step work lists and the kernel launchers.
//
// Suave's prototype (Sect. 3.2.2) takes nnew and flatness on top of Vegas's
// sampling arguments.  Every region keeps its own Vegas grid and the values
// of its own sample; a step bisects the regions of largest variance along the
// dimension whose halves fluctuate least, and samples each child with nnew
// points through the parent's grid restricted to the child.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.h"

namespace ccuba {

constexpr int kSuaveMaxSplit = 1024;  // regions split per step at most
constexpr int kSuaveBlock = 256;      // threads of the sampling workgroups
constexpr int kSuaveTile = 4096;      // points per sampling workgroup
constexpr int kSuaveChunk = 4096;     // sample points per split-statistics workgroup

// The regions of one integral in position order (device arrays).
struct SRegions {
  double *lo, *hi;          // [R][d] bounds
  double *grid;             // [R][d][N + 1] relative grid edges
  double *I, *var, *chi2;   // [R] combined estimate, its variance, chi^2
  int *dof;                 // [R] estimates combined - 1
  double *inh_I, *inh_var;  // [R] estimate inherited from the parent (var 0: none)
  double *v;                // [R][nnew] values of the region's own sample
  uint16_t *side;           // [R][nnew] bit j: the point lies in the upper half along j
};

// Totals over the regions after a step.
struct SState {
  double I, var, chi2, prob;
  int dof, pad;
};

struct SuaveArgs {
  SRegions R;
  int d, N, family, flags;
  long long nnew;
  uint32_t key0, key1, sid;
  int ntiles;             // sampling tiles per child
  int nchunks;            // split-statistics chunks per region
  double flatness;
  int ipow;               // flatness when it is a whole number in [1, 4096], else 0
  int pad;
  const double *p64;      // [2][kParamRow] integrand constants
  int *sel;               // [K] selected positions in selection order
  int *chpos, *chser;     // [2K] children's positions and sampling serials
  double *fl1;            // [K][nchunks][d][9] pass-1 split statistics
  double *fl2;            // [K][nchunks][d][2] pass-2 power sums
  double *hs;             // [K][d][10] pass 1 over all chunks: cnt, S1, S2, m, M per half
  double *tsum;           // [2K][ntiles][2] tile sums
  double *thist;          // [2K][ntiles][d N] tile histograms
  int *cut;               // [splits] dimension of every split, in order
  SState *state;
};

size_t suave_sample_lds(int d, int N);
size_t suave_fold_lds(int d, int N);
hipError_t suave_set_kernel_limits();
// the root region [0,1]^d with the uniform grid, to be sampled as child 0
hipError_t launch_suave_root(const SuaveArgs &A, hipStream_t s);
hipError_t launch_suave_select(const SuaveArgs &A, int R, int K, hipStream_t s);
// sel[0..K) = positions of the K largest of key[0..R) (all >= 0), largest
// first, ties to the lower position; 1 <= K <= min(R, kSuaveMaxSplit)
hipError_t launch_topk(const double *key, int R, int K, int *sel, hipStream_t s);
hipError_t launch_suave_fluct(const SuaveArgs &A, int K, hipStream_t s);
hipError_t launch_suave_split(const SuaveArgs &A, int R, long long Q, int K, hipStream_t s);
hipError_t launch_suave_sample(const SuaveArgs &A, int nchild, hipStream_t s);
hipError_t launch_suave_fold(const SuaveArgs &A, int nchild, hipStream_t s);
hipError_t launch_suave_totals(const SuaveArgs &A, int R, hipStream_t s);

}  // namespace ccuba
