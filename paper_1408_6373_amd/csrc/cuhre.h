// cuhre.h -- kernel arguments and launchers of the Cuhre DoSample engine.
#pragma once
#include "engine.h"

namespace ccuba {

// Structure-of-arrays store of the subregions of one integral (the resident
// region heap).  c and h are dimension-major: c[j * cap + r].
struct CRegions {
  double *c, *h;
  double *I7, *I5, *err;
  int *axis;
  long long *id;
  long long cap;
};

// A run of consecutive regions of one integral to evaluate in a rule launch.
struct CSeg {
  int ndim, family;
  const double *par;  // [2][kParamRow] Genz constants of the integral (FP64 row)
  long long first, count;
  CRegions regs;
};

struct RuleArgs {
  const CSeg *segs;          // device table (nseg > 1)
  int nseg;
  const long long *seg_end;  // inclusive prefix sums of the segment counts
  long long total;
  CSeg one;                  // the segment itself when nseg == 1 (no table)
  const double *w7, *w5;     // [ndim][5] rule weights (rows 0..16)
  double l2, l3, l4, l5;
};

// Per-integral scratch for selection, compaction and totals.
struct CScratch {
  unsigned long long *prefix;  // [2]: selected key prefix, mask
  long long *krem;             // [2]: remaining K, count of keys == threshold to take
  unsigned *hist;              // [256] radix digit histogram
  int *flag;                   // [cap] selection flags
  long long *bsum;             // [nblocks] block sums for scans
  double *tot;                 // [nblocks*2] partial totals, [2] final (I, err)
  long long nbmax;
};

hipError_t launch_rule(const RuleArgs &A, hipStream_t s);
// The root region of [0,1]^d (centre 1/2, half-width 1/2, id 0) at position 0.
hipError_t launch_root(const CRegions &R, int ndim, hipStream_t s);
// Top-K selection of n regions by (err desc, position asc): flag[i] = 1 for
// the K chosen.  Positions are in ascending id order.
hipError_t launch_select(const CRegions &R, long long n, long long K, const CScratch &S,
                         hipStream_t s);
// Copy unselected regions of `src' to the front of `dst' in order, the two
// children of the j-th selected region (ascending position) to
// dst[n - K + 2j], dst[n - K + 2j + 1], with ids next_id + 2j, + 2j + 1.
hipError_t launch_split(const CRegions &src, const CRegions &dst, int ndim, long long n,
                        long long K, long long next_id, bool all, const CScratch &S,
                        hipStream_t s);
// Fixed-order totals of I7 and err over n regions into S.tot[0], S.tot[1].
hipError_t launch_totals(const CRegions &R, long long n, const CScratch &S, double *out,
                         hipStream_t s);
long long scratch_blocks(long long n);
hipError_t cuhre_set_kernel_limits();

}  // namespace ccuba
