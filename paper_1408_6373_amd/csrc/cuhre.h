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
  const int *done;           // a run's stop flag (null: none): set, the launch does nothing
};

// Per-integral scratch for selection, compaction and totals.
struct CScratch {
  unsigned long long *prefix;  // [2]: selected key prefix, mask; then the threshold key
  long long *krem;             // [2]: remaining K, count of keys == threshold to take;
                               // then the threshold position
  int *flag;                   // [cap] selection flags
  long long *bsum;             // [nblocks] block sums for scans
  double *tot;                 // [nblocks*2] partial totals, [2] final (I, err)
  long long nbmax;
  // The run's stop flag, set on the device when a step's totals end the run
  // (null: none).  Every selection, split, totals and rule kernel launched
  // with it does nothing once it is set, so that a host that has queued the
  // next step before learning the outcome of this one loses nothing but the
  // empty launches.
  int *done;
  // top-K by a 16-bit first digit: the digit histogram (zero between uses),
  // and the keys and positions of the boundary digit's regions ([cap] each)
  unsigned *hist16;
  unsigned long long *cand_key;
  long long *cand_pos;
  unsigned long long *cand_cnt;  // [1]
};

// What ends a run after a step's totals: the accuracy test (neval >= mineval
// and err <= max(epsabs, epsrel |I|)) or a total that is not finite.
struct CStop {
  double epsrel, epsabs;
  long long mineval, neval;
};

hipError_t launch_rule(const RuleArgs &A, hipStream_t s);
// The root region of [0,1]^d (centre 1/2, half-width 1/2, id 0) at position 0.
hipError_t launch_root(const CRegions &R, int ndim, hipStream_t s);
// Top-K selection of n regions by (err desc, position asc), positions in
// ascending id order: a histogram of the keys' top 16 bits finds the boundary
// digit, then an exact rank among the boundary digit's regions only gives the
// threshold (key, position), written to S.prefix[0], S.krem[0]; launch_split's
// counting pass sets the flags of the K chosen.
hipError_t launch_select16(const CRegions &R, long long n, long long K, const CScratch &S,
                           hipStream_t s);
// Copy unselected regions of `src' to the front of `dst' in order, the two
// children of the j-th selected region (ascending position) to
// dst[n - K + 2j], dst[n - K + 2j + 1], with ids next_id + 2j, + 2j + 1.
// Unless all regions split, the selection is the threshold that
// launch_select16 left in S.
hipError_t launch_split(const CRegions &src, const CRegions &dst, int ndim, long long n,
                        long long K, long long next_id, bool all, const CScratch &S,
                        hipStream_t s);
// Fixed-order totals of I7 and err over n regions into out[0], out[1].
hipError_t launch_totals(const CRegions &R, long long n, const CScratch &S, double *out,
                         hipStream_t s);
// The same, then the stop rule of `stop': out[2] = 0 (go on), 1 (converged)
// or 2 (a total is not finite), and in the last two cases S.done is set.
// Nothing is written once S.done is set.
hipError_t launch_totals_decide(const CRegions &R, long long n, const CScratch &S, double *out,
                                const CStop &stop, hipStream_t s);
// The root region, and the run's stop flag cleared.
hipError_t launch_root_clear(const CRegions &R, int ndim, int *done, hipStream_t s);
long long scratch_blocks(long long n);
hipError_t cuhre_set_kernel_limits();

}  // namespace ccuba
