// cuhre.h -- kernel arguments and launchers of the Cuhre DoSample engine.
#pragma once
#include "engine.h"

namespace ccuba {

// Structure-of-arrays store of the subregions of one integral (the resident
// region heap).  c and h are dimension-major: c[j * cap + r].  The store only
// grows, so a region's position is its id: the root is 0, and the children
// of the j-th region split in a step (in position order) go to next + 2j and
// next + 2j + 1, next being the store's length before the step.  A region
// that has been split stays where it is, retired: its error is set to -1,
// which no live region's |I7 - I5| can be.
struct CRegions {
  double *c, *h;
  double *I7, *I5, *err;
  int *axis;
  long long cap;
};

// A run of consecutive regions of one integral to evaluate in a rule launch.
struct CSeg {
  int ndim, family;
  const double *par;  // [2][kParamRow] Genz constants of the integral (FP64 row)
  long long first, count;
  CRegions regs;
  // children != 0 (count even): regions first + 2j and first + 2j + 1 are
  // the lower and upper halves, along its split axis, of the region at
  // position parent[j] (parent set) or pbase + j (parent null); the rule
  // launch forms and stores their centres and widths first.  With retire,
  // the lower child's thread also retires the parent.  children == 0: the
  // regions' centres and widths are already in the store.
  int children, retire;
  const long long *parent;
  long long pbase;
};

// What ends a run after a step's totals: the accuracy test (neval >= mineval
// and err <= max(epsabs, epsrel |I|)) or a total that is not finite.
struct CStop {
  double epsrel, epsabs;
  long long mineval, neval;
};

// The totals of a state as rows: row r holds one block's sums of I7 (at
// r) and err (at stride + r) over its share of the live regions.  A launch
// that opens a step (in set) first sums the nin rows in row order in every
// block, so that all blocks reach the same outcome, and applies the stop
// rule: block 0 writes I and err to slot[0..1] and then, as one 64-bit
// system-scope store, seq << 8 | outcome (0 go on, 1 converged, 2 not
// finite) to slot[2], so that a host polling slot[2] in host-coherent memory
// learns the outcome while the launch still runs (I and err are complete
// once the stream has finished the launch); unless the outcome is 0 it sets
// the run's stop flag, and the launch then does nothing.  A launch that
// produces rows of the next state (out set) writes one row per block from
// row out0 on.
struct CRows {
  const double *in;
  long long nin;
  double *out;
  long long out0;
  long long stride;
  double *slot;
  long long seq;
  CStop stop;
};

struct RuleArgs {
  const CSeg *segs;          // device table (nseg > 1)
  int nseg;
  const long long *seg_end;  // inclusive prefix sums of the segment counts
  long long total;
  CSeg one;                  // the segment itself when nseg == 1 (no table)
  const double *w7, *w5;     // [ndim][5] rule weights (rows 0..16)
  double l2, l3, l4, l5;
  int *done;                 // a run's stop flag (null: none): set, the launch does nothing
  CRows rows;                // step opening and rows of the next state (zero: neither)
};

// Per-integral scratch for selection, splitting and totals.
struct CScratch {
  unsigned long long *prefix;  // [1]: the boundary digit, then the threshold key
  long long *krem;             // [1]: the rank wanted within the digit, then the
                               // threshold position
  long long *bsum;             // [nblocks] block counts, then their exclusive scan
  double *tot;                 // [nblocks*2] partial totals (launch_totals)
  long long nbmax;
  long long *parent;           // [cap / 2] positions of the regions split in a step
  // The run's stop flag, set on the device when a step's totals end the run
  // (null: none).  Every selection, split, totals and rule kernel launched
  // with it does nothing once it is set, so that a host that has queued the
  // next step before learning the outcome of this one loses nothing but the
  // empty launches.
  int *done;
  // top-K by a 16-bit first digit: the digit histogram and the histogram of
  // its top 8 bits (zero between uses), and the keys and positions of the
  // boundary digit's regions ([cap] each)
  unsigned *hist16;
  unsigned *coarse;
  unsigned long long *cand_key;
  long long *cand_pos;
  unsigned long long *cand_cnt;  // [1]
};

hipError_t launch_rule(const RuleArgs &A, hipStream_t s);
// Blocks of the rule launch that launch_rule makes for A (one row each).
long long rule_blocks(const RuleArgs &A);
// Top-K selection among the m regions of a store (retired ones never
// qualify) by (err desc, position asc): a histogram of the keys' top 16 bits
// finds the boundary digit, then an exact rank among the boundary digit's
// regions only gives the threshold (key, position), written to S.prefix[0],
// S.krem[0].
hipError_t launch_select16(const CRegions &R, long long m, long long K, const CScratch &S,
                           hipStream_t s, const CRows *open = nullptr);
// The split of the K regions at or above the threshold that launch_select16
// left in S: each is retired and its position written to S.parent[j], j its
// rank in position order.  A rule launch in children mode (CSeg::parent =
// S.parent) then forms and evaluates the children.  With rows (out set),
// the sums of the regions that stay live go to split_rows(m) rows.  Clears
// the top-K histograms for the next selection.
hipError_t launch_split(const CRegions &R, long long m, long long K, const CScratch &S,
                        hipStream_t s, const CRows *rows = nullptr);
long long split_rows(long long m);
// Most rows a state of a store of cap regions can have (split rows plus the
// rule launch's).
long long step_rows(long long cap);
// A launch that only opens a step (decides on rows.in).
hipError_t launch_decide(const CRows &rows, int *done, hipStream_t s);
// Fixed-order totals of I7 and err over the live regions among the m of a
// store into out[0], out[1].
hipError_t launch_totals(const CRegions &R, long long m, const CScratch &S, double *out,
                         hipStream_t s);
// The root region of [0,1]^d (centre 1/2, half-width 1/2) at position 0, and
// the run's stop flag cleared (done may be null).
hipError_t launch_root_clear(const CRegions &R, int ndim, int *done, hipStream_t s);
long long scratch_blocks(long long n);

hipError_t cuhre_set_kernel_limits();

}  // namespace ccuba
