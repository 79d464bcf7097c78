// cuhre_engine.h -- host driver of Cuhre: one integral's resident region heap
// advanced one batch step at a time.
#pragma once
#include "context.h"
#include "cuhre.h"

namespace ccuba {

struct CuhreSpec {
  int ndim = 2, family = 0;
  double a[kMaxDim] = {0}, u[kMaxDim] = {0};
  double epsrel = 1e-3, epsabs = 0;
  long long mineval = 0, maxeval = 0, batch = 100000;
};

int validate_cuhre(const CuhreSpec &s);
long long gm_npoints(int ndim);

// Rule weights (w7, w5: [17][5]) and generators, from Genz & Malik (1980).
struct GMTables {
  double w7[17 * 5], w5[17 * 5];
  double l2, l3, l4, l5;
};
const GMTables &gm_tables();

class CuhreRun {
 public:
  explicit CuhreRun(ccuba_ctx *ctx) : ctx_(ctx) {}
  // Allocate, evaluate the root region (asynchronous).
  int start(const CuhreSpec &spec, hipStream_t s);
  // Totals of the current leaves into the device result (asynchronous).
  int launch_totals(hipStream_t s);
  // After the totals are read: decide, and if work remains select + split.
  // Returns 1 if a rule launch over new children is pending, 0 if finished.
  int plan_and_split(hipStream_t s);
  // The segment of children awaiting the rule (valid after plan_and_split
  // returned 1); the caller launches the rule, possibly with other segments.
  CSeg pending_segment() const;
  void commit_pending();
  // Copy the device totals to host (synchronous on s).
  int read_totals(hipStream_t s);
  // Write the totals to pinned host memory (host and device addresses of 2
  // doubles) instead; read_totals then reads them there and the caller must
  // have synchronised the stream since launch_totals.
  void set_mapped_totals(double *host, double *dev) {
    mapped_host_ = host;
    mapped_dev_ = dev;
  }
  // Run to completion alone.  The host queues each step's selection, split
  // and rule launch before it learns whether the step's totals end the run
  // (the totals kernel decides on the device and sets the run's stop flag,
  // which turns the queued launches into empty ones), so the device does not
  // wait for the host between steps.
  int run(hipStream_t s);
  int rule_only(long long nreg, const double *c, const double *h, double *I7, double *I5,
                double *err, int *axis, hipStream_t s);

  bool done() const { return done_; }
  int fail() const { return fail_; }
  long long neval() const { return neval_; }
  long long nregions() const { return n_; }  // live regions
  double integral() const { return I_; }
  double error() const { return E_; }
  int batches() const { return batches_; }
  const CuhreSpec &spec() const { return spec_; }
  size_t bytes() const;
  // (rows: step opening and rows of the next state; *blocks: the launch's
  // blocks, one row each)
  int launch_rule_alone(const CSeg &seg, hipStream_t s, const CRows *rows = nullptr,
                        long long *blocks = nullptr);
  const double *params_dev() const { return params_.p; }

 private:
  int ensure(long long need, hipStream_t s);
  int alloc_store(CRegions &R, DevBuf<double> &cb, DevBuf<double> &hb, DevBuf<double> &vals,
                  DevBuf<int> &ax, long long cap);
  int alloc_scratch(long long cap);
  // The segment of the 2K children of step with K splits: formed from the
  // live regions [next_id_ - n_, next_id_) when all split and they are
  // contiguous, else from the positions launch_split wrote.
  CSeg children_segment(long long K, bool from_range) const;
  ccuba_ctx *ctx_;
  CuhreSpec spec_;
  // n_ live regions among the next_id_ of the store (positions are ids)
  long long np_ = 0, n_ = 0, next_id_ = 1, neval_ = 0, cap_ = 0, pendK_ = 0;
  int fail_ = 1, batches_ = 0;
  bool done_ = false;
  bool contig_ = true;       // the live regions are the last n_ of the store
  bool pend_range_ = false;  // the pending children come from a range of parents
  // the current state's totals as rows (CRows) in half rows_par_ of tot_
  int rows_par_ = 0;
  long long rows_n_ = 0, rows_stride_ = 0;
  double I_ = 0, E_ = 0;
  CRegions R_{};
  DevBuf<double> c_, h_, vals_;
  DevBuf<int> axis_;
  DevBuf<unsigned long long> prefix_;
  DevBuf<long long> krem_, bsum_, parent_;
  DevBuf<unsigned> coarse_;
  DevBuf<double> tot_, out_, params_, w7_, w5_;
  DevBuf<int> stop_;  // the run's stop flag (CScratch::done)
  DevBuf<unsigned> hist16_;  // the top-K digit histogram (CScratch::hist16)
  DevBuf<unsigned long long> cand_key_, cand_cnt_;
  DevBuf<long long> cand_pos_;
  DevBuf<CSeg> seg_;
  DevBuf<long long> seg_end_;
  CScratch S_{};
  double hp64_[2][kParamRow];  // host source of the parameter upload
  double *mapped_host_ = nullptr, *mapped_dev_ = nullptr;
};

// Launch the rule over segments of several integrals in one kernel.  segs
// and ends are host arrays copied to the device buffers given.
int launch_rule_segments(ccuba_ctx *ctx, const CSeg *segs, int nseg, DevBuf<CSeg> &dsegs,
                         DevBuf<long long> &dends, const double *w7_dev, const double *w5_dev,
                         hipStream_t s, int *done = nullptr, const CRows *rows = nullptr,
                         long long *blocks = nullptr);

}  // namespace ccuba
