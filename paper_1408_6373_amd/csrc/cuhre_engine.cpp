// cuhre_engine.cpp -- host driver of Cuhre (globally adaptive subdivision in
// batches; see cuhre.hip for the kernels).
//
// Readings where the paper is silent (it only fixes the interface, Sect.
// 3.2.2): error |I7 - I5|; each step splits the K = min(B/2, #regions)
// regions of largest error (ties: lower id), K shrinking so that neval never
// passes maxeval; the run ends when neval >= mineval and the summed error is
// within max(epsabs, epsrel |I|) (fail 0) or when no child fits maxeval
// (fail 1); the root is region 0 and the j-th selected parent in id order
// gets children next+2j (lower half) and next+2j+1; prob = 0.
#include "cuhre_engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "genz.h"
#include "vegas_engine.h"

namespace ccuba {

long long gm_npoints(int d) { return (1ll << d) + 2ll * d * d + 2ll * d + 1; }

int validate_cuhre(const CuhreSpec &s) {
  if (s.ndim < 2 || s.ndim > kMaxDim || s.family < 0 || s.family > 4 || s.batch < 2 ||
      s.maxeval < 0 || !(s.epsrel >= 0) || !(s.epsabs >= 0))
    return CCUBA_EINVAL;
  for (int j = 0; j < s.ndim; ++j)
    if (!std::isfinite(s.a[j]) || !std::isfinite(s.u[j])) return CCUBA_EINVAL;
  return CCUBA_OK;
}

const GMTables &gm_tables() {
  static GMTables T = [] {
    GMTables t{};
    for (int d = 0; d <= 16; ++d) {
      const double p2 = std::ldexp(1.0, d), dd = d;
      double *w7 = t.w7 + 5 * d, *w5 = t.w5 + 5 * d;
      w7[0] = p2 * (12824.0 - 9120.0 * dd + 400.0 * dd * dd) / 19683.0;
      w7[1] = p2 * 980.0 / 6561.0;
      w7[2] = p2 * (1820.0 - 400.0 * dd) / 19683.0;
      w7[3] = p2 * 200.0 / 19683.0;
      w7[4] = 6859.0 / 19683.0;
      w5[0] = p2 * (729.0 - 950.0 * dd + 50.0 * dd * dd) / 729.0;
      w5[1] = p2 * 245.0 / 486.0;
      w5[2] = p2 * (265.0 - 100.0 * dd) / 1458.0;
      w5[3] = p2 * 25.0 / 729.0;
      w5[4] = 0.0;
    }
    t.l2 = std::sqrt(9.0 / 70.0);
    t.l3 = std::sqrt(9.0 / 10.0);
    t.l4 = std::sqrt(9.0 / 10.0);
    t.l5 = std::sqrt(9.0 / 19.0);
    return t;
  }();
  return T;
}

// bytes of store per region (centre, width, I7, I5, err, axis) and of the
// selection scratch (candidate key and position, parent position)
static double region_bytes(int d) { return (2.0 * d + 3.0) * 8.0 + 4.0 + 16.0 + 4.0; }

size_t CuhreRun::bytes() const { return (size_t)((double)cap_ * region_bytes(spec_.ndim)); }

int CuhreRun::alloc_store(CRegions &R, DevBuf<double> &cb, DevBuf<double> &hb,
                          DevBuf<double> &vals, DevBuf<int> &ax, long long cap) {
  const int d = spec_.ndim;
  int rc;
  if ((rc = cb.alloc(ctx_, (size_t)d * cap)) || (rc = hb.alloc(ctx_, (size_t)d * cap)) ||
      (rc = vals.alloc(ctx_, (size_t)3 * cap)) || (rc = ax.alloc(ctx_, cap)))
    return rc;
  R.c = cb.p;
  R.h = hb.p;
  R.I7 = vals.p;
  R.I5 = vals.p + cap;
  R.err = vals.p + 2 * cap;
  R.axis = ax.p;
  R.cap = cap;
  return CCUBA_OK;
}

// Scratch sized for a store of cap regions.
int CuhreRun::alloc_scratch(long long cap) {
  int rc;
  const long long nb = scratch_blocks(cap);
  rows_stride_ = step_rows(cap);
  // two halves of rows (this state's and the next), each I rows then err rows
  if ((rc = bsum_.alloc(ctx_, nb)) || (rc = tot_.alloc(ctx_, 4 * rows_stride_)) ||
      (rc = parent_.alloc(ctx_, cap / 2 + 1)) || (rc = cand_key_.alloc(ctx_, cap)) ||
      (rc = cand_pos_.alloc(ctx_, cap)))
    return rc;
  // (positions read by a rule launch are always in the store)
  CCUBA_HIP(hipMemset(parent_.p, 0, parent_.n * sizeof(long long)));
  S_.cand_key = cand_key_.p;
  S_.cand_pos = cand_pos_.p;
  S_.parent = parent_.p;
  S_.bsum = bsum_.p;
  S_.tot = tot_.p;
  S_.nbmax = nb;
  return CCUBA_OK;
}

// Grow the store to hold `need' regions, keeping the first next_id_.
int CuhreRun::ensure(long long need, hipStream_t s) {
  if (need <= cap_) return CCUBA_OK;
  long long cap = std::max<long long>(cap_ * 4, need);
  const long long limit = spec_.maxeval / np_ + 2;  // no run can hold more regions
  cap = std::max(need, std::min(cap, limit));
  const int d = spec_.ndim;
  // a tight budget: grow only as needed (the new store must fit beside what
  // the context holds now, the old store included; size-class slack 1.25)
  const double per = region_bytes(d) * 1.25;
  if ((double)ctx_->used.load() + per * (double)cap + 65536.0 > (double)ctx_->budget) cap = need;
  CRegions R{};
  DevBuf<double> cb, hb, vals;
  DevBuf<int> ax;
  int rc = alloc_store(R, cb, hb, vals, ax, cap);
  if (rc) return rc;
  const CRegions &O = R_;
  const long long m = next_id_;
  if (m > 0) {
    for (int j = 0; j < d; ++j) {
      CCUBA_HIP(hipMemcpyAsync(R.c + j * cap, O.c + j * O.cap, m * 8, hipMemcpyDeviceToDevice, s));
      CCUBA_HIP(hipMemcpyAsync(R.h + j * cap, O.h + j * O.cap, m * 8, hipMemcpyDeviceToDevice, s));
    }
    CCUBA_HIP(hipMemcpyAsync(R.I7, O.I7, m * 8, hipMemcpyDeviceToDevice, s));
    CCUBA_HIP(hipMemcpyAsync(R.I5, O.I5, m * 8, hipMemcpyDeviceToDevice, s));
    CCUBA_HIP(hipMemcpyAsync(R.err, O.err, m * 8, hipMemcpyDeviceToDevice, s));
    CCUBA_HIP(hipMemcpyAsync(R.axis, O.axis, m * 4, hipMemcpyDeviceToDevice, s));
  }
  CCUBA_HIP(hipStreamSynchronize(s));
  c_.swap(cb);
  h_.swap(hb);
  vals_.swap(vals);
  axis_.swap(ax);
  R_ = R;
  cb.release();
  hb.release();
  vals.release();
  ax.release();
  if ((rc = alloc_scratch(cap))) return rc;
  cap_ = cap;
  return CCUBA_OK;
}

int CuhreRun::start(const CuhreSpec &spec, hipStream_t s) {
  if (validate_cuhre(spec)) return CCUBA_EINVAL;
  spec_ = spec;
  const int d = spec.ndim;
  np_ = gm_npoints(d);
  n_ = 0;
  next_id_ = 1;
  neval_ = 0;
  batches_ = 0;
  done_ = false;
  contig_ = true;
  fail_ = 1;
  cap_ = 0;
  int rc;
  if ((rc = prefix_.alloc(ctx_, 1)) || (rc = krem_.alloc(ctx_, 1)) ||
      (rc = out_.alloc(ctx_, 2)) ||
      (rc = params_.alloc(ctx_, 2 * kParamRow)) || (rc = w7_.alloc(ctx_, 17 * 5)) ||
      (rc = w5_.alloc(ctx_, 17 * 5)) || (rc = seg_.alloc(ctx_, 1)) ||
      (rc = seg_end_.alloc(ctx_, 1)) || (rc = stop_.alloc(ctx_, 1)) ||
      (rc = hist16_.alloc(ctx_, 1 << 16)) || (rc = coarse_.alloc(ctx_, 256)) ||
      (rc = cand_cnt_.alloc(ctx_, 1)))
    return rc;
  S_.done = stop_.p;
  S_.hist16 = hist16_.p;
  S_.coarse = coarse_.p;
  S_.cand_cnt = cand_cnt_.p;
  // (the top-K kernels leave the histograms cleared after every use)
  CCUBA_HIP(hipMemsetAsync(hist16_.p, 0, (1 << 16) * sizeof(unsigned), s));
  CCUBA_HIP(hipMemsetAsync(coarse_.p, 0, 256 * sizeof(unsigned), s));
  S_.prefix = prefix_.p;
  S_.krem = krem_.p;
  // room for the first few batches, so that the store rarely grows (growing
  // means a new allocation and a copy)
  const long long first_cap = std::max<long long>(
      16, std::min<long long>(std::min<long long>(8 * spec.batch + 1, 1 << 23),
                              spec.maxeval / np_ + 2));
  // the initial store (room for one batch only if a tight budget refuses more)
  long long cap0 = first_cap;
  for (;;) {
    rc = alloc_store(R_, c_, h_, vals_, axis_, cap0);
    if (rc != CCUBA_ENOMEM) break;
    const long long small = std::max<long long>(
        16, std::min<long long>(2 * spec.batch + 1, spec.maxeval / np_ + 2));
    if (cap0 <= small) break;
    cap0 = small;
  }
  if (rc) return rc;
  if ((rc = alloc_scratch(cap0))) return rc;
  cap_ = cap0;
  // constants
  VegasSpec vs;
  vs.ndim = d;
  vs.family = spec.family;
  for (int j = 0; j < d; ++j) {
    vs.a[j] = spec.a[j];
    vs.u[j] = spec.u[j];
  }
  float p32[2][kParamRow];
  genz_constants(vs, hp64_, p32);
  const GMTables &T = gm_tables();
  // (host sources: members and static tables, alive while the copies run)
  CCUBA_HIP(hipMemcpyAsync(params_.p, hp64_, sizeof(hp64_), hipMemcpyHostToDevice, s));
  CCUBA_HIP(hipMemcpyAsync(w7_.p, T.w7, sizeof(T.w7), hipMemcpyHostToDevice, s));
  CCUBA_HIP(hipMemcpyAsync(w5_.p, T.w5, sizeof(T.w5), hipMemcpyHostToDevice, s));
  // root region [0,1]^d: centre 1/2, half-width 1/2, id 0; the stop flag clear
  CCUBA_HIP(launch_root_clear(R_, d, stop_.p, s));
  CSeg seg{};
  seg.ndim = d;
  seg.family = spec.family;
  seg.par = params_.p;
  seg.first = 0;
  seg.count = 1;
  seg.regs = R_;
  n_ = 1;
  neval_ = np_;
  // the root's totals: rows of half 0
  const CRows rows{nullptr, 0, tot_.p, 0, rows_stride_, nullptr, 0, CStop{}};
  rows_par_ = 0;
  return launch_rule_alone(seg, s, &rows, &rows_n_);
}

int CuhreRun::launch_rule_alone(const CSeg &seg, hipStream_t s, const CRows *rows,
                                long long *blocks) {
  return launch_rule_segments(ctx_, &seg, 1, seg_, seg_end_, w7_.p, w5_.p, s, stop_.p, rows,
                              blocks);
}

int launch_rule_segments(ccuba_ctx *ctx, const CSeg *segs, int nseg, DevBuf<CSeg> &dsegs,
                         DevBuf<long long> &dends, const double *w7_dev, const double *w5_dev,
                         hipStream_t s, int *done, const CRows *rows, long long *blocks) {
  if (nseg <= 0) return CCUBA_OK;
  int rc;
  std::vector<long long> ends(nseg);
  long long tot = 0;
  for (int q = 0; q < nseg; ++q) {
    tot += segs[q].count;
    ends[q] = tot;
  }
  const GMTables &T = gm_tables();
  RuleArgs A{};
  A.nseg = nseg;
  A.total = tot;
  if (nseg == 1) {
    A.one = segs[0];  // by value: nothing to upload, nothing to wait for
  } else {
    if ((int)dsegs.n < nseg && (rc = dsegs.alloc(ctx, nseg))) return rc;
    if ((int)dends.n < nseg && (rc = dends.alloc(ctx, nseg))) return rc;
    CCUBA_HIP(hipMemcpyAsync(dsegs.p, segs, nseg * sizeof(CSeg), hipMemcpyHostToDevice, s));
    CCUBA_HIP(hipMemcpyAsync(dends.p, ends.data(), nseg * sizeof(long long),
                             hipMemcpyHostToDevice, s));
    A.segs = dsegs.p;
    A.seg_end = dends.p;
  }
  A.w7 = w7_dev;
  A.w5 = w5_dev;
  A.done = done;
  A.l2 = T.l2;
  A.l3 = T.l3;
  A.l4 = T.l4;
  A.l5 = T.l5;
  if (rows) A.rows = *rows;
  if (blocks) *blocks = rule_blocks(A);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->profile) {
    CCUBA_HIP(hipEventCreate(&e0));
    CCUBA_HIP(hipEventCreate(&e1));
    CCUBA_HIP(hipEventRecord(e0, s));
  }
  CCUBA_HIP(launch_rule(A, s));
  if (ctx->profile) {
    CCUBA_HIP(hipEventRecord(e1, s));
    CCUBA_HIP(hipEventSynchronize(e1));
    float ms = 0;
    CCUBA_HIP(hipEventElapsedTime(&ms, e0, e1));
    ctx->stats.rule_launches += 1;
    ctx->stats.rule_ms += ms;
    long long ev = 0;
    for (int q = 0; q < nseg; ++q) ev += segs[q].count * gm_npoints(segs[q].ndim);
    ctx->stats.rule_evals += ev;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  // the host arrays of a multi-segment launch must stay alive until the
  // copies ran
  if (nseg > 1) CCUBA_HIP(hipStreamSynchronize(s));
  return CCUBA_OK;
}

int CuhreRun::launch_totals(hipStream_t s) {
  CCUBA_HIP(ccuba::launch_totals(R_, next_id_, S_, mapped_dev_ ? mapped_dev_ : out_.p, s));
  return CCUBA_OK;
}

int CuhreRun::read_totals(hipStream_t s) {
  if (mapped_host_) {  // the caller has synchronised s
    I_ = mapped_host_[0];
    E_ = mapped_host_[1];
    return CCUBA_OK;
  }
  double t[2];
  CCUBA_HIP(hipMemcpyAsync(t, out_.p, sizeof(t), hipMemcpyDeviceToHost, s));
  CCUBA_HIP(hipStreamSynchronize(s));
  I_ = t[0];
  E_ = t[1];
  return CCUBA_OK;
}

CSeg CuhreRun::children_segment(long long K, bool from_range) const {
  CSeg seg{};
  seg.ndim = spec_.ndim;
  seg.family = spec_.family;
  seg.par = params_.p;
  seg.first = next_id_;
  seg.count = 2 * K;
  seg.regs = R_;
  seg.children = 1;
  if (from_range) {  // every live region splits, and they are the last n_
    seg.pbase = next_id_ - n_;
    seg.retire = 1;
  } else {  // launch_split retired them and wrote their positions
    seg.parent = parent_.p;
  }
  return seg;
}

int CuhreRun::plan_and_split(hipStream_t s) {
  pendK_ = 0;
  if (done_) return 0;
  if (!std::isfinite(I_) || !std::isfinite(E_)) {  // a non-finite integrand value
    done_ = true;
    fail_ = -4;
    I_ = E_ = 0.0;
    return 0;
  }
  if (neval_ >= spec_.mineval && E_ <= std::max(spec_.epsabs, spec_.epsrel * std::fabs(I_))) {
    done_ = true;
    fail_ = 0;
    return 0;
  }
  long long K = std::min(spec_.batch / 2, n_);
  const long long budget = spec_.maxeval > neval_ ? (spec_.maxeval - neval_) / (2 * np_) : 0;
  K = std::min(K, budget);
  if (K <= 0) {
    done_ = true;
    fail_ = 1;
    return 0;
  }
  int rc = ensure(next_id_ + 2 * K, s);
  if (rc) return rc < 0 ? rc : CCUBA_EHIP;
  pend_range_ = K == n_ && contig_;
  if (!pend_range_) {
    CCUBA_HIP(launch_select16(R_, next_id_, K, S_, s));
    CCUBA_HIP(launch_split(R_, next_id_, K, S_, s));
    contig_ = false;
  }
  pendK_ = K;
  return 1;
}

CSeg CuhreRun::pending_segment() const { return children_segment(pendK_, pend_range_); }

void CuhreRun::commit_pending() {
  n_ += pendK_;
  next_id_ += 2 * pendK_;
  neval_ += 2 * pendK_ * np_;
  ++batches_;
  pendK_ = 0;
}

int CuhreRun::run(hipStream_t s) {
  // The host state of a step before its totals: what the host plans is
  // deterministic (K depends on n and the budget only); only the end of the
  // run is decided on the device.
  struct Plan {
    long long n, neval, next_id;
    int batches;
  };
  // the totals of the state before step t go to slot t % 2 of host-coherent
  // pinned memory: I, err and the word seq << 8 | outcome (CRows), which the
  // host polls; the caller's mapped block if given, else one of our own
  constexpr int kSlots = 2;
  double *dev_slots = mapped_dev_, *host_slots = mapped_host_;
  struct Pinned {
    void *p = nullptr;
    ~Pinned() {
      if (p) (void)hipHostFree(p);
    }
  } own;
  if (!host_slots) {
    CCUBA_HIP(hipHostMalloc(&own.p, 4 * kSlots * sizeof(double),
                            hipHostMallocMapped | hipHostMallocCoherent));
    void *d = nullptr;
    CCUBA_HIP(hipHostGetDevicePointer(&d, own.p, 0));
    host_slots = (double *)own.p;
    dev_slots = (double *)d;
  }
  auto slot = [&](int t) { return 4 * (t % kSlots); };
  auto word = [&](int t) {
    return (volatile unsigned long long *)(host_slots + slot(t) + 2);
  };
  for (int q = 0; q < kSlots; ++q) *word(q) = ~0ull;  // no state's word
  // the outcome of state t: 0 go on, 1 converged, 2 not finite.  Polled: a
  // blocking wait adds a wake-up of ~10 us to every step, longer than a
  // small step's work, and an event recorded per step costs the device ~5 us
  // (a system-scope release).  If the word does not come within a second,
  // the stream is drained and it is read once more.
  auto outcome = [&](int t) -> int {
    const unsigned long long want = (unsigned long long)t;
    auto t0 = std::chrono::steady_clock::now();
    for (unsigned spin = 0;; ++spin) {
      const unsigned long long w = *word(t);
      if ((w >> 8) == want) return (int)(w & 0xFFull);
      if ((spin & 4095u) == 4095u &&
          std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) {
        CCUBA_HIP(hipStreamSynchronize(s));
        const unsigned long long w2 = *word(t);
        return (w2 >> 8) == want ? (int)(w2 & 0xFFull) : CCUBA_EHIP;
      }
    }
  };
  // finish with state q, whose outcome (code) ended the run
  auto finish = [&](const Plan &p, int q, int code) -> int {
    CCUBA_HIP(hipStreamSynchronize(s));  // queued launches run empty; the last ones end
    n_ = p.n;
    neval_ = p.neval;
    next_id_ = p.next_id;
    batches_ = p.batches;
    done_ = true;
    pendK_ = 0;
    if (code == 2) {  // a non-finite integrand value
      fail_ = -4;
      I_ = E_ = 0.0;
    } else {
      fail_ = code == 1 ? 0 : 1;
      I_ = host_slots[slot(q)];
      E_ = host_slots[slot(q) + 1];
    }
    return CCUBA_OK;
  };
  // Outcomes are learned in step order; `known' is the last step learned
  // (all of them "go on").
  int known = -1;
  // learn state q's outcome (p: the plan of state q); true when it ended
  // the run, which is then finished
  auto learn = [&](int q, const Plan &p, int *rc) -> bool {
    const int code = outcome(q);
    if (code < 0) {
      *rc = code;
      return true;
    }
    known = q;
    if (code == 0) return false;
    *rc = finish(p, q, code);
    return true;
  };
  Plan prev{};
  for (int t = 0;; ++t) {
    const Plan cur{n_, neval_, next_id_, batches_};
    const CStop stop{spec_.epsrel, spec_.epsabs, spec_.mineval, neval_};
    // this state's rows; the step's first launch decides on them
    CRows open{tot_.p + 2 * rows_stride_ * rows_par_, rows_n_, nullptr, 0, rows_stride_,
               dev_slots + slot(t), t, stop};
    long long K = std::min(spec_.batch / 2, n_);
    const long long budget = spec_.maxeval > neval_ ? (spec_.maxeval - neval_) / (2 * np_) : 0;
    K = std::min(K, budget);
    int rc = 0;
    const bool grow = K > 0 && next_id_ + 2 * K > cap_;
    bool opened = false;
    if (K <= 0 || grow) {  // decided by a launch of its own
      CCUBA_HIP(launch_decide(open, stop_.p, s));
      opened = true;
    }
    if (grow) {
      // the store must grow (a synchronisation and a copy; the rows move
      // too): only for a step known to run, so learn steps t - 1 and t first
      if (t - 1 > known && learn(t - 1, prev, &rc)) return rc;
      if (learn(t, cur, &rc)) return rc;
      if ((rc = ensure(next_id_ + 2 * K, s))) return rc < 0 ? rc : CCUBA_EHIP;
    }
    if (K > 0) {  // queue step t's work, possibly before learning step t - 1's outcome
      const int npar = 1 - rows_par_;
      double *next = tot_.p + 2 * rows_stride_ * npar;
      long long rb = 0;
      if (K == n_ && contig_) {  // every region splits: no selection
        CRows rows{opened ? nullptr : open.in, open.nin, next, 0, rows_stride_, open.slot, t, stop};
        if ((rc = launch_rule_alone(children_segment(K, true), s, &rows, &rb))) return rc;
        rows_n_ = rb;
      } else {
        CCUBA_HIP(launch_select16(R_, next_id_, K, S_, s, opened ? nullptr : &open));
        const long long sr = split_rows(next_id_);
        const CRows keep{nullptr, 0, next, 0, rows_stride_, nullptr, 0, CStop{}};
        CCUBA_HIP(launch_split(R_, next_id_, K, S_, s, &keep));
        const CRows kids{nullptr, 0, next, sr, rows_stride_, nullptr, 0, CStop{}};
        if ((rc = launch_rule_alone(children_segment(K, false), s, &kids, &rb))) return rc;
        rows_n_ = sr + rb;
        contig_ = false;
      }
      rows_par_ = npar;
      pendK_ = K;
      commit_pending();
    }
    if (t - 1 > known && learn(t - 1, prev, &rc)) return rc;
    if (K <= 0) {  // out of budget after step t, unless its totals ended it first
      if (t > known && learn(t, cur, &rc)) return rc;
      return finish(cur, t, 0);  // fail 1
    }
    prev = cur;
  }
}

int CuhreRun::rule_only(long long nreg, const double *c, const double *h, double *I7, double *I5,
                        double *err, int *axis, hipStream_t s) {
  const int d = spec_.ndim;
  int rc = ensure(nreg, s);
  if (rc) return rc;
  const CRegions &R = R_;
  for (int j = 0; j < d; ++j) {
    CCUBA_HIP(hipMemcpyAsync(R.c + j * R.cap, c + (size_t)j * nreg, nreg * 8,
                             hipMemcpyHostToDevice, s));
    CCUBA_HIP(hipMemcpyAsync(R.h + j * R.cap, h + (size_t)j * nreg, nreg * 8,
                             hipMemcpyHostToDevice, s));
  }
  CSeg seg{};
  seg.ndim = d;
  seg.family = spec_.family;
  seg.par = params_.p;
  seg.first = 0;
  seg.count = nreg;
  seg.regs = R;
  if ((rc = launch_rule_alone(seg, s))) return rc;
  if (I7) CCUBA_HIP(hipMemcpyAsync(I7, R.I7, nreg * 8, hipMemcpyDeviceToHost, s));
  if (I5) CCUBA_HIP(hipMemcpyAsync(I5, R.I5, nreg * 8, hipMemcpyDeviceToHost, s));
  if (err) CCUBA_HIP(hipMemcpyAsync(err, R.err, nreg * 8, hipMemcpyDeviceToHost, s));
  if (axis) CCUBA_HIP(hipMemcpyAsync(axis, R.axis, nreg * 4, hipMemcpyDeviceToHost, s));
  CCUBA_HIP(hipStreamSynchronize(s));
  return CCUBA_OK;
}

}  // namespace ccuba
