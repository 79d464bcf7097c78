// divonne.cpp -- oracle: Divonne's partitioning phase (TEST INFRASTRUCTURE ONLY).
//
// Sect. 2.2 describes the phase: the integration region is split into
// subregions of about equal spread, Spread(r) = 1/2 Vol(r) (sup_r f - inf_r f),
// with the extrema sought by numerical optimisation, one point at a time;
// the parallel version hands every worker an entire region to search and
// subdivide, with the recursion replaced by bookkeeping of the regions.  The
// paper does not give the search or the cut, so these steps are a reading:
//  1. Search of region r (bounds lo, hi, widths w = hi - lo; search serial
//     q): nsearch points x_j = fma(y_j, w_j, lo_j), y from the Philox words
//     of counter (i, (q<<8)|b, sid, 0) (word j%4 of block j/4, FP64 uniform
//     y = r 2^-32 + 2^-33); the largest and the smallest value, ties to the
//     lower i (a NaN is never taken), start two compass searches.
//  2. Compass search (for the maximum; the minimum mirrors it): steps
//     h_j = w_j/4; each of niter iterations evaluates the 2d candidates
//     x +- h_j e_j (candidate 2j is +, 2j+1 is -; each clipped to
//     [lo_j, hi_j]); the best one (largest value, ties to the lower
//     candidate) is taken if it beats the current value, else every step is
//     halved.  A search costs nsearch + 4 d niter evaluations.
//  3. Spread(r) = 1/2 V (fmax - fmin) with V = prod w_j.
//  4. Steps: while the largest spread exceeds spread_tol and fewer than
//     maxregions regions exist, the K = min(nsplit, #regions,
//     maxregions - #regions) regions of largest spread (ties to the lower
//     position) are bisected at the midpoint of the dimension whose move
//     from the maximum's point to the minimum's loses most value:
//     j* = argmax_j fmax - f(xmax with x_j := xmin_j), ties to the lower j
//     (d evaluations per split).  The lower
//     child takes its parent's position, the upper one goes after the existing
//     regions in order of selection; the j-th split of the run searches its
//     children with serials 2j+1 and 2j+2 (the root: 0).  fail is 0 when the
//     spreads end below spread_tol, 1 when the region budget ends the phase.
// A non-finite spread (a non-finite integrand value) ends the phase with
// fail -4.  The spreads' total is a Neumaier sum in position order.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "oracle.h"

namespace {

struct Region {
  std::vector<double> lo, hi, xmin, xmax;
  double fmin = 0.0, fmax = 0.0, spread = 0.0;
};

struct Search {
  int d, nvec;
  unsigned long long seed;
  unsigned int sid;
  int nsearch, niter;
  oracle_integrand_t f;
  void *ud;
  long long neval = 0;

  // values of the n points xs[n][d]
  void eval(const std::vector<double> &xs, int n, std::vector<double> &fv) {
    fv.resize(n);
    const int one = 1, core = 32768;
    for (int p0 = 0; p0 < n; p0 += nvec) {
      const int cnt = std::min(nvec, n - p0);
      f(&d, xs.data() + (size_t)p0 * d, &one, fv.data() + p0, ud, &cnt, &core);
    }
    neval += n;
  }

  // step 2: sign +1 climbs to the maximum, -1 descends to the minimum
  double compass(const Region &r, std::vector<double> &x, double fx, int sign) {
    std::vector<double> h(d), cand((size_t)2 * d * d), fc;
    for (int j = 0; j < d; ++j) h[j] = (r.hi[j] - r.lo[j]) / 4.0;
    for (int t = 0; t < niter; ++t) {
      for (int c = 0; c < 2 * d; ++c) {
        const int j = c / 2;
        for (int k = 0; k < d; ++k) cand[(size_t)c * d + k] = x[k];
        const double z = c % 2 == 0 ? x[j] + h[j] : x[j] - h[j];
        cand[(size_t)c * d + j] = std::min(std::max(z, r.lo[j]), r.hi[j]);
      }
      eval(cand, 2 * d, fc);
      int best = 0;
      for (int c = 1; c < 2 * d; ++c)
        if (sign * fc[c] > sign * fc[best]) best = c;
      if (sign * fc[best] > sign * fx) {
        fx = fc[best];
        for (int k = 0; k < d; ++k) x[k] = cand[(size_t)best * d + k];
      } else {
        for (int j = 0; j < d; ++j) h[j] *= 0.5;
      }
    }
    return fx;
  }

  // steps 1-3
  void search(Region &r, int q) {
    std::vector<double> xs((size_t)nsearch * d), fv;
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffull), (uint32_t)(seed >> 32)};
    for (int i = 0; i < nsearch; ++i) {
      uint32_t words[16];
      for (int b = 0; b < (d + 3) / 4; ++b) {
        const uint32_t ctr[4] = {(uint32_t)i, ((uint32_t)q << 8) | (uint32_t)b, sid, 0u};
        oracle_philox4x32_10(ctr, key, words + 4 * b);
      }
      for (int j = 0; j < d; ++j) {
        const double y = (double)words[j] * 0x1p-32 + 0x1p-33;
        xs[(size_t)i * d + j] = std::fma(y, r.hi[j] - r.lo[j], r.lo[j]);
      }
    }
    eval(xs, nsearch, fv);
    // a NaN value is never an extremum (it compares false with everything);
    // with no other value the searches start from -inf and +inf
    int imax = -1, imin = -1;
    for (int i = 0; i < nsearch; ++i) {
      if (std::isnan(fv[i])) continue;
      if (imax < 0 || fv[i] > fv[imax]) imax = i;
      if (imin < 0 || fv[i] < fv[imin]) imin = i;
    }
    const double f0max = imax < 0 ? -INFINITY : fv[imax], f0min = imin < 0 ? INFINITY : fv[imin];
    imax = std::max(imax, 0);
    imin = std::max(imin, 0);
    r.xmax.assign(xs.begin() + (size_t)imax * d, xs.begin() + (size_t)(imax + 1) * d);
    r.xmin.assign(xs.begin() + (size_t)imin * d, xs.begin() + (size_t)(imin + 1) * d);
    r.fmax = compass(r, r.xmax, f0max, +1);
    r.fmin = compass(r, r.xmin, f0min, -1);
    double V = 1.0;
    for (int j = 0; j < d; ++j) V *= r.hi[j] - r.lo[j];
    r.spread = 0.5 * V * (r.fmax - r.fmin);
  }
};

}  // namespace

extern "C" int oracle_divonne_partition(int ndim, oracle_integrand_t integrand, void *userdata,
                                        int nvec, unsigned long long seed,
                                        unsigned int stream_id, int nsearch, int niter,
                                        int maxregions, int nsplit, double spread_tol,
                                        int *nregions, long long *neval, int *fail,
                                        double *total_spread, oracle_partition_trace *trace) {
  if (ndim < 1 || ndim > 16 || !integrand || nvec < 1 || nsearch < 1 || nsearch > (1 << 30) ||
      niter < 0 ||
      niter > 4096 || maxregions < 1 || maxregions > (1 << 23) || nsplit < 1 ||
      !(spread_tol >= 0.0) || !nregions || !neval || !fail || !total_spread)
    return -1;
  const int d = ndim;
  Search S{d, nvec, seed, stream_id, nsearch, niter, integrand, userdata};
  std::vector<Region> R(1);
  R[0].lo.assign(d, 0.0);
  R[0].hi.assign(d, 1.0);
  S.search(R[0], 0);
  std::vector<int> cuts;
  long long nsplits = 0;
  int status;
  for (;;) {
    double top = 0.0;
    bool finite = true;
    for (const Region &r : R) {
      top = std::max(top, r.spread);
      finite = finite && std::isfinite(r.spread);
    }
    if (!finite) {
      status = -4;
      break;
    }
    if (top <= spread_tol) {
      status = 0;
      break;
    }
    const long long K = std::min<long long>(
        {(long long)nsplit, (long long)R.size(), (long long)maxregions - (long long)R.size()});
    if (K <= 0) {
      status = 1;
      break;
    }
    std::vector<int> order(R.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return R[a].spread > R[b].spread; });
    std::vector<Region> lower(K), upper(K);
    std::vector<double> probe((size_t)d * d), fp;
    for (long long s = 0; s < K; ++s) {
      const Region &p = R[order[s]];
      for (int j = 0; j < d; ++j)
        for (int k = 0; k < d; ++k) probe[(size_t)j * d + k] = k == j ? p.xmin[k] : p.xmax[k];
      S.eval(probe, d, fp);
      int c = 0;
      for (int j = 1; j < d; ++j)
        if (p.fmax - fp[j] > p.fmax - fp[c]) c = j;
      cuts.push_back(c);
      const double mid = 0.5 * (p.lo[c] + p.hi[c]);
      lower[s].lo = upper[s].lo = p.lo;
      lower[s].hi = upper[s].hi = p.hi;
      lower[s].hi[c] = mid;
      upper[s].lo[c] = mid;
    }
    const size_t base = R.size();
    for (long long s = 0; s < K; ++s) R[order[s]] = lower[s];
    for (long long s = 0; s < K; ++s) R.push_back(upper[s]);
    for (long long s = 0; s < K; ++s) {
      const int q = (int)(nsplits + s);
      S.search(R[order[s]], 2 * q + 1);
      S.search(R[base + s], 2 * q + 2);
    }
    nsplits += K;
  }
  double tot = 0.0, comp = 0.0;  // Neumaier
  for (const Region &r : R) {
    const double t = tot + r.spread;
    comp += std::fabs(tot) >= std::fabs(r.spread) ? (tot - t) + r.spread : (r.spread - t) + tot;
    tot = t;
  }
  *nregions = (int)R.size();
  *neval = S.neval;
  *fail = status;
  *total_spread = status == -4 ? 0.0 : tot + comp;
  if (trace) {
    trace->nregions = (int)R.size();
    trace->nsplits = (int)cuts.size();
    for (int i = 0; i < (int)R.size() && i < trace->max_regions; ++i) {
      const Region &r = R[i];
      for (int j = 0; j < d; ++j) {
        if (trace->lo) trace->lo[(size_t)i * d + j] = r.lo[j];
        if (trace->hi) trace->hi[(size_t)i * d + j] = r.hi[j];
        if (trace->xmin) trace->xmin[(size_t)i * d + j] = r.xmin[j];
        if (trace->xmax) trace->xmax[(size_t)i * d + j] = r.xmax[j];
      }
      if (trace->fmin) trace->fmin[i] = r.fmin;
      if (trace->fmax) trace->fmax[i] = r.fmax;
      if (trace->spread) trace->spread[i] = r.spread;
    }
    for (int s = 0; s < (int)cuts.size() && s < trace->max_splits; ++s)
      if (trace->cut) trace->cut[s] = cuts[s];
  }
  return 0;
}
