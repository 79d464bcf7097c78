// suave.cpp -- oracle: plain serial Suave (TEST INFRASTRUCTURE ONLY).
//
// The paper gives Suave's prototype (Sect. 3.2.2: ..., mineval, maxeval,
// nnew, flatness, statefile, spin, nregions, neval, fail, ...) and names it
// among the four Cuba integrators, but not its steps.  The reading taken here
// is subregion-adaptive Vegas: Vegas sampling in every region, each region
// with its own grid, and bisection of the regions with the largest variance.
// Its steps, in order:
//  1. The root region [0,1]^d with the uniform grid is sampled with nnew
//     points (sampling serial 0).
//  2. Sampling region r (bounds lo, hi; volume V; grid E; serial q): the
//     Vegas point map of the Vegas oracle with iteration number q gives the
//     relative point x' and grid weight w' = prod_j N dE_j; the point is
//     x_j = fma(x'_j, hi_j - lo_j, lo_j), its value v = (w' V) f(x).  From
//     the n = nnew values: I = S1/n, sigma^2 = max(0, S2/n - I^2)/(n-1), and
//     the histogram H_j[k_j] += v^2 refines the region's grid with the Vegas
//     rule (unless the grid is frozen).  Point i records the side bits
//     b_ij = [x'_ij >= 1/2] (upper half of dimension j).
//  3. A region's result combines its estimates -- the one inherited from its
//     parent (if any) and its own sample -- with inverse-variance weights
//     (if some variance is 0: the mean of those estimates, variance 0);
//     chi^2_r = sum (I_k - I_r)^2/sigma_k^2, dof_r = #estimates - 1.
//  4. Totals: I = sum_r I_r, sigma^2 = sum_r sigma_r^2, chi^2 and dof
//     summed, prob = P(dof/2, chi^2/2) (0 when dof = 0).  Stop with fail 0
//     when neval >= mineval and sigma <= max(epsabs, epsrel |I|).
//  5. A step splits K' = min(K, #regions, (maxeval - neval) div 2 nnew)
//     regions; K' = 0 stops with fail 1.  The selected regions are those of
//     largest sigma_r^2, ties to the lower position.
//  6. Split dimension: for each j and half h, with the n_h samples of the
//     region on that side (mean m_h),
//       F_h = (n_h/n) ((1/n_h) sum |v_i - m_h|^p)^(1/p),   p = flatness,
//     (0 for an empty half); the cut is along the j of least F_0 + F_1,
//     ties to the lower j, at the midpoint of the region.
//  7. Child h of a region cut along c: bounds halved along c; grid equal to
//     the parent's in every other dimension and, along c, the parent's map
//     X (piecewise linear through (k/N, E_k)) restricted to the half:
//       lower: E'_k = 2 X(y* k/N),   upper: E'_k = 2 X(y* + (1-y*) k/N) - 1,
//     with X(y*) = 1/2, E'_0 = 0, E'_N = 1, made non-decreasing; inherited
//     estimate from the parent's samples on side h: I = S1_h/n,
//     sigma^2 = max(0, S2_h/n - I^2)/(n-1), n the parent's sample count
//     (the restriction estimator), kept only when sigma^2 > 0.
//  8. Positions: the lower child takes its parent's position, the upper one
//     goes after the existing regions, in the order of selection.  The j-th
//     split of the run (counted from 0 over all steps) samples its children
//     with serials 2j+1 (lower) and 2j+2 (upper).  All splits of a step are
//     decided before any child is sampled.
// A non-finite total (a non-finite integrand value) ends the run with fail -4
// and zero results.  All sums are Neumaier-compensated FP64 in point (or
// position) order.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "oracle.h"

namespace {

struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double v) {
    const double t = s + v;
    if (std::fabs(s) >= std::fabs(v))
      c += (s - t) + v;
    else
      c += (v - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

struct Estimate {
  double I, var;
};

struct Region {
  std::vector<double> lo, hi, grid;  // grid: ndim rows of N + 1 edges
  bool has_inh = false;
  Estimate inh{0.0, 0.0};
  double I = 0.0, var = 0.0, chi2 = 0.0;
  int dof = 0;
  std::vector<double> v;        // the values of the region's own sample
  std::vector<uint32_t> side;   // side bits of each point
};

// step 3
void combine(Region &r, const Estimate &own) {
  std::vector<Estimate> e;
  if (r.has_inh) e.push_back(r.inh);
  e.push_back(own);
  r.dof = (int)e.size() - 1;
  r.chi2 = 0.0;
  int nzero = 0;
  double zsum = 0.0;
  for (const Estimate &k : e)
    if (k.var == 0.0) {
      ++nzero;
      zsum += k.I;
    }
  if (nzero > 0) {
    r.I = zsum / nzero;
    r.var = 0.0;
    return;
  }
  double wsum = 0.0, wisum = 0.0;
  for (const Estimate &k : e) {
    wsum += 1.0 / k.var;
    wisum += k.I / k.var;
  }
  r.I = wisum / wsum;
  r.var = 1.0 / wsum;
  for (const Estimate &k : e) r.chi2 += (k.I - r.I) * (k.I - r.I) / k.var;
}

// step 7: the parent's map along one dimension restricted to half h
void inherit_dim(int N, const double *E, int h, double *out) {
  auto X = [&](double y) {
    const double z = y * N;
    int k = (int)std::floor(z);
    if (k > N - 1) k = N - 1;
    if (k < 0) k = 0;
    return std::fma(z - k, E[k + 1] - E[k], E[k]);
  };
  int ks = 0;  // the last edge at or below 1/2 (E_0 = 0, E_N = 1)
  while (ks < N - 1 && E[ks + 1] <= 0.5) ++ks;
  const double ystar = (ks + (0.5 - E[ks]) / (E[ks + 1] - E[ks])) / N;
  for (int k = 0; k <= N; ++k) {
    const double t = (double)k / N;
    out[k] = h == 0 ? 2.0 * X(ystar * t) : 2.0 * X(std::fma(1.0 - ystar, t, ystar)) - 1.0;
  }
  out[0] = 0.0;
  out[N] = 1.0;
  for (int k = 1; k <= N; ++k) out[k] = std::max(out[k], out[k - 1]);
}

struct Run {
  int ndim, N, nvec, flags;
  unsigned long long seed;
  unsigned int sid;
  long long nnew;
  oracle_integrand_t f;
  void *ud;

  // step 2; returns -999 when the integrand aborts
  int sample(Region &r, int serial) {
    const int d = ndim;
    double V = 1.0;
    for (int j = 0; j < d; ++j) V *= r.hi[j] - r.lo[j];
    r.v.assign(nnew, 0.0);
    r.side.assign(nnew, 0u);
    Neumaier s1, s2;
    std::vector<Neumaier> H((size_t)d * N);
    std::vector<double> xr((size_t)nvec * d), x((size_t)nvec * d), w(nvec), fv(nvec);
    std::vector<int> k((size_t)nvec * d);
    const int core = 32768;
    for (long long i0 = 0; i0 < nnew; i0 += nvec) {
      const int cnt = (int)std::min<long long>(nvec, nnew - i0);
      oracle_vegas_points(d, N, ORACLE_FP64, seed, sid, serial, r.grid.data(), i0, cnt, nullptr,
                          xr.data(), w.data(), k.data());
      for (int p = 0; p < cnt; ++p)
        for (int j = 0; j < d; ++j)
          x[(size_t)p * d + j] =
              std::fma(xr[(size_t)p * d + j], r.hi[j] - r.lo[j], r.lo[j]);
      const int one = 1;
      if (f(&ndim, x.data(), &one, fv.data(), ud, &cnt, &core) == -999) return -999;
      for (int p = 0; p < cnt; ++p) {
        const double v = (w[p] * V) * fv[p];
        uint32_t bits = 0;
        for (int j = 0; j < d; ++j)
          if (xr[(size_t)p * d + j] >= 0.5) bits |= 1u << j;
        r.v[i0 + p] = v;
        r.side[i0 + p] = bits;
        s1.add(v);
        s2.add(v * v);
        for (int j = 0; j < d; ++j) H[(size_t)j * N + k[(size_t)p * d + j]].add(v * v);
      }
    }
    const double n = (double)nnew;
    Estimate own;
    own.I = s1.value() / n;
    own.var = std::max(0.0, s2.value() / n - own.I * own.I) / (n - 1.0);
    combine(r, own);
    if (!(flags & ORACLE_FREEZE_GRID)) {
      std::vector<double> h(N), enew(N + 1);
      for (int j = 0; j < d; ++j) {
        for (int b = 0; b < N; ++b) h[b] = H[(size_t)j * N + b].value();
        double *E = r.grid.data() + (size_t)j * (N + 1);
        oracle_vegas_refine_dim(N, h.data(), E, enew.data());
        std::copy(enew.begin(), enew.end(), E);
      }
    }
    return 0;
  }
};

// step 6: F_0 + F_1 for a cut along dimension j
double split_score(const Region &r, int j, double p) {
  const double n = (double)r.v.size();
  double score = 0.0;
  for (uint32_t h = 0; h < 2; ++h) {
    Neumaier s;
    long long nh = 0;
    for (size_t i = 0; i < r.v.size(); ++i)
      if (((r.side[i] >> j) & 1u) == h) {
        s.add(r.v[i]);
        ++nh;
      }
    if (nh == 0) continue;
    const double m = s.value() / nh;
    double M = 0.0;  // the largest deviation scales the p-th powers
    for (size_t i = 0; i < r.v.size(); ++i)
      if (((r.side[i] >> j) & 1u) == h) M = std::max(M, std::fabs(r.v[i] - m));
    if (M == 0.0) continue;
    Neumaier q;
    for (size_t i = 0; i < r.v.size(); ++i)
      if (((r.side[i] >> j) & 1u) == h) q.add(std::pow(std::fabs(r.v[i] - m) / M, p));
    score += (nh / n) * M * std::pow(q.value() / nh, 1.0 / p);
  }
  return score;
}

// step 7: the two children of r cut along c
void split(const Region &r, int c, int N, Region &lower, Region &upper) {
  const int d = (int)r.lo.size();
  const double n = (double)r.v.size();
  Region *ch[2] = {&lower, &upper};
  for (int h = 0; h < 2; ++h) {
    Region &q = *ch[h];
    q = Region();
    q.lo = r.lo;
    q.hi = r.hi;
    const double mid = 0.5 * (r.lo[c] + r.hi[c]);
    (h == 0 ? q.hi[c] : q.lo[c]) = mid;
    q.grid = r.grid;
    inherit_dim(N, r.grid.data() + (size_t)c * (N + 1), h, q.grid.data() + (size_t)c * (N + 1));
    Neumaier s1, s2;
    for (size_t i = 0; i < r.v.size(); ++i)
      if (((r.side[i] >> c) & 1u) == (uint32_t)h) {
        s1.add(r.v[i]);
        s2.add(r.v[i] * r.v[i]);
      }
    q.inh.I = s1.value() / n;
    q.inh.var = std::max(0.0, s2.value() / n - q.inh.I * q.inh.I) / (n - 1.0);
    q.has_inh = q.inh.var > 0.0;
  }
  (void)d;
}

}  // namespace

extern "C" int oracle_suave(int ndim, int ncomp, oracle_integrand_t integrand, void *userdata,
                            int nvec, double epsrel, double epsabs, int flags,
                            unsigned long long seed, long long mineval, long long maxeval,
                            long long nnew, double flatness, int nbins, int nsplit,
                            unsigned int stream_id, int *nregions, long long *neval, int *fail,
                            double integral[], double error[], double prob[],
                            oracle_suave_trace *trace) {
  if (ndim < 1 || ndim > 16 || ncomp != 1 || nvec < 1 || nbins < 2 || nbins > 256 || nnew < 2 ||
      nnew >= (1ll << 32) || !(flatness > 0.0) || !std::isfinite(flatness) || nsplit < 1 ||
      (flags & ORACLE_PRECISION_MASK) != ORACLE_FP64 || !integrand || !nregions || !neval ||
      !fail || !integral || !error || !prob)
    return -1;
  const int d = ndim, N = nbins;
  Run run{ndim, N, nvec, flags, seed, stream_id, nnew, integrand, userdata};
  std::vector<Region> R;
  long long nev = 0;
  long long nsplits = 0;
  int status = 1;
  double I = 0.0, var = 0.0, chi2 = 0.0;
  int dof = 0;
  bool aborted = false;
  std::vector<int> cuts;

  auto totals = [&]() {  // step 4
    Neumaier si, sv, sc;
    dof = 0;
    for (const Region &r : R) {
      si.add(r.I);
      sv.add(r.var);
      sc.add(r.chi2);
      dof += r.dof;
    }
    I = si.value();
    var = sv.value();
    chi2 = sc.value();
  };

  if (nnew <= maxeval) {  // step 1
    Region root;
    root.lo.assign(d, 0.0);
    root.hi.assign(d, 1.0);
    root.grid.resize((size_t)d * (N + 1));
    for (int j = 0; j < d; ++j)
      for (int k = 0; k <= N; ++k) root.grid[(size_t)j * (N + 1) + k] = (double)k / N;
    if (run.sample(root, 0) == -999) {
      aborted = true;
    } else {
      nev = nnew;
      R.push_back(std::move(root));
      totals();
    }
  }
  bool nonfinite = false;
  while (!aborted && !R.empty()) {
    if (!std::isfinite(I) || !std::isfinite(var)) {
      nonfinite = true;
      break;
    }
    if (nev >= mineval && std::sqrt(var) <= std::max(epsabs, epsrel * std::fabs(I))) {
      status = 0;
      break;
    }
    long long K = std::min<long long>(nsplit, (long long)R.size());
    K = std::min<long long>(K, (maxeval - nev) / (2 * nnew));
    if (K > 0 && 2 * (nsplits + K) >= (1ll << 24)) K = 0;  // serials run out
    if (K <= 0) break;
    // step 5: the K regions of largest variance, ties to the lower position
    std::vector<int> order(R.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return R[a].var > R[b].var; });
    // steps 6-7 for every selected region, before any sampling
    std::vector<Region> lower(K), upper(K);
    for (long long j = 0; j < K; ++j) {
      const Region &r = R[order[j]];
      int best = 0;
      double bscore = split_score(r, 0, flatness);
      for (int c = 1; c < d; ++c) {
        const double s = split_score(r, c, flatness);
        if (s < bscore) {
          bscore = s;
          best = c;
        }
      }
      cuts.push_back(best);
      split(r, best, N, lower[j], upper[j]);
    }
    // step 8
    const size_t base = R.size();
    for (long long j = 0; j < K; ++j) R[order[j]] = std::move(lower[j]);
    for (long long j = 0; j < K; ++j) R.push_back(std::move(upper[j]));
    for (long long j = 0; j < K && !aborted; ++j) {
      const int q = (int)(nsplits + j);
      aborted = run.sample(R[order[j]], 2 * q + 1) == -999 ||
                run.sample(R[base + j], 2 * q + 2) == -999;
    }
    if (aborted) break;
    nsplits += K;
    nev += 2 * K * nnew;
    totals();
  }
  if (aborted) {
    *nregions = (int)R.size();
    *neval = nev;
    *fail = -99;
    integral[0] = error[0] = prob[0] = 0.0;
    return 0;
  }
  if (nonfinite) {
    *nregions = (int)R.size();
    *neval = nev;
    *fail = -4;
    integral[0] = error[0] = prob[0] = 0.0;
    return 0;
  }
  *nregions = (int)R.size();
  *neval = nev;
  *fail = status;
  integral[0] = I;
  error[0] = std::sqrt(var);
  prob[0] = dof > 0 ? oracle_gammainc_lower(0.5 * dof, 0.5 * chi2) : 0.0;
  if (trace) {
    trace->nregions = (int)R.size();
    trace->nsplits = (int)cuts.size();
    trace->chi2 = chi2;
    trace->dof = dof;
    for (int r = 0; r < (int)R.size() && r < trace->max_regions; ++r) {
      const Region &g = R[r];
      for (int j = 0; j < d; ++j) {
        if (trace->lo) trace->lo[(size_t)r * d + j] = g.lo[j];
        if (trace->hi) trace->hi[(size_t)r * d + j] = g.hi[j];
      }
      if (trace->I) trace->I[r] = g.I;
      if (trace->var) trace->var[r] = g.var;
      if (trace->inh_I) trace->inh_I[r] = g.has_inh ? g.inh.I : 0.0;
      if (trace->inh_var) trace->inh_var[r] = g.has_inh ? g.inh.var : 0.0;
      if (trace->grid)
        std::copy(g.grid.begin(), g.grid.end(), trace->grid + (size_t)r * d * (N + 1));
    }
    for (int s = 0; s < (int)cuts.size() && s < trace->max_splits; ++s)
      if (trace->cut) trace->cut[s] = cuts[s];
  }
  return 0;
}
