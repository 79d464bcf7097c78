// refine.h -- device pieces shared by the Vegas and Suave finishing kernels:
// wave-wide scans, the regularized incomplete gamma function of the chi^2
// probability, and Lepage's refinement of one grid dimension.
#pragma once
#include <hip/hip_runtime.h>

#include "vegas_sample.h"  // wave_sum

namespace ccuba {

__device__ __forceinline__ double wave_scan_incl(double v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lower regularized incomplete gamma P(a, x) for the chi^2 probability, by
// its power series below a+1 and Legendre's continued fraction for Q = 1-P
// above (Abramowitz & Stegun 6.5.29, 6.5.31; Lentz's evaluation).
__device__ inline double gamma_p(double a, double x) {
  if (x <= 0.0) return 0.0;
  if (isinf(x)) return 1.0;
  const double lead = exp(-x + a * log(x) - lgamma(a));
  if (x < a + 1.0) {
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 100000; ++n) {
      term *= x / (a + n);
      sum += term;
      if (fabs(term) < fabs(sum) * 1e-17) break;
    }
    return sum * lead;
  }
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, dd = 1.0 / b, h = dd;
  for (int i = 1; i < 100000; ++i) {
    const double an = -i * (i - a);
    b += 2.0;
    dd = an * dd + b;
    if (fabs(dd) < tiny) dd = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    dd = 1.0 / dd;
    const double delta = dd * c;
    h *= delta;
    if (fabs(delta - 1.0) < 1e-17) break;
  }
  return 1.0 - lead * h;
}

// a7, the grid: one dimension's refinement by one wavefront.  The histogram
// row h is smoothed, damped and prefix-summed (lanes own contiguous runs of
// bins, wave-wide scans), and every new edge is placed in the old bin whose
// prefix-sum interval holds its share, by the lane that owns that bin (the
// bin a binary search of the prefix sums would find).  h, dd and Eo are LDS
// rows (h is overwritten with the prefix sums); En receives the N + 1 new
// edges.
__device__ __forceinline__ void rebin_dimension(double *h, double *dd, const double *Eo,
                                                double *En, int N, int lane) {
  const int per = (N + 63) >> 6;  // contiguous bins per lane
  const int k0 = lane * per, k1 = min(k0 + per, N);
  // smoothing and the two row sums
  double hs = 0.0, ds = 0.0;
  for (int k = k0; k < k1; ++k) {
    double v;
    if (k == 0)
      v = (h[0] + h[1]) / 2.0;
    else if (k == N - 1)
      v = (h[N - 2] + h[N - 1]) / 2.0;
    else
      v = (h[k - 1] + h[k] + h[k + 1]) / 3.0;
    hs += h[k];
    ds += v;
    dd[k] = v;
  }
  hs = wave_sum(hs);
  ds = wave_sum(ds);
  if (!(hs > 0.0)) {  // nothing sampled in this dimension: the edges are kept
    for (int i = lane; i <= N; i += 64) En[i] = Eo[i];
    return;
  }
  // damping, then prefix sums of m into h (the histogram is no longer needed)
  wave_sync_lds();
  double run = 0.0;
  for (int k = k0; k < k1; ++k) {
    const double r = dd[k] / ds;
    double m;
    if (r == 0.0)
      m = 0.0;
    else if (r == 1.0)
      m = 1.0;
    else {
      const double q = (r - 1.0) / log(r);
      m = q * sqrt(q);  // q^1.5
    }
    dd[k] = m;
    run += m;
  }
  const double incl = wave_scan_incl(run, lane);
  double acc = incl - run;
  for (int k = k0; k < k1; ++k) {
    acc += dd[k];
    h[k] = acc;
  }
  wave_sync_lds();
  const double share = h[N - 1] / N;
  // new edge i (0 < i < N) lies in the smallest old bin k with C_k >= i *
  // share (the last bin if there is none): each lane places the edges of its
  // own bins, those with C_{k-1} < i * share <= C_k, a contiguous run of i
  if (lane == 0) {
    En[0] = 0.0;
    En[N] = 1.0;
  }
  for (int k = k0; k < k1; ++k) {
    const bool last = k == N - 1;
    const double below = k > 0 ? h[k - 1] : 0.0;  // C_{k-1}; targets are > 0
    const double above = h[k];
    if (!last && !(above > below)) continue;  // an empty bin holds no edge
    // the first i with i * share > C_{k-1}: an estimate, then corrected
    int i = k > 0 ? (int)fmin(below / share, (double)N) : 1;
    if (i < 1) i = 1;
    while (i > 1 && (double)(i - 1) * share > below) --i;
    while (i < N && !((double)i * share > below)) ++i;
    for (; i < N; ++i) {
      const double target = i * share;
      if (!last && !(target <= above)) break;
      En[i] = Eo[k] + (target - below) / dd[k] * (Eo[k + 1] - Eo[k]);
    }
  }
}

}  // namespace ccuba
