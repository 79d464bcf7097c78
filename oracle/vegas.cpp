// vegas.cpp -- oracle: plain serial Vegas (TEST INFRASTRUCTURE ONLY).
//
// The paper fixes the interface (Sect. 3.2.2, Vegas prototype: ndim, ncomp,
// integrand, userdata, nvec, epsrel, epsabs, flags, seed, mineval, maxeval,
// nstart, nincrease, nbatch, ..., neval, fail, integral, error, prob) and says
// that every sample comes from one generator so that no random number is used
// twice (Sect. 2).  The algorithm is Lepage's (J. Comput. Phys. 27 (1978)
// 192), taken step by step; readings where the paper is silent:
//  * points: Philox4x32-10 words W_b = philox(ctr = (i, (t<<8)|b, sid, 0),
//    key = (seed mod 2^32, seed div 2^32)) for point i of iteration t and
//    dimension block b = j/4; coordinate j uses word j%4 of block j/4;
//  * uniform: FP64 y = r 2^-32 + 2^-33; FP32 y = (r>>9) 2^-23 + 2^-24, so y is
//    exact in its precision and never 0 or 1;
//  * map: z = y N, k = min(floor z, N-1), x = E[k] + (z-k)(E[k+1]-E[k]) (one
//    fused multiply-add), weight w = prod_j N (E_j[k+1]-E_j[k]);
//  * estimator: v = w f, I_t = the mean of v, sigma_t^2 = max(0, mean of v^2
//    - I_t^2)/(n-1); histogram H_j[k_j] += v^2.  The sums are taken about
//    c = I_{t-1} (0 for t = 0): S1 = sum (v - c), S2 = sum (v - c)^2,
//    I_t = c + S1/n, sigma_t^2 = max(0, S2/n - (S1/n)^2)/(n-1), which is the
//    same quantity, evaluated without the cancellation between the mean of
//    v^2 and I_t^2 that costs log10(mean v^2 / variance) digits;
//  * refinement (each dimension with sum H > 0): 3-point smoothing, damping
//    m_k = ((r_k-1)/ln r_k)^1.5 with r_k the normalised smoothed histogram,
//    then new edges that give every new bin the same share of sum m, with m_k
//    spread uniformly over old bin k;
//  * combination over all iterations: inverse-variance weighted mean, its
//    error (sum 1/sigma_t^2)^-1/2, chi^2 = sum (I_t - I)^2 / sigma_t^2 with
//    dof = T-1, prob = P(dof/2, chi^2/2); if some sigma_t = 0 the result is
//    the mean of those I_t with error 0, chi^2 0, prob 0;
//  * stop after an iteration when neval >= mineval and
//    error <= max(epsabs, epsrel |I|) (fail 0); before an iteration of n_t =
//    nstart + t nincrease points that would take neval past maxeval, stop
//    with fail 1;
//  * nbatch only partitions the sampling internally (Sect. 3.2.7) and has no
//    effect on any result, so it is only validated here;
//  * an iteration whose sums are not finite (a non-finite integrand value)
//    ends the run with fail -4 and zero results; neval counts it;
//  * several components (ncomp > 1): every component has its own sums,
//    iteration results, combination, chi^2 and probability over the same
//    points; the one grid adapts to the histogram of component 0; the
//    accuracy test needs every component within its tolerance.
// All sums are Neumaier-compensated FP64 in point order.
#include <cmath>
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

// Map one point (steps a1-a3).  Returns w; fills x[ndim] and k[ndim].
double map_point(int ndim, int nbins, int precision, unsigned long long seed,
                 unsigned int sid, int t, const double *grid, long long i,
                 uint32_t *words_out, double *x, int *k) {
  const int nblk = (ndim + 3) / 4;
  uint32_t words[16];
  const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffull),
                           (uint32_t)(seed >> 32)};
  for (int b = 0; b < nblk; ++b) {
    const uint32_t ctr[4] = {(uint32_t)i, ((uint32_t)t << 8) | (uint32_t)b,
                             sid, 0u};
    oracle_philox4x32_10(ctr, key, words + 4 * b);
  }
  if (words_out)
    for (int q = 0; q < 4 * nblk; ++q) words_out[q] = words[q];

  if (precision == ORACLE_FP32_EVAL) {
    float w = 1.0f;
    for (int j = 0; j < ndim; ++j) {
      const uint32_t r = words[j];
      const float y = (float)(r >> 9) * 0x1p-23f + 0x1p-24f;
      const float z = y * (float)nbins;
      int kk = (int)floorf(z);
      if (kk > nbins - 1) kk = nbins - 1;
      const float frac = z - (float)kk;
      const double *E = grid + (long long)j * (nbins + 1);
      const float lo = (float)E[kk], hi = (float)E[kk + 1];
      const float width = hi - lo;
      x[j] = (double)fmaf(frac, width, lo);
      w = w * ((float)nbins * width);
      k[j] = kk;
    }
    return (double)w;
  }
  double w = 1.0;
  for (int j = 0; j < ndim; ++j) {
    const uint32_t r = words[j];
    const double y = (double)r * 0x1p-32 + 0x1p-33;
    const double z = y * (double)nbins;
    int kk = (int)std::floor(z);
    if (kk > nbins - 1) kk = nbins - 1;
    const double frac = z - (double)kk;
    const double *E = grid + (long long)j * (nbins + 1);
    const double width = E[kk + 1] - E[kk];
    x[j] = std::fma(frac, width, E[kk]);
    w = w * ((double)nbins * width);
    k[j] = kk;
  }
  return w;
}

struct Combined {
  double integral, error, chi2, prob;
  int dof;
};

Combined combine(const std::vector<double> &I, const std::vector<double> &var) {
  Combined r{0.0, 0.0, 0.0, 0.0, 0};
  const int T = (int)I.size();
  r.dof = T - 1;
  int nzero = 0;
  double zsum = 0.0;
  for (int t = 0; t < T; ++t)
    if (var[t] == 0.0) {
      ++nzero;
      zsum += I[t];
    }
  if (nzero > 0) {
    r.integral = zsum / nzero;
    return r;
  }
  double wsum = 0.0, wisum = 0.0;
  for (int t = 0; t < T; ++t) {
    wsum += 1.0 / var[t];
    wisum += I[t] / var[t];
  }
  r.integral = wisum / wsum;
  r.error = std::sqrt(1.0 / wsum);
  double chi2 = 0.0;
  for (int t = 0; t < T; ++t) {
    const double dlt = I[t] - r.integral;
    chi2 += dlt * dlt / var[t];
  }
  r.chi2 = chi2;
  r.prob = r.dof > 0 ? oracle_gammainc_lower(0.5 * r.dof, 0.5 * chi2) : 0.0;
  return r;
}

}  // namespace

extern "C" void oracle_vegas_refine_dim(int nbins, const double *H,
                                        const double *E_in, double *E_out) {
  const int N = nbins;
  double hsum = 0.0;
  for (int k = 0; k < N; ++k) hsum += H[k];
  if (!(hsum > 0.0)) {
    for (int k = 0; k <= N; ++k) E_out[k] = E_in[k];
    return;
  }
  // smoothing
  std::vector<double> d(N);
  d[0] = (H[0] + H[1]) / 2.0;
  d[N - 1] = (H[N - 2] + H[N - 1]) / 2.0;
  for (int k = 1; k < N - 1; ++k) d[k] = (H[k - 1] + H[k] + H[k + 1]) / 3.0;
  double dsum = 0.0;
  for (int k = 0; k < N; ++k) dsum += d[k];
  // damping
  std::vector<double> m(N);
  for (int k = 0; k < N; ++k) {
    const double r = d[k] / dsum;
    if (r == 0.0)
      m[k] = 0.0;
    else if (r == 1.0)
      m[k] = 1.0;
    else
      m[k] = std::pow((r - 1.0) / std::log(r), 1.5);
  }
  // rebinning: prefix sums of m, equal shares of the total
  std::vector<double> C(N);
  double acc = 0.0;
  for (int k = 0; k < N; ++k) {
    acc += m[k];
    C[k] = acc;
  }
  const double share = C[N - 1] / N;
  E_out[0] = 0.0;
  E_out[N] = 1.0;
  int k = 0;
  for (int i = 1; i < N; ++i) {
    const double target = i * share;
    while (k < N - 1 && C[k] < target) ++k;
    const double before = k > 0 ? C[k - 1] : 0.0;
    E_out[i] = E_in[k] + (target - before) / m[k] * (E_in[k + 1] - E_in[k]);
  }
}

extern "C" int oracle_vegas_points(int ndim, int nbins, int precision,
                                   unsigned long long seed,
                                   unsigned int stream_id, int iteration,
                                   const double *grid, long long i0,
                                   long long npts, uint32_t *words, double *x,
                                   double *w, int *bin) {
  if (ndim < 1 || ndim > 16 || nbins < 2 || nbins > 256 || npts < 0 ||
      i0 < 0 || i0 + npts > (1ll << 32))
    return -1;
  const int nblk = (ndim + 3) / 4;
  std::vector<double> xx(ndim);
  std::vector<int> kk(ndim);
  for (long long p = 0; p < npts; ++p) {
    uint32_t wd[16];
    const double ww = map_point(ndim, nbins, precision, seed, stream_id,
                                iteration, grid, i0 + p, wd, xx.data(),
                                kk.data());
    if (words)
      for (int q = 0; q < 4 * nblk; ++q) words[p * 4 * nblk + q] = wd[q];
    if (x)
      for (int j = 0; j < ndim; ++j) x[p * ndim + j] = xx[j];
    if (bin)
      for (int j = 0; j < ndim; ++j) bin[p * ndim + j] = kk[j];
    if (w) w[p] = ww;
  }
  return 0;
}

extern "C" int oracle_vegas_from(const double *grid_in, int ndim, int ncomp,
                                 oracle_integrand_t integrand, void *userdata, int nvec,
                                 double epsrel, double epsabs, int flags,
                                 unsigned long long seed, long long mineval,
                                 long long maxeval, long long nstart, long long nincrease,
                                 long long nbatch, int nbins, unsigned int stream_id,
                                 long long *neval, int *fail, double integral[],
                                 double error[], double prob[], oracle_vegas_trace *trace);

extern "C" int oracle_vegas(int ndim, int ncomp, oracle_integrand_t integrand,
                            void *userdata, int nvec, double epsrel,
                            double epsabs, int flags, unsigned long long seed,
                            long long mineval, long long maxeval,
                            long long nstart, long long nincrease,
                            long long nbatch, int nbins,
                            unsigned int stream_id, long long *neval,
                            int *fail, double integral[], double error[],
                            double prob[], oracle_vegas_trace *trace) {
  return oracle_vegas_from(nullptr, ndim, ncomp, integrand, userdata, nvec, epsrel, epsabs,
                           flags, seed, mineval, maxeval, nstart, nincrease, nbatch, nbins,
                           stream_id, neval, fail, integral, error, prob, trace);
}

// The same run started from a given grid (ndim rows of nbins + 1 edges)
// instead of the uniform one: the grid of an earlier integration reused for a
// new one (iterations, sums and counters start afresh).
extern "C" int oracle_vegas_from(const double *grid_in, int ndim, int ncomp,
                                 oracle_integrand_t integrand, void *userdata, int nvec,
                                 double epsrel, double epsabs, int flags,
                                 unsigned long long seed, long long mineval,
                                 long long maxeval, long long nstart, long long nincrease,
                                 long long nbatch, int nbins, unsigned int stream_id,
                                 long long *neval, int *fail, double integral[],
                                 double error[], double prob[], oracle_vegas_trace *trace) {
  const int precision = flags & ORACLE_PRECISION_MASK;
  if (ndim < 1 || ndim > 16 || ncomp < 1 || ncomp > 16 || nvec < 1 || nbins < 2 ||
      nbins > 256 || nstart < 2 || nincrease < 0 || nbatch < 1 ||
      (precision != ORACLE_FP64 && precision != ORACLE_FP32_EVAL) ||
      !integrand)
    return -1;
  const int N = nbins;
  std::vector<double> grid((size_t)ndim * (N + 1));
  for (int j = 0; j < ndim; ++j)
    for (int k = 0; k <= N; ++k)
      grid[(size_t)j * (N + 1) + k] =
          grid_in ? grid_in[(size_t)j * (N + 1) + k] : (double)k / N;

  std::vector<double> hist((size_t)ndim * N);
  std::vector<std::vector<double>> It(ncomp), vart(ncomp);
  std::vector<Combined> res(ncomp, Combined{0.0, 0.0, 0.0, 0.0, -1});
  long long nev = 0;
  int status_fail = 1;
  std::vector<double> xbuf((size_t)nvec * ndim), fbuf((size_t)nvec * ncomp),
      wbuf(nvec);
  std::vector<int> kbuf((size_t)nvec * ndim);
  const int core = 32768;  // the master samples (serial mode)
  std::vector<double> shift(ncomp, 0.0);  // I_{t-1} of every component (0 at t = 0)

  for (int t = 0;; ++t) {
    const long long n = nstart + (long long)t * nincrease;
    if (n >= (1ll << 32) || t >= (1 << 24)) break;
    if (nev + n > maxeval) break;
    std::vector<Neumaier> s1(ncomp), s2(ncomp);
    std::vector<Neumaier> h((size_t)ndim * N);
    bool aborted = false;
    for (long long i0 = 0; i0 < n; i0 += nvec) {
      const int cnt = (int)((n - i0) < nvec ? (n - i0) : nvec);
      for (int p = 0; p < cnt; ++p)
        wbuf[p] = map_point(ndim, N, precision, seed, stream_id, t,
                            grid.data(), i0 + p, nullptr,
                            xbuf.data() + (size_t)p * ndim,
                            kbuf.data() + (size_t)p * ndim);
      const int nd = ndim, nc = ncomp;
      if (integrand(&nd, xbuf.data(), &nc, fbuf.data(), userdata, &cnt,
                    &core) == -999) {
        aborted = true;
        nev += i0 + cnt;  // every point handed to the integrand counts
        break;
      }
      for (int p = 0; p < cnt; ++p)
        for (int c = 0; c < ncomp; ++c) {
          double v;
          if (precision == ORACLE_FP32_EVAL)
            v = (double)((float)wbuf[p] * (float)fbuf[(size_t)p * ncomp + c]);
          else
            v = wbuf[p] * fbuf[(size_t)p * ncomp + c];
          const double v2 = v * v;
          const double dv = v - shift[c];
          s1[c].add(dv);
          s2[c].add(dv * dv);
          if (c == 0)
            for (int j = 0; j < ndim; ++j)
              h[(size_t)j * N + kbuf[(size_t)p * ndim + j]].add(v2);
        }
    }
    if (aborted) {
      *neval = nev;
      *fail = -99;
      for (int c = 0; c < ncomp; ++c) integral[c] = error[c] = prob[c] = 0.0;
      if (trace) trace->n_iter = (int)It[0].size();
      return 0;
    }
    nev += n;
    bool bad = false;
    for (int c = 0; c < ncomp; ++c)
      bad = bad || !std::isfinite(s1[c].value()) || !std::isfinite(s2[c].value());
    if (bad) {
      *neval = nev;
      *fail = -4;
      for (int c = 0; c < ncomp; ++c) integral[c] = error[c] = prob[c] = 0.0;
      if (trace) trace->n_iter = (int)It[0].size();
      return 0;
    }
    bool all = nev >= mineval;
    for (int c = 0; c < ncomp; ++c) {
      const double m = s1[c].value() / (double)n;
      const double I = shift[c] + m;
      double var = s2[c].value() / (double)n - m * m;
      if (var < 0.0) var = 0.0;
      var /= (double)(n - 1);
      shift[c] = I;
      It[c].push_back(I);
      vart[c].push_back(var);
      res[c] = combine(It[c], vart[c]);
      const double tol = std::fmax(epsabs, epsrel * std::fabs(res[c].integral));
      all = all && res[c].error <= tol;
    }
    for (size_t q = 0; q < hist.size(); ++q) hist[q] = h[q].value();
    if (all) {
      status_fail = 0;
      break;
    }
    if (!(flags & ORACLE_FREEZE_GRID)) {
      std::vector<double> enew(N + 1);
      for (int j = 0; j < ndim; ++j) {
        double *E = grid.data() + (size_t)j * (N + 1);
        oracle_vegas_refine_dim(N, hist.data() + (size_t)j * N, E, enew.data());
        for (int k = 0; k <= N; ++k) E[k] = enew[k];
      }
    }
  }
  *neval = nev;
  *fail = status_fail;
  for (int c = 0; c < ncomp; ++c) {
    integral[c] = res[c].integral;
    error[c] = res[c].error;
    prob[c] = res[c].prob;
  }
  if (trace) {  // component 0
    trace->n_iter = (int)It[0].size();
    for (int t = 0; t < (int)It[0].size() && t < trace->max_iter; ++t) {
      if (trace->iter_I) trace->iter_I[t] = It[0][t];
      if (trace->iter_var) trace->iter_var[t] = vart[0][t];
    }
    trace->chi2 = res[0].chi2;
    trace->dof = res[0].dof;
    if (trace->grid)
      for (size_t q = 0; q < grid.size(); ++q) trace->grid[q] = grid[q];
    if (trace->hist)
      for (size_t q = 0; q < hist.size(); ++q) trace->hist[q] = hist[q];
  }
  return 0;
}
