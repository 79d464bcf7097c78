// cuhre.cpp -- oracle: plain serial Cuhre (TEST INFRASTRUCTURE ONLY).
//
// The paper fixes the interface (Sect. 3.2.2, Cuhre prototype: ndim, ncomp,
// integrand, userdata, nvec, epsrel, epsabs, flags, mineval, maxeval, key,
// ..., nregions, neval, fail, integral, error, prob) and leaves the rule to
// the literature.  The rule is the degree-7 rule of Genz and Malik
// (J. Comput. Appl. Math. 6 (1980) 295) with its embedded degree-5 rule, on
// the cube [-1,1]^d with generators
//   class 1: the centre                               (1 point)
//   class 2: +-l2 e_i,           l2^2 = 9/70          (2d points)
//   class 3: +-l3 e_i,           l3^2 = 9/10          (2d points)
//   class 4: +-l4 e_i +- l4 e_j, l4^2 = 9/10, i < j   (2d(d-1) points)
//   class 5: (+-l5, ..., +-l5),  l5^2 = 9/19          (2^d points)
// and weights (per point, cube volume 2^d included)
//   degree 7: 2^d (12824 - 9120 d + 400 d^2)/19683, 2^d 980/6561,
//             2^d (1820 - 400 d)/19683, 2^d 200/19683, 6859/19683
//   degree 5: 2^d (729 - 950 d + 50 d^2)/729, 2^d 245/486,
//             2^d (265 - 100 d)/1458, 2^d 25/729, 0.
// A region with centre c and half-widths h gets I = prod(h) sum w f(c + l.h).
// Readings where the paper is silent:
//  * error estimate err = |I7 - I5|;
//  * split axis: the largest fourth difference
//      D_i = |f(c+l2 h_i e_i) + f(c-l2 h_i e_i) - 2 f(c)
//             - (l2^2/l3^2)(f(c+l3 h_i e_i) + f(c-l3 h_i e_i) - 2 f(c))|,
//    lowest i on ties (Genz & Malik's subdivision criterion);
//  * global adaptivity in batches: while sum err > max(epsabs, epsrel |sum I7|)
//    or neval < mineval, pick K = min(floor(B/2), #regions) regions of largest
//    err (ties: lower id), bisect each along its split axis and evaluate the
//    2K children; K shrinks so that neval never passes maxeval, and if it
//    reaches 0 the run stops with fail 1;
//  * region ids in creation order: the root is 0; the j-th selected parent in
//    ascending id order gets children next+2j (lower half) and next+2j+1;
//  * prob = 0 (Cuhre has no chi^2 here);
//  * a non-finite total after the rule (a non-finite integrand value) ends
//    the run with fail -4 and zero results.
// Totals are Neumaier-compensated FP64 sums in ascending id order.
#include <algorithm>
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

struct Weights {
  double w7[5], w5[5];
  double l2, l3, l4, l5;
};

Weights gm_weights(int d) {
  Weights W;
  const double p2 = std::ldexp(1.0, d), dd = (double)d;
  W.w7[0] = p2 * (12824.0 - 9120.0 * dd + 400.0 * dd * dd) / 19683.0;
  W.w7[1] = p2 * 980.0 / 6561.0;
  W.w7[2] = p2 * (1820.0 - 400.0 * dd) / 19683.0;
  W.w7[3] = p2 * 200.0 / 19683.0;
  W.w7[4] = 6859.0 / 19683.0;
  W.w5[0] = p2 * (729.0 - 950.0 * dd + 50.0 * dd * dd) / 729.0;
  W.w5[1] = p2 * 245.0 / 486.0;
  W.w5[2] = p2 * (265.0 - 100.0 * dd) / 1458.0;
  W.w5[3] = p2 * 25.0 / 729.0;
  W.w5[4] = 0.0;
  W.l2 = std::sqrt(9.0 / 70.0);
  W.l3 = std::sqrt(9.0 / 10.0);
  W.l4 = std::sqrt(9.0 / 10.0);
  W.l5 = std::sqrt(9.0 / 19.0);
  return W;
}

struct Region {
  long long id;
  std::vector<double> c, h;
  double I7, I5, err;
  int axis;
};

// Lay out the rule points of one region in class order; cls[p] = class 0..4.
void rule_points(int d, const Weights &W, const double *c, const double *h,
                 std::vector<double> &x, std::vector<int> &cls) {
  x.clear();
  cls.clear();
  auto push = [&](const std::vector<double> &p, int k) {
    x.insert(x.end(), p.begin(), p.end());
    cls.push_back(k);
  };
  std::vector<double> p(c, c + d);
  push(p, 0);
  for (int i = 0; i < d; ++i) {
    for (int s = 0; s < 2; ++s) {
      p.assign(c, c + d);
      p[i] = s == 0 ? c[i] + W.l2 * h[i] : c[i] - W.l2 * h[i];
      push(p, 1);
    }
  }
  for (int i = 0; i < d; ++i) {
    for (int s = 0; s < 2; ++s) {
      p.assign(c, c + d);
      p[i] = s == 0 ? c[i] + W.l3 * h[i] : c[i] - W.l3 * h[i];
      push(p, 2);
    }
  }
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j < d; ++j)
      for (int s = 0; s < 4; ++s) {
        p.assign(c, c + d);
        p[i] = (s & 1) ? c[i] - W.l4 * h[i] : c[i] + W.l4 * h[i];
        p[j] = (s & 2) ? c[j] - W.l4 * h[j] : c[j] + W.l4 * h[j];
        push(p, 3);
      }
  for (long long s = 0; s < (1ll << d); ++s) {
    for (int i = 0; i < d; ++i)
      p[i] = ((s >> i) & 1) ? c[i] - W.l5 * h[i] : c[i] + W.l5 * h[i];
    push(p, 4);
  }
}

// Evaluate the rule on one region; returns 0 or -99 (abort).
int apply_rule(int d, oracle_integrand_t integrand, void *userdata, int nvec,
               const double *c, const double *h, double *I7, double *I5,
               double *err, int *axis, double *dfour) {
  const Weights W = gm_weights(d);
  std::vector<double> x;
  std::vector<int> cls;
  rule_points(d, W, c, h, x, cls);
  const long long np = (long long)cls.size();
  std::vector<double> f(np);
  const int core = 32768, ncomp = 1;
  for (long long p0 = 0; p0 < np; p0 += nvec) {
    const int cnt = (int)(np - p0 < nvec ? np - p0 : nvec);
    if (integrand(&d, x.data() + p0 * d, &ncomp, f.data() + p0, userdata, &cnt,
                  &core) == -999)
      return -99;
  }
  double S[5] = {0, 0, 0, 0, 0};
  for (long long p = 0; p < np; ++p) S[cls[p]] += f[p];
  double vol = 1.0;
  for (int i = 0; i < d; ++i) vol *= h[i];
  double r7 = 0.0, r5 = 0.0;
  for (int k = 0; k < 5; ++k) {
    r7 += W.w7[k] * S[k];
    r5 += W.w5[k] * S[k];
  }
  *I7 = vol * r7;
  *I5 = vol * r5;
  *err = std::fabs(*I7 - *I5);
  // fourth differences: class-2 points 1 + 2i (+), 2 + 2i (-);
  // class-3 points 1 + 2d + 2i (+), 2 + 2d + 2i (-)
  const double f0 = f[0];
  const double ratio = (W.l2 * W.l2) / (W.l3 * W.l3);
  int best = 0;
  double bestD = -1.0;
  for (int i = 0; i < d; ++i) {
    const double a2 = f[1 + 2 * i] + f[2 + 2 * i] - 2.0 * f0;
    const double a3 = f[1 + 2 * d + 2 * i] + f[2 + 2 * d + 2 * i] - 2.0 * f0;
    const double D = std::fabs(a2 - ratio * a3);
    if (dfour) dfour[i] = D;
    if (D > bestD) {
      bestD = D;
      best = i;
    }
  }
  *axis = best;
  return 0;
}

}  // namespace

extern "C" long long oracle_gm_npoints(int ndim) {
  return (1ll << ndim) + 2ll * ndim * ndim + 2ll * ndim + 1;
}

extern "C" int oracle_gm_rule(int ndim, oracle_integrand_t integrand,
                              void *userdata, int nvec, const double *c,
                              const double *h, double *I7, double *I5,
                              double *err, int *axis, double *dfour) {
  if (ndim < 2 || ndim > 16 || nvec < 1 || !integrand) return -1;
  return apply_rule(ndim, integrand, userdata, nvec, c, h, I7, I5, err, axis,
                    dfour);
}

extern "C" int oracle_cuhre(int ndim, int ncomp, oracle_integrand_t integrand,
                            void *userdata, int nvec, double epsrel,
                            double epsabs, int flags, long long mineval,
                            long long maxeval, int key,
                            long long max_regions_per_batch, int *nregions,
                            long long *neval, int *fail, double integral[],
                            double error[], double prob[],
                            oracle_cuhre_trace *trace) {
  (void)flags;
  if (ndim < 2 || ndim > 16 || ncomp != 1 || nvec < 1 || !integrand ||
      (key != 0 && key != 7) || max_regions_per_batch < 2)
    return -1;
  const int d = ndim;
  const long long np = oracle_gm_npoints(d);
  std::vector<Region> leaves;
  Region root;
  root.id = 0;
  root.c.assign(d, 0.5);
  root.h.assign(d, 0.5);
  long long nev = 0;
  int batches = 0;
  auto finish = [&](int f, double I, double E) {
    *nregions = (int)leaves.size();
    *neval = nev;
    *fail = f;
    integral[0] = I;
    error[0] = E;
    prob[0] = 0.0;
    if (trace) trace->n_batches = batches;
    return 0;
  };
  if (apply_rule(d, integrand, userdata, nvec, root.c.data(), root.h.data(),
                 &root.I7, &root.I5, &root.err, &root.axis, nullptr) != 0) {
    nev += np;
    return finish(-99, 0.0, 0.0);
  }
  nev += np;
  leaves.push_back(root);
  long long next_id = 1;
  for (;;) {
    Neumaier tI, tE;
    for (const Region &r : leaves) {
      tI.add(r.I7);
      tE.add(r.err);
    }
    const double I = tI.value(), E = tE.value();
    if (!std::isfinite(I) || !std::isfinite(E)) return finish(-4, 0.0, 0.0);
    if (nev >= mineval && E <= std::fmax(epsabs, epsrel * std::fabs(I)))
      return finish(0, I, E);
    long long K = std::min(max_regions_per_batch / 2, (long long)leaves.size());
    const long long budget = maxeval > nev ? (maxeval - nev) / (2 * np) : 0;
    K = std::min(K, budget);
    if (K <= 0) return finish(1, I, E);
    // top-K by (err descending, id ascending); leaves are in ascending id
    std::vector<size_t> order(leaves.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
      return leaves[a].err > leaves[b].err;
    });
    std::vector<char> chosen(leaves.size(), 0);
    for (long long q = 0; q < K; ++q) chosen[order[q]] = 1;
    std::vector<Region> kept, children;
    for (size_t q = 0; q < leaves.size(); ++q) {
      if (!chosen[q]) {
        kept.push_back(leaves[q]);
        continue;
      }
      const Region &P = leaves[q];
      const int s = P.axis;
      for (int side = 0; side < 2; ++side) {
        Region ch;
        ch.id = next_id++;
        ch.c = P.c;
        ch.h = P.h;
        ch.h[s] = P.h[s] / 2.0;
        ch.c[s] = side == 0 ? P.c[s] - ch.h[s] : P.c[s] + ch.h[s];
        children.push_back(ch);
      }
    }
    for (Region &ch : children) {
      if (apply_rule(d, integrand, userdata, nvec, ch.c.data(), ch.h.data(),
                     &ch.I7, &ch.I5, &ch.err, &ch.axis, nullptr) != 0) {
        nev += np;
        leaves = kept;
        return finish(-99, 0.0, 0.0);
      }
      nev += np;
    }
    ++batches;
    leaves = kept;
    leaves.insert(leaves.end(), children.begin(), children.end());
  }
}
