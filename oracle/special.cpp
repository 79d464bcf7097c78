// special.cpp -- oracle: lower regularized incomplete gamma function
// (TEST INFRASTRUCTURE ONLY).
//
// Vegas returns a chi^2 probability per component (Sect. 3.2.2, output
// prob[]).  The reading taken: prob = P(dof/2, chi2/2), the lower regularized
// incomplete gamma function, i.e. the chi^2 cumulative distribution at the
// observed chi^2 with dof = iterations - 1.
//
// P(a,x) is evaluated with the two classical expansions (Abramowitz & Stegun
// 6.5.29 and 6.5.31):
//   x <  a+1 : P = x^a e^-x / Gamma(a+1) * sum_n x^n / ((a+1)...(a+n))
//   x >= a+1 : Q = 1 - P from Legendre's continued fraction
//              Q = x^a e^-x / Gamma(a) * 1/(x+1-a- 1(1-a)/(x+3-a- 2(2-a)/(x+5-a- ...)))
//              evaluated with the modified Lentz algorithm.
#include <cmath>

#include "oracle.h"

namespace {

double series_p(double a, double x) {
  double term = 1.0 / a;
  double sum = term;
  for (int n = 1; n < 100000; ++n) {
    term *= x / (a + n);
    sum += term;
    if (std::fabs(term) < std::fabs(sum) * 1e-17) break;
  }
  return sum * std::exp(-x + a * std::log(x) - std::lgamma(a));
}

double contfrac_q(double a, double x) {
  const double tiny = 1e-300;
  double b = x + 1.0 - a;
  double c = 1.0 / tiny;
  double d = 1.0 / b;
  double h = d;
  for (int i = 1; i < 100000; ++i) {
    const double an = -i * (i - a);
    b += 2.0;
    d = an * d + b;
    if (std::fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double delta = d * c;
    h *= delta;
    if (std::fabs(delta - 1.0) < 1e-17) break;
  }
  return std::exp(-x + a * std::log(x) - std::lgamma(a)) * h;
}

}  // namespace

extern "C" double oracle_gammainc_lower(double a, double x) {
  if (!(a > 0.0) || x < 0.0) return NAN;
  if (x == 0.0) return 0.0;
  if (std::isinf(x)) return 1.0;
  if (x < a + 1.0) return series_p(a, x);
  return 1.0 - contfrac_q(a, x);
}
