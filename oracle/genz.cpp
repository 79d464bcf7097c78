// genz.cpp -- oracle: the Genz test families (TEST INFRASTRUCTURE ONLY).
//
// The workloads integrate Genz's test families (A. Genz, "A package for
// testing multiple integration subroutines", 1987) over [0,1]^d:
//   Gaussian      exp(-sum a_i^2 (x_i - u_i)^2)
//   oscillatory   cos(2 pi u_1 + sum a_i x_i)
//   product peak  prod 1 / (a_i^-2 + (x_i - u_i)^2)
//   corner peak   (1 + sum a_i x_i)^-(d+1)
//   C0            exp(-sum a_i |x_i - u_i|)
// In FP32-evaluate mode every operation is done in IEEE binary32 (C float,
// built with contraction off), with per-dimension constants rounded once from
// FP64, and the result is widened back to double.
#include <cmath>

#include "oracle.h"

namespace {

const double kTwoPi = 6.283185307179586476925286766559;

double genz_fp64(const oracle_genz *g, const double *x) {
  const int d = g->ndim;
  switch (g->family) {
    case ORACLE_GAUSSIAN: {
      double s = 0.0;
      for (int i = 0; i < d; ++i) {
        const double t = x[i] - g->u[i];
        s += g->a[i] * g->a[i] * t * t;
      }
      return std::exp(-s);
    }
    case ORACLE_OSCILLATORY: {
      double s = kTwoPi * g->u[0];
      for (int i = 0; i < d; ++i) s += g->a[i] * x[i];
      return std::cos(s);
    }
    case ORACLE_PRODUCT_PEAK: {
      double p = 1.0;
      for (int i = 0; i < d; ++i) {
        const double t = x[i] - g->u[i];
        p *= 1.0 / (1.0 / (g->a[i] * g->a[i]) + t * t);
      }
      return p;
    }
    case ORACLE_CORNER_PEAK: {
      double s = 1.0;
      for (int i = 0; i < d; ++i) s += g->a[i] * x[i];
      return std::pow(s, -(double)(d + 1));
    }
    case ORACLE_C0: {
      double s = 0.0;
      for (int i = 0; i < d; ++i) s += g->a[i] * std::fabs(x[i] - g->u[i]);
      return std::exp(-s);
    }
  }
  return NAN;
}

float genz_fp32(const oracle_genz *g, const double *xd) {
  const int d = g->ndim;
  switch (g->family) {
    case ORACLE_GAUSSIAN: {
      float s = 0.0f;
      for (int i = 0; i < d; ++i) {
        const float a2 = (float)(g->a[i] * g->a[i]);
        const float t = (float)xd[i] - (float)g->u[i];
        s = s + a2 * (t * t);
      }
      return expf(-s);
    }
    case ORACLE_OSCILLATORY: {
      float s = (float)(kTwoPi * g->u[0]);
      for (int i = 0; i < d; ++i) s = s + (float)g->a[i] * (float)xd[i];
      return cosf(s);
    }
    case ORACLE_PRODUCT_PEAK: {
      float p = 1.0f;
      for (int i = 0; i < d; ++i) {
        const float b = (float)(1.0 / (g->a[i] * g->a[i]));
        const float t = (float)xd[i] - (float)g->u[i];
        p = p * (b + t * t);
      }
      return 1.0f / p;
    }
    case ORACLE_CORNER_PEAK: {
      float s = 1.0f;
      for (int i = 0; i < d; ++i) s = s + (float)g->a[i] * (float)xd[i];
      return powf(s, -(float)(d + 1));
    }
    case ORACLE_C0: {
      float s = 0.0f;
      for (int i = 0; i < d; ++i)
        s = s + (float)g->a[i] * fabsf((float)xd[i] - (float)g->u[i]);
      return expf(-s);
    }
  }
  return NAN;
}

}  // namespace

extern "C" double oracle_genz_eval(const oracle_genz *g, const double *x) {
  if (g->precision == ORACLE_FP32_EVAL) return (double)genz_fp32(g, x);
  return genz_fp64(g, x);
}

extern "C" int oracle_genz_integrand(const int *ndim, const double x[],
                                     const int *ncomp, double f[],
                                     void *userdata, const int *nvec,
                                     const int *core) {
  (void)core;
  const oracle_genz *g = (const oracle_genz *)userdata;
  if (*ndim != g->ndim) return -999;
  for (int p = 0; p < *nvec; ++p) {
    f[p * *ncomp] = oracle_genz_eval(g, x + (long long)p * *ndim);
    for (int c = 1; c < *ncomp; ++c) f[p * *ncomp + c] = 0.0;
  }
  return 0;
}
