// genz.h -- device Genz test families, evaluated one dimension at a time.
//
// The workloads integrate Genz's families over [0,1]^d (Genz 1987):
//   Gaussian      exp(-sum a_i^2 (x_i - u_i)^2)
//   oscillatory   cos(2 pi u_1 + sum a_i x_i)
//   product peak  prod 1 / (a_i^-2 + (x_i - u_i)^2)
//   corner peak   (1 + sum a_i x_i)^-(d+1)
//   C0            exp(-sum a_i |x_i - u_i|)
// Each family is a sum or a product over dimensions, so a point's value is
// accumulated while its coordinates are produced and never needs all d
// coordinates in registers at once.
//
// Per-dimension constants are prepared once per integrand on the host, in
// FP64, and stored per precision (p[0][j], p[1][j]):
//   family        FP64 (p0, p1)        FP32 (p0, p1)
//   Gaussian      (a^2, u)             (a^2 log2 e, u)       f = 2^-s
//   oscillatory   (a, 2 pi u_1 in p1[0]) (a / 2 pi, u_1 in p1[0])  revolutions
//   product peak  (a^-2, u)            (a^-2, u)
//   corner peak   (a, -)               (a, -)
//   C0            (a, u)               (a log2 e, u)         f = 2^-s
// The FP32 forms fold the log2 e / 2 pi conversions into the constants, so
// that the hardware exp2 and a revolution-based cosine take the accumulated
// argument directly.
#pragma once
#ifndef CCUBA_RTC  // (hiprtc provides the HIP runtime)
#include <hip/hip_runtime.h>
#endif

#include "engine.h"

namespace ccuba {

template <typename T, int FAM>
struct Genz;

// ---- FP64 ------------------------------------------------------------------
template <>
struct Genz<double, GAUSSIAN> {
  static __device__ __forceinline__ double init(double) { return 0.0; }
  static __device__ __forceinline__ double step(double s, double x, double p0, double p1) {
    const double t = x - p1;
    return fma(p0, t * t, s);
  }
  static __device__ __forceinline__ double finish(double s, int) { return exp(-s); }
};
template <>
struct Genz<double, OSCILLATORY> {
  static __device__ __forceinline__ double init(double phase0) { return phase0; }
  static __device__ __forceinline__ double step(double s, double x, double p0, double) {
    return fma(p0, x, s);
  }
  static __device__ __forceinline__ double finish(double s, int) { return cos(s); }
};
template <>
struct Genz<double, PRODUCT_PEAK> {
  static __device__ __forceinline__ double init(double) { return 1.0; }
  static __device__ __forceinline__ double step(double s, double x, double p0, double p1) {
    const double t = x - p1;
    return s * fma(t, t, p0);
  }
  static __device__ __forceinline__ double finish(double s, int) { return 1.0 / s; }
};
template <>
struct Genz<double, CORNER_PEAK> {
  static __device__ __forceinline__ double init(double) { return 1.0; }
  static __device__ __forceinline__ double step(double s, double x, double p0, double) {
    return fma(p0, x, s);
  }
  static __device__ __forceinline__ double finish(double s, int d) {
    // s^(d+1) by binary powering, then one reciprocal
    double r = 1.0, b = s;
    for (int e = d + 1; e; e >>= 1) {
      if (e & 1) r *= b;
      b *= b;
    }
    return 1.0 / r;
  }
};
template <>
struct Genz<double, C0> {
  static __device__ __forceinline__ double init(double) { return 0.0; }
  static __device__ __forceinline__ double step(double s, double x, double p0, double p1) {
    return fma(p0, fabs(x - p1), s);
  }
  static __device__ __forceinline__ double finish(double s, int) { return exp(-s); }
};

// ---- FP32 ------------------------------------------------------------------
template <>
struct Genz<float, GAUSSIAN> {
  static __device__ __forceinline__ float init(float) { return 0.0f; }
  static __device__ __forceinline__ float step(float s, float x, float p0, float p1) {
    const float t = x - p1;
    return fmaf(p0, t * t, s);
  }
  static __device__ __forceinline__ float finish(float s, int) { return exp2f(-s); }
};
template <>
struct Genz<float, OSCILLATORY> {
  static __device__ __forceinline__ float init(float phase0) { return phase0; }
  static __device__ __forceinline__ float step(float s, float x, float p0, float) {
    return fmaf(p0, x, s);
  }
  static __device__ __forceinline__ float finish(float s, int) {
    const float r = s - rintf(s);  // exact: revolutions reduced to [-1/2, 1/2]
    return cospif(2.0f * r);
  }
};
template <>
struct Genz<float, PRODUCT_PEAK> {
  static __device__ __forceinline__ float init(float) { return 1.0f; }
  static __device__ __forceinline__ float step(float s, float x, float p0, float p1) {
    const float t = x - p1;
    return s * fmaf(t, t, p0);
  }
  static __device__ __forceinline__ float finish(float s, int) { return 1.0f / s; }
};
template <>
struct Genz<float, CORNER_PEAK> {
  static __device__ __forceinline__ float init(float) { return 1.0f; }
  static __device__ __forceinline__ float step(float s, float x, float p0, float) {
    return fmaf(p0, x, s);
  }
  static __device__ __forceinline__ float finish(float s, int d) {
    float r = 1.0f, b = s;
    for (int e = d + 1; e; e >>= 1) {
      if (e & 1) r *= b;
      b *= b;
    }
    return 1.0f / r;
  }
};
template <>
struct Genz<float, C0> {
  static __device__ __forceinline__ float init(float) { return 0.0f; }
  static __device__ __forceinline__ float step(float s, float x, float p0, float p1) {
    return fmaf(p0, fabsf(x - p1), s);
  }
  static __device__ __forceinline__ float finish(float s, int) { return exp2f(-s); }
};

}  // namespace ccuba
