// cuhre.hip -- Cuhre on gfx950: the degree-7 Genz-Malik rule over batches of
// subregions, top-K selection, bisection and compaction of the region heap.
//
// a8 (the DoSample of Cuhre): one wavefront per region.  The lanes walk the
//    2^d + 2d^2 + 2d + 1 rule points (Genz & Malik 1980) of their region,
//    decoding each point index to its generator class and axes, evaluate the
//    Genz integrand in FP64, and keep five class sums; the class-2 and
//    class-3 values and the centre go to LDS for the fourth differences.
//    Wave shuffles reduce the class sums; lane 0 forms
//      I7 = prod(h) sum_k w7_k S_k,  I5 = prod(h) sum_k w5_k S_k,
//      err = |I7 - I5|,
//    and the lanes j < d form the fourth difference
//      D_j = |f(c+l2 h_j e_j) + f(c-l2 h_j e_j) - 2 f(c)
//             - (l2^2/l3^2)(f(c+l3 h_j e_j) + f(c-l3 h_j e_j) - 2 f(c))|,
//    whose arg-max (lowest j on ties) is the split axis.  A launch takes a
//    list of segments, so regions of several integrals share one launch.
// a9 (region step): the store of regions only grows (a region's position is
//    its id) and a split region is retired in place.  Selection of the K
//    largest errors by a 16-bit digit histogram and an exact rank within the
//    boundary digit (ties go to the lower position, i.e. the lower region
//    id); a counting pass and a scan give each selected region its rank j,
//    and the rule launch forms the two halves of the j-th at the end of the
//    store before it evaluates them; a fixed-order reduction gives the
//    totals.  Where a step needs the whole grid's results (a scan of block
//    counts, a reduction of block sums, a pick from the histogram), a
//    one-workgroup kernel follows: no block ever waits for another, and no
//    block fences for another (a device-scope release writes back the L2
//    of its XCD, ~0.7 us each, serialised per XCD, which costs more per
//    block than a kernel boundary costs once).
#include <algorithm>

#include "cuhre.h"
#include "genz.h"

namespace ccuba {

namespace {

constexpr int kLaneRuleMaxDim = 8;          // lane-per-region rule up to this d
constexpr long long kLaneRuleMinRegions = 512;  // and from this many regions on
constexpr long long kOneLaneRuleMinRegions = 49152;  // one lane per region from here
constexpr long long kWaveRuleBlocks = 2048;       // most blocks of a wave-per-region launch
constexpr int kScanItems = 4;
constexpr int kScanBlock = 256;
constexpr int kScanTile = kScanItems * kScanBlock;  // elements per scan block

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Selection key of a region: the IEEE bit pattern of its error plus one,
// which orders the non-negative doubles; 0 for a retired region (negative
// error), below every live one.
__device__ __forceinline__ unsigned long long key_of(double e) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(e);
  return (b >> 63) ? 0ull : b + 1ull;
}

__device__ __forceinline__ bool retired(double e) { return signbit(e); }

// The geometry of region r of a segment: loaded, or formed from its parent
// (children mode) and stored.  Lane `j' (< d) handles coordinate j.
__device__ __forceinline__ void child_coord(const CSeg &S, long long r, int j, double *cj,
                                            double *hj) {
  const long long cap = S.regs.cap;
  if (!S.children) {
    *cj = S.regs.c[j * cap + r];
    *hj = S.regs.h[j * cap + r];
    return;
  }
  const long long k = r - S.first;
  const long long p = S.parent ? S.parent[k >> 1] : S.pbase + (k >> 1);
  double c = S.regs.c[j * cap + p], h = S.regs.h[j * cap + p];
  if (j == S.regs.axis[p]) {
    h = h / 2.0;
    c = (k & 1) ? c + h : c - h;
  }
  S.regs.c[j * cap + r] = c;
  S.regs.h[j * cap + r] = h;
  if (S.retire && j == 0 && !(k & 1)) S.regs.err[p] = -1.0;
  *cj = c;
  *hj = h;
}

// Evaluate the Genz family FAM at the rule point described by (cls, i, jj,
// sgn): class 0 centre; 1 and 2: axis i with sign bit 0; 3: axes i < jj with
// sign bits 0 (i) and 1 (jj); 4: every axis, sign bit j for axis j.
template <int FAM>
__device__ __forceinline__ double rule_point_f(int d, const double *c, const double *h,
                                               const double *p0, const double *p1, int cls,
                                               int i, int jj, unsigned sgn, double lam,
                                               double phase0) {
  double acc = Genz<double, FAM>::init(phase0);
  for (int j = 0; j < d; ++j) {
    double x = c[j];
    bool on;
    bool neg;
    if (cls == 4) {
      on = true;
      neg = (sgn >> j) & 1u;
    } else if (cls == 3) {
      on = (j == i) || (j == jj);
      neg = (j == i) ? (sgn & 1u) : ((sgn >> 1) & 1u);
    } else {
      on = (cls != 0) && (j == i);
      neg = sgn & 1u;
    }
    if (on) {
      const double t = lam * h[j];
      x = neg ? x - t : x + t;
    }
    acc = Genz<double, FAM>::step(acc, x, p0[j], p1[j]);
  }
  return Genz<double, FAM>::finish(acc, d);
}

// One region per wavefront; returns (I7, err) in lane 0.
template <int FAM>
__device__ double2 rule_region(const RuleArgs &A, const CSeg &S, long long r, int w, int lane,
                               double (*sc)[kMaxDim], double (*sh)[kMaxDim],
                               double (*sf)[4 * kMaxDim + 1], double (*sx)[2 * kMaxDim]) {
  const int d = S.ndim;
  if (lane < d) child_coord(S, r, lane, &sc[w][lane], &sh[w][lane]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const double *c = sc[w], *h = sh[w];
  const double *p0 = S.par;
  const double *p1 = S.par + kParamRow;
  const double phase0 = p1[0];
  const long long n2 = 2ll * d, n4 = 2ll * d * (d - 1);
  const long long b2 = 1, b3 = 1 + n2, b4 = 1 + 2 * n2, b5 = 1 + 2 * n2 + n4;
  double Sk[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  // classes 0-3 (a few hundred points at most)
  for (long long p = lane; p < b5; p += 64) {
    int cls, i = 0, jj = 0;
    unsigned sgn = 0;
    double lam = 0.0;
    if (p == 0) {
      cls = 0;
    } else if (p < b3) {
      cls = 1;
      i = (int)((p - b2) >> 1);
      sgn = (unsigned)((p - b2) & 1);
      lam = A.l2;
    } else if (p < b4) {
      cls = 2;
      i = (int)((p - b3) >> 1);
      sgn = (unsigned)((p - b3) & 1);
      lam = A.l3;
    } else if (p < b5) {
      cls = 3;
      long long q = (p - b4) >> 2;
      sgn = (unsigned)((p - b4) & 3);
      i = 0;
      int row = d - 1;
      while (q >= row) {
        q -= row;
        ++i;
        --row;
      }
      jj = i + 1 + (int)q;
      lam = A.l4;
    } else {
      cls = 4;
      sgn = (unsigned)(p - b5);
      lam = A.l5;
    }
    const double f = rule_point_f<FAM>(d, c, h, p0, p1, cls, i, jj, sgn, lam, phase0);
    Sk[cls] += f;
    if (cls == 0) sf[w][4 * kMaxDim] = f;
    if (cls == 1) sf[w][(int)(p - b2)] = f;                 // [2i + sign]
    if (cls == 2) sf[w][2 * kMaxDim + (int)(p - b3)] = f;   // [2d.. + 2i + sign]
  }
  // class 4, the 2^d corners (all of the work at large d): both coordinates
  // of every axis, c - l5 h and c + l5 h, are formed once per region (the
  // values rule_point_f forms per point), so a corner is d selects and the
  // integrand's own steps
  if (lane < d) {
    const double t = A.l5 * h[lane];
    sx[w][2 * lane] = c[lane] + t;
    sx[w][2 * lane + 1] = c[lane] - t;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const unsigned ncorner = 1u << d;
  for (unsigned sg = lane; sg < ncorner; sg += 64) {
    double acc = Genz<double, FAM>::init(phase0);
    for (int j = 0; j < d; ++j)
      acc = Genz<double, FAM>::step(acc, sx[w][2 * j + ((sg >> j) & 1u)], p0[j], p1[j]);
    Sk[4] += Genz<double, FAM>::finish(acc, d);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) Sk[k] = wsum(Sk[k]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // fourth differences and the arg-max axis (lowest axis on ties)
  double D = -1.0;
  if (lane < d) {
    const double f0 = sf[w][4 * kMaxDim];
    const double a2 = sf[w][2 * lane] + sf[w][2 * lane + 1] - 2.0 * f0;
    const double a3 = sf[w][2 * kMaxDim + 2 * lane] + sf[w][2 * kMaxDim + 2 * lane + 1] - 2.0 * f0;
    const double ratio = (A.l2 * A.l2) / (A.l3 * A.l3);
    D = fabs(a2 - ratio * a3);
  }
  int best = lane;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double oD = __shfl_xor(D, o, 64);
    const int ob = __shfl_xor(best, o, 64);
    if (oD > D || (oD == D && ob < best)) {
      D = oD;
      best = ob;
    }
  }
  if (lane == 0) {
    double vol = 1.0;
    for (int j = 0; j < d; ++j) vol *= h[j];
    const double *w7 = A.w7 + d * 5, *w5 = A.w5 + d * 5;
    double r7 = 0.0, r5 = 0.0;
    for (int k = 0; k < 5; ++k) {
      r7 += w7[k] * Sk[k];
      r5 += w5[k] * Sk[k];
    }
    const double I7 = vol * r7, I5 = vol * r5;
    S.regs.I7[r] = I7;
    S.regs.I5[r] = I5;
    S.regs.err[r] = fabs(I7 - I5);
    S.regs.axis[r] = best;
    return make_double2(I7, fabs(I7 - I5));
  }
  return make_double2(0.0, 0.0);
}

// One lane per region, for a single integral of dimension D <= 8: every lane
// takes the rule points in the same order, so the point's class and axes are
// the same across the wavefront (decoded once, in scalar registers) and only
// the region's centre and widths differ.  The point values are the same
// arithmetic as rule_point_f; the class sums are taken in point order.
template <int FAM, int D>
__device__ __forceinline__ double lane_point(const double (&c)[D], const double (&h)[D],
                                             const double *p0, const double *p1,
                                             double phase0, int i, bool ni, int jj, bool nj,
                                             double lam) {
  double acc = Genz<double, FAM>::init(phase0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double x = c[j];
    if (j == i || j == jj) {
      const double t = lam * h[j];
      const bool neg = j == i ? ni : nj;
      x = neg ? x - t : x + t;
    }
    acc = Genz<double, FAM>::step(acc, x, p0[j], p1[j]);
  }
  return Genz<double, FAM>::finish(acc, D);
}

// All the rule points of one region in one lane, in point order (the
// arithmetic of rule_region's points); returns (I7, err).
template <int FAM, int D>
__device__ double2 rule_region_lane(const RuleArgs &A, const CSeg &S, long long r) {
  const long long cap = S.regs.cap;
  double c[D], h[D];
  if (!S.children) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      c[j] = S.regs.c[j * cap + r];
      h[j] = S.regs.h[j * cap + r];
    }
  } else {  // a child: formed from its parent, as child_coord does per axis
    const long long k = r - S.first;
    const long long p = S.parent ? S.parent[k >> 1] : S.pbase + (k >> 1);
    const int ax = S.regs.axis[p];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      c[j] = S.regs.c[j * cap + p];
      h[j] = S.regs.h[j * cap + p];
      if (j == ax) {
        h[j] = h[j] / 2.0;
        c[j] = (k & 1) ? c[j] + h[j] : c[j] - h[j];
      }
      S.regs.c[j * cap + r] = c[j];
      S.regs.h[j * cap + r] = h[j];
    }
    if (S.retire && !(k & 1)) S.regs.err[p] = -1.0;
  }
  const double *p0 = S.par;
  const double *p1 = S.par + kParamRow;
  const double phase0 = p1[0];
  double Sk[5];
  // class 0: the centre
  const double f0 = lane_point<FAM, D>(c, h, p0, p1, phase0, -1, false, -1, false, 0.0);
  Sk[0] = f0;
  // classes 1 and 2: +-lambda on one axis; the fourth differences
  double s1 = 0.0, s2 = 0.0, Dmax = -1.0;
  int best = 0;
  double a2[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double fp = lane_point<FAM, D>(c, h, p0, p1, phase0, i, false, -1, false, A.l2);
    const double fm = lane_point<FAM, D>(c, h, p0, p1, phase0, i, true, -1, false, A.l2);
    s1 += fp;
    s1 += fm;
    a2[i] = fp + fm - 2.0 * f0;
  }
  const double ratio = (A.l2 * A.l2) / (A.l3 * A.l3);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double fp = lane_point<FAM, D>(c, h, p0, p1, phase0, i, false, -1, false, A.l3);
    const double fm = lane_point<FAM, D>(c, h, p0, p1, phase0, i, true, -1, false, A.l3);
    s2 += fp;
    s2 += fm;
    const double a3 = fp + fm - 2.0 * f0;
    const double Dj = fabs(a2[i] - ratio * a3);
    if (Dj > Dmax) {  // strictly greater: the lowest axis wins ties
      Dmax = Dj;
      best = i;
    }
  }
  Sk[1] = s1;
  Sk[2] = s2;
  // class 3: +-lambda4 on two axes i < jj
  double s3 = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int jj = i + 1; jj < D; ++jj)
#pragma unroll
      for (int sg = 0; sg < 4; ++sg)
        s3 += lane_point<FAM, D>(c, h, p0, p1, phase0, i, sg & 1, jj, (sg >> 1) & 1, A.l4);
  Sk[3] = s3;
  // class 4: every corner at +-lambda5
  double s4 = 0.0;
  for (unsigned sg = 0; sg < (1u << D); ++sg) {
    double acc = Genz<double, FAM>::init(phase0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double t = A.l5 * h[j];
      const double x = ((sg >> j) & 1u) ? c[j] - t : c[j] + t;
      acc = Genz<double, FAM>::step(acc, x, p0[j], p1[j]);
    }
    s4 += Genz<double, FAM>::finish(acc, D);
  }
  Sk[4] = s4;
  double vol = 1.0;
#pragma unroll
  for (int j = 0; j < D; ++j) vol *= h[j];
  const double *w7 = A.w7 + D * 5, *w5 = A.w5 + D * 5;
  double r7 = 0.0, r5 = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    r7 += w7[k] * Sk[k];
    r5 += w5[k] * Sk[k];
  }
  const double I7 = vol * r7, I5 = vol * r5;
  S.regs.I7[r] = I7;
  S.regs.I5[r] = I5;
  S.regs.err[r] = fabs(I7 - I5);
  S.regs.axis[r] = best;
  return make_double2(I7, fabs(I7 - I5));
}

// The rule points of one region split over the four wavefronts of a block
// (lane l of every wavefront holds region l of the block's 64): wavefront 0
// takes the centre, classes 1 and 2 and the fourth differences; classes 3
// (the pairs of axes, in order, dealt round-robin to wavefronts 1-3) and 4
// (corner sg to wavefront sg mod 4) are shared.  Each wavefront's class sums
// go to LDS (sums[w][k][lane]); wavefront 0 adds the four in wavefront order
// and forms I7, I5, err and the split axis.  Returns (I7, err) in
// wavefront 0's lanes of live regions.
template <int FAM, int D>
__device__ double2 rule_region_quad(const RuleArgs &A, const CSeg &S, long long r, bool live,
                                    int w, int lane, double (*sums)[5][64]) {
  const long long cap = S.regs.cap;
  double c[D], h[D];
#pragma unroll
  for (int j = 0; j < D; ++j) c[j] = h[j] = 0.5;  // (a lane past the end computes on these)
  if (live && !S.children) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      c[j] = S.regs.c[j * cap + r];
      h[j] = S.regs.h[j * cap + r];
    }
  } else if (live) {  // a child: formed from its parent, as child_coord does per axis
    const long long k = r - S.first;
    const long long p = S.parent ? S.parent[k >> 1] : S.pbase + (k >> 1);
    const int ax = S.regs.axis[p];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      c[j] = S.regs.c[j * cap + p];
      h[j] = S.regs.h[j * cap + p];
      if (j == ax) {
        h[j] = h[j] / 2.0;
        c[j] = (k & 1) ? c[j] + h[j] : c[j] - h[j];
      }
      if (w == 0) {
        S.regs.c[j * cap + r] = c[j];
        S.regs.h[j * cap + r] = h[j];
      }
    }
    if (w == 0 && S.retire && !(k & 1)) S.regs.err[p] = -1.0;
  }
  const double *p0 = S.par;
  const double *p1 = S.par + kParamRow;
  const double phase0 = p1[0];
  double Sk[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int best = 0;
  if (w == 0) {
    // class 0: the centre
    const double f0 = lane_point<FAM, D>(c, h, p0, p1, phase0, -1, false, -1, false, 0.0);
    Sk[0] = f0;
    // classes 1 and 2: +-lambda on one axis; the fourth differences
    double s1 = 0.0, s2 = 0.0, Dmax = -1.0;
    double a2[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double fp = lane_point<FAM, D>(c, h, p0, p1, phase0, i, false, -1, false, A.l2);
      const double fm = lane_point<FAM, D>(c, h, p0, p1, phase0, i, true, -1, false, A.l2);
      s1 += fp;
      s1 += fm;
      a2[i] = fp + fm - 2.0 * f0;
    }
    const double ratio = (A.l2 * A.l2) / (A.l3 * A.l3);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double fp = lane_point<FAM, D>(c, h, p0, p1, phase0, i, false, -1, false, A.l3);
      const double fm = lane_point<FAM, D>(c, h, p0, p1, phase0, i, true, -1, false, A.l3);
      s2 += fp;
      s2 += fm;
      const double a3 = fp + fm - 2.0 * f0;
      const double Dj = fabs(a2[i] - ratio * a3);
      if (Dj > Dmax) {  // strictly greater: the lowest axis wins ties
        Dmax = Dj;
        best = i;
      }
    }
    Sk[1] = s1;
    Sk[2] = s2;
  } else {
    // class 3: +-lambda4 on two axes i < jj, pair q to wavefront 1 + q mod 3
    double s3 = 0.0;
    int q = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int jj = i + 1; jj < D; ++jj, ++q)
        if (q % 3 == w - 1)
#pragma unroll
          for (int sg = 0; sg < 4; ++sg)
            s3 += lane_point<FAM, D>(c, h, p0, p1, phase0, i, sg & 1, jj, (sg >> 1) & 1, A.l4);
    Sk[3] = s3;
  }
  // class 4: the corners at +-lambda5, corner sg to wavefront sg mod 4
  double s4 = 0.0;
  for (unsigned sg = (unsigned)w; sg < (1u << D); sg += 4u) {
    double acc = Genz<double, FAM>::init(phase0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double t = A.l5 * h[j];
      const double x = ((sg >> j) & 1u) ? c[j] - t : c[j] + t;
      acc = Genz<double, FAM>::step(acc, x, p0[j], p1[j]);
    }
    s4 += Genz<double, FAM>::finish(acc, D);
  }
  Sk[4] = s4;
#pragma unroll
  for (int k = 0; k < 5; ++k) sums[w][k][lane] = Sk[k];
  __syncthreads();
  if (w != 0 || !live) return make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 5; ++k)
    Sk[k] = ((sums[0][k][lane] + sums[1][k][lane]) + sums[2][k][lane]) + sums[3][k][lane];
  double vol = 1.0;
#pragma unroll
  for (int j = 0; j < D; ++j) vol *= h[j];
  const double *w7 = A.w7 + D * 5, *w5 = A.w5 + D * 5;
  double r7 = 0.0, r5 = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    r7 += w7[k] * Sk[k];
    r5 += w5[k] * Sk[k];
  }
  const double I7 = vol * r7, I5 = vol * r5;
  S.regs.I7[r] = I7;
  S.regs.I5[r] = I5;
  S.regs.err[r] = fabs(I7 - I5);
  S.regs.axis[r] = best;
  return make_double2(I7, fabs(I7 - I5));
}

}  // namespace

__global__ void cuhre_root_kernel(CRegions R, int d, int *done) {
  const int j = threadIdx.x;
  if (j < d) {
    R.c[j * R.cap] = 0.5;
    R.h[j * R.cap] = 0.5;
  }
  if (j == 0 && done) *done = 0;
}

// a run's launches do nothing once its stop flag is set
__device__ __forceinline__ bool stopped(const int *done) { return done && *done != 0; }

namespace {

// Sums over a block of up to 1024 threads in a fixed order (a butterfly in
// each wavefront, lane 0's result, then the wavefronts in order); every
// thread gets the sums.
__device__ __forceinline__ double2 block_sum2(double a, double b) {
  __shared__ double s[2][16];
  a = wsum(a);
  b = wsum(b);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();  // an earlier call's readers are done with s
  if ((threadIdx.x & 63) == 0) {
    s[0][w] = a;
    s[1][w] = b;
  }
  __syncthreads();
  double x = 0.0, y = 0.0;
  for (int q = 0; q < nw; ++q) {
    x += s[0][q];
    y += s[1][q];
  }
  return make_double2(x, y);
}

// The stop rule on a step's totals: 0 go on, 1 converged, 2 not finite.
__device__ __forceinline__ int stop_code(double I, double E, const CStop &stop) {
  if (!isfinite(I) || !isfinite(E)) return 2;
  if (stop.neval >= stop.mineval && E <= fmax(stop.epsabs, stop.epsrel * fabs(I))) return 1;
  return 0;
}

// The opening of a step (CRows): true if the run goes on.  Every thread of
// the block must call it.
__device__ __forceinline__ bool open_step(const CRows &R, int *done) {
  if (!R.in) return true;
  double x = 0.0, y = 0.0;
  for (long long i = threadIdx.x; i < R.nin; i += blockDim.x) {
    x += R.in[i];
    y += R.in[R.stride + i];
  }
  const double2 T = block_sum2(x, y);
  const int code = stop_code(T.x, T.y, R.stop);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    R.slot[0] = T.x;
    R.slot[1] = T.y;
    __hip_atomic_store((unsigned long long *)(R.slot + 2),
                       ((unsigned long long)R.seq << 8) | (unsigned long long)code,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (code && done) *done = 1;
  }
  return code == 0;
}

// One row of the next state: the block's sums (every thread calls it).
__device__ __forceinline__ void put_row(const CRows &R, double a, double b) {
  if (!R.out) return;
  const double2 t = block_sum2(a, b);
  if (threadIdx.x == 0) {
    R.out[R.out0 + blockIdx.x] = t.x;
    R.out[R.stride + R.out0 + blockIdx.x] = t.y;
  }
}

}  // namespace

// One integral (A.one), dimension D, one lane per region: for launches large
// enough to fill the device with a wavefront per 64 regions.
template <int FAM, int D>
__global__ void __launch_bounds__(256) gm_rule_lane1_kernel(RuleArgs A) {
  if (stopped(A.done) || !open_step(A.rows, A.done)) return;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double2 v = make_double2(0.0, 0.0);
  if (g < A.total) v = rule_region_lane<FAM, D>(A, A.one, A.one.first + g);
  put_row(A.rows, v.x, v.y);
}

// One integral (A.one), dimension D: 64 regions per block, one lane of each
// of the block's four wavefronts per region (rule_region_quad).
template <int FAM, int D>
__global__ void __launch_bounds__(256) gm_rule_lane_kernel(RuleArgs A) {
  __shared__ double sums[4][5][64];
  if (stopped(A.done) || !open_step(A.rows, A.done)) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long g = (long long)blockIdx.x * 64 + lane;
  const double2 v =
      rule_region_quad<FAM, D>(A, A.one, A.one.first + g, g < A.total, w, lane, sums);
  put_row(A.rows, v.x, v.y);
}

// A wavefront per region, the regions of a launch taken in turn by the grid's
// wavefronts (a launch has at most kWaveRuleBlocks blocks).
__global__ void __launch_bounds__(256) gm_rule_kernel(RuleArgs A) {
  __shared__ double sc[4][kMaxDim], sh[4][kMaxDim];
  __shared__ double sf[4][4 * kMaxDim + 1];
  __shared__ double sx[4][2 * kMaxDim];
  if (stopped(A.done) || !open_step(A.rows, A.done)) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double a = 0.0, b = 0.0;
  for (long long g = (long long)blockIdx.x * 4 + w; g < A.total; g += (long long)gridDim.x * 4) {
    CSeg S;
    long long before = 0;
    if (A.nseg == 1) {
      S = A.one;
    } else {
      int lo = 0, hi = A.nseg - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A.seg_end[mid] > g)
          hi = mid;
        else
          lo = mid + 1;
      }
      S = A.segs[lo];
      before = lo > 0 ? A.seg_end[lo - 1] : 0;
    }
    const long long r = S.first + (g - before);
    double2 v;
    switch (S.family) {
      case GAUSSIAN: v = rule_region<GAUSSIAN>(A, S, r, w, lane, sc, sh, sf, sx); break;
      case OSCILLATORY: v = rule_region<OSCILLATORY>(A, S, r, w, lane, sc, sh, sf, sx); break;
      case PRODUCT_PEAK: v = rule_region<PRODUCT_PEAK>(A, S, r, w, lane, sc, sh, sf, sx); break;
      case CORNER_PEAK: v = rule_region<CORNER_PEAK>(A, S, r, w, lane, sc, sh, sf, sx); break;
      default: v = rule_region<C0>(A, S, r, w, lane, sc, sh, sf, sx); break;
    }
    a += v.x;  // lane 0 only: the others hold 0
    b += v.y;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the LDS rows are reused by the next region
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  put_row(A.rows, a, b);
}

// A step opened alone (one block).
__global__ void __launch_bounds__(256) cuhre_decide_kernel(CRows R, int *done) {
  if (stopped(done)) return;
  (void)open_step(R, done);
}

// ---------------------------------------------------------------------------
// block-level exclusive scan of per-thread counts (256 threads)

__device__ __forceinline__ long long block_excl_scan(long long v, long long *total) {
  __shared__ long long wtot[kScanBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  long long incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  long long off = 0, tot = 0;
  for (int q = 0; q < kScanBlock / 64; ++q) {
    if (q < w) off += wtot[q];
    tot += wtot[q];
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

// Whether the region at position i is at or above the threshold (key thr,
// position tpos) in the selection order (key descending, position
// ascending).
__device__ __forceinline__ bool selected(double e, long long i, unsigned long long thr,
                                         long long tpos) {
  const unsigned long long k = key_of(e);
  return k > thr || (k == thr && i <= tpos);
}

constexpr int kTopBins = 1 << 16;
constexpr int kTopThreads = 1024;

// Per tile of kScanTile positions, the count of selected regions.  Also
// clears the top-K histograms, which this step's selection has used.
__global__ void __launch_bounds__(kScanBlock) sel_count_kernel(const double *err, long long m,
                                                               const unsigned long long *prefix,
                                                               const long long *krem,
                                                               long long *bsum, unsigned *ghist,
                                                               unsigned *gcoarse,
                                                               const int *done) {
  if (stopped(done)) return;
  for (long long i = (long long)blockIdx.x * kScanBlock + threadIdx.x; i < kTopBins + 256;
       i += (long long)gridDim.x * kScanBlock) {
    if (i < kTopBins)
      ghist[i] = 0u;
    else
      gcoarse[i - kTopBins] = 0u;
  }
  const unsigned long long thr = prefix[0];
  const long long tpos = krem[0];
  const long long base = (long long)blockIdx.x * kScanTile;
  long long c = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q * kScanBlock + threadIdx.x;
    if (i < m && selected(err[i], i, thr, tpos)) ++c;
  }
  long long tot;
  (void)block_excl_scan(c, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Each selected region is retired and its position written to parent[j],
// j its rank in position order: the counts of the tiles before this one
// (summed by every block itself) plus the selected positions before it in
// the tile (the tile's kScanItems chunks of 256 in order, within a chunk the
// wavefronts in order, within a wavefront the lanes below).  With rows, the
// block's sums over the regions that stay live.
__global__ void __launch_bounds__(kScanBlock) split_mark_kernel(double *err, const double *I7,
                                                                long long m,
                                                                const unsigned long long *prefix,
                                                                const long long *krem,
                                                                const long long *bsum,
                                                                long long *parent, long long K,
                                                                CRows rows, const int *done) {
  if (stopped(done)) return;
  __shared__ int cnt[kScanItems][kScanBlock / 64];
  const unsigned long long thr = prefix[0];
  const long long tpos = krem[0];
  const long long base = (long long)blockIdx.x * kScanTile;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  long long before = 0;
  for (long long q = threadIdx.x; q < blockIdx.x; q += kScanBlock) before += bsum[q];
  bool f[kScanItems];
  unsigned long long bal[kScanItems];
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q * kScanBlock + threadIdx.x;
    f[q] = false;
    if (i < m) {
      const double e = err[i];
      f[q] = selected(e, i, thr, tpos);
      if (!f[q] && !retired(e)) {
        a += I7[i];
        b += e;
      }
    }
    bal[q] = __ballot(f[q]);
    if (lane == 0) cnt[q][w] = __popcll(bal[q]);
  }
  long long rank;
  (void)block_excl_scan(before, &rank);  // (also orders cnt's writes before the reads)
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    long long pre = 0, all = 0;
#pragma unroll
    for (int v = 0; v < kScanBlock / 64; ++v) {
      if (v < w) pre += cnt[q][v];
      all += cnt[q][v];
    }
    const long long j = rank + pre + __popcll(bal[q] & below);
    if (f[q] && j < K) {  // (exactly K are selected)
      const long long i = base + q * kScanBlock + threadIdx.x;
      parent[j] = i;
      err[i] = -1.0;
    }
    rank += all;
  }
  put_row(rows, a, b);
}

// top-K by a 16-bit first digit ------------------------------------------------
//
// The K largest keys, ties to the lower position, in three launches: the
// histogram of the keys' top 16 bits (sign, exponent and 4 mantissa bits of
// the error) and of their top 8 bits; the digit that holds the K-th key (the
// 8-bit digit first, then the 16-bit one within it, found by every block)
// and the keys and positions of that digit's regions gathered; the exact
// K-th (key, position) among them.

__device__ __forceinline__ long long block_excl_scan_1024(long long v, long long *total) {
  __shared__ long long wtot[kTopThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  long long incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  long long off = 0, tot = 0;
  for (int q = 0; q < kTopThreads / 64; ++q) {
    if (q < w) off += wtot[q];
    tot += wtot[q];
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

// Among nb = 256 * PER digit counts, thread t of 1024 holding the PER
// counts of digits nb - 1 - (PER t + q), q = 0 .. PER - 1 (from the top
// digit down; threads past nb hold none): the digit where the running count
// reaches `need', the need left within it, and its count.
template <int PER>
__device__ __forceinline__ void pick_digit(const long long (&c)[PER], long long need, int nb,
                                           int *dg, long long *left, long long *count) {
  __shared__ int s_dg;
  __shared__ long long s_left, s_cnt;
  const int t = threadIdx.x;
  if (t == 0) {  // (not kept while need <= the total, as it always is)
    s_dg = 0;
    s_left = 1;
    s_cnt = 1;
  }
  long long sum = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) sum += c[q];
  long long tot;
  long long above = block_excl_scan_1024(sum, &tot);
  if (above < need && above + sum >= need) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      if (above + c[q] >= need) {
        s_dg = nb - 1 - (PER * t + q);
        s_left = need - above;
        s_cnt = c[q];
        break;
      }
      above += c[q];
    }
  }
  __syncthreads();
  *dg = s_dg;
  *left = s_left;
  *count = s_cnt;
  __syncthreads();
}

// Per block a histogram of 16-bit counters in LDS (two to a 32-bit word: a
// block sees fewer than 2^16 keys, so a half never carries into the other),
// added into the global 16-bit-digit histogram and its 8-bit-digit one.
// Opens the step (open) and clears the candidate count.
__global__ void __launch_bounds__(kTopThreads) topk_hist_kernel(const double *err, long long m,
                                                                unsigned *ghist,
                                                                unsigned *gcoarse,
                                                                unsigned long long *cnt,
                                                                CRows open, int *done) {
  if (stopped(done) || !open_step(open, done)) return;
  extern __shared__ unsigned lh[];  // kTopBins / 2 words, then 256 coarse counters
  unsigned *lc = lh + kTopBins / 2;
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[0] = 0ull;
  for (int q = threadIdx.x; q < kTopBins / 2 + 256; q += kTopThreads) lh[q] = 0u;
  __syncthreads();
  for (long long i = (long long)blockIdx.x * kTopThreads + threadIdx.x; i < m;
       i += (long long)gridDim.x * kTopThreads) {
    const unsigned b = (unsigned)(key_of(err[i]) >> 48);
    atomicAdd(&lh[b >> 1], 1u << ((b & 1u) << 4));
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kTopBins / 2; q += kTopThreads) {
    const unsigned w = lh[q], lo = w & 0xFFFFu, hi = w >> 16;
    if (lo) atomicAdd(&ghist[2 * q], lo);
    if (hi) atomicAdd(&ghist[2 * q + 1], hi);
    if (w) atomicAdd(&lc[q >> 7], lo + hi);  // words q hold digits 2q, 2q + 1
  }
  __syncthreads();
  if (threadIdx.x < 256 && lc[threadIdx.x]) atomicAdd(&gcoarse[threadIdx.x], lc[threadIdx.x]);
}

// Every block finds the boundary digit (the 8-bit digit holding the K-th
// key, then the 16-bit digit within it) from the histograms; block 0 writes
// it to prefix[0] and the rank wanted within it (from 1) to krem[0].  Then
// the keys and positions of the digit's regions are gathered (any order),
// one atomic add per block and pass.
__global__ void __launch_bounds__(kTopThreads) topk_gather_kernel(const double *err, long long m,
                                                                  long long K,
                                                                  const unsigned *ghist,
                                                                  const unsigned *gcoarse,
                                                                  unsigned long long *prefix,
                                                                  long long *krem,
                                                                  unsigned long long *ckey,
                                                                  long long *cpos,
                                                                  unsigned long long *cnt,
                                                                  const int *done) {
  if (stopped(done)) return;
  __shared__ unsigned wc[kTopThreads / 64];
  __shared__ unsigned long long s_base;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int hi8, lo8;
  long long need, c8;
  {
    const long long c1[1] = {t < 256 ? (long long)gcoarse[255 - t] : 0};
    pick_digit<1>(c1, K, 256, &hi8, &need, &c8);
    const long long c2[1] = {t < 256 ? (long long)ghist[(hi8 << 8) + 255 - t] : 0};
    pick_digit<1>(c2, need, 256, &lo8, &need, &c8);
  }
  // (pick_digit counts digit 255 - t for thread t; threads from 256 on hold 0)
  const unsigned long long dg = (unsigned long long)((hi8 << 8) | lo8);
  if (blockIdx.x == 0 && t == 0) {
    prefix[0] = dg;
    krem[0] = need;
  }
  for (long long i0 = (long long)blockIdx.x * kTopThreads; i0 < m;
       i0 += (long long)gridDim.x * kTopThreads) {
    const long long i = i0 + t;
    const unsigned long long k = i < m ? key_of(err[i]) : 0ull;
    const bool sel = i < m && (k >> 48) == dg;
    const unsigned long long bal = __ballot(sel);
    if (lane == 0) wc[w] = (unsigned)__popcll(bal);
    __syncthreads();
    unsigned off = 0, all = 0;
    for (int q = 0; q < kTopThreads / 64; ++q) {
      if (q < w) off += wc[q];
      all += wc[q];
    }
    if (t == 0 && all) s_base = atomicAdd(cnt, (unsigned long long)all);
    __syncthreads();
    if (sel) {
      const unsigned long long o = s_base + off + __popcll(bal & ((1ull << lane) - 1ull));
      ckey[o] = k;
      cpos[o] = i;
    }
    __syncthreads();  // wc and s_base are rewritten by the next pass
  }
}

// One workgroup: among the gathered regions, the one of rank krem[0] (from
// 1) in the order key descending, position ascending: radix passes of 12
// bits over the key's low 48 bits (descending), until at most 1024
// candidates share the bits fixed so far, which then rank themselves
// directly; if all 48 bits get fixed first: when the regions with that key
// are not all taken (a tie across the threshold), passes of 8 bits over the
// positions (ascending), else the largest of their positions.  Its key to
// prefix[0], its position to krem[0].
__global__ void __launch_bounds__(kTopThreads) topk_exact_kernel(const unsigned long long *ckey,
                                                                 const long long *cpos,
                                                                 const unsigned long long *cnt,
                                                                 unsigned long long *prefix,
                                                                 long long *krem,
                                                                 const int *done) {
  if (stopped(done)) return;
  __shared__ unsigned h[4096];
  __shared__ unsigned long long s_max;
  const int t = threadIdx.x;
  const unsigned long long dg = prefix[0];
  const long long mc = (long long)cnt[0];
  long long need = krem[0], group = 0;
  unsigned long long pre = dg << 48, mask = 0xFFFFull << 48;  // key bits fixed so far
  int dig;
  // up to kExactReg keys per thread stay in registers across the passes (the
  // padding ~0 has top digit 0xFFFF, which no live key has: the sign bit of
  // a live error is clear)
  constexpr int kExactReg = 16;
  constexpr long long kDirect = kTopThreads;  // candidates ranked directly
  const bool inreg = mc <= (long long)kExactReg * kTopThreads;
  unsigned long long kr[kExactReg];
#pragma unroll
  for (int q = 0; q < kExactReg; ++q) {
    const long long i = t + (long long)q * kTopThreads;
    kr[q] = inreg && i < mc ? ckey[i] : ~0ull;
  }
  for (int shift = 36; shift >= 0; shift -= 12) {
    for (int q = t; q < 4096; q += kTopThreads) h[q] = 0u;
    __syncthreads();
    if (inreg) {
#pragma unroll
      for (int q = 0; q < kExactReg; ++q)
        if ((kr[q] & mask) == pre) atomicAdd(&h[(kr[q] >> shift) & 4095ull], 1u);
    } else {
      for (long long i = t; i < mc; i += kTopThreads) {
        const unsigned long long k = ckey[i];
        if ((k & mask) == pre) atomicAdd(&h[(k >> shift) & 4095ull], 1u);
      }
    }
    __syncthreads();
    long long c4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) c4[q] = h[4095 - (4 * t + q)];
    pick_digit<4>(c4, need, 4096, &dig, &need, &group);
    pre |= (unsigned long long)dig << shift;
    mask |= 4095ull << shift;
    if (group <= kDirect) break;  // (group is the same in every thread)
  }
  unsigned long long tpos;
  if (group <= kDirect) {
    // few candidates left with the bits fixed so far: each takes its own
    // rank among them directly, (key desc, position asc), and the one of
    // rank need - 1 is the threshold
    __shared__ unsigned long long gk[kDirect];
    __shared__ long long gp[kDirect];
    __shared__ int gcnt;
    __shared__ unsigned long long s_key;
    __shared__ long long s_pos;
    if (t == 0) gcnt = 0;
    __syncthreads();
    if (inreg) {
#pragma unroll
      for (int q = 0; q < kExactReg; ++q)
        if ((kr[q] & mask) == pre) {
          const int o = atomicAdd(&gcnt, 1);
          gk[o] = kr[q];
          gp[o] = cpos[t + (long long)q * kTopThreads];
        }
    } else {
      for (long long i = t; i < mc; i += kTopThreads) {
        const unsigned long long k = ckey[i];
        if ((k & mask) == pre) {
          const int o = atomicAdd(&gcnt, 1);
          gk[o] = k;
          gp[o] = cpos[i];
        }
      }
    }
    __syncthreads();
    const int c = gcnt;
    if (t < c) {
      const unsigned long long mk = gk[t];
      const long long mp = gp[t];
      long long r = 0;
      for (int i = 0; i < c; ++i) r += gk[i] > mk || (gk[i] == mk && gp[i] < mp);
      if (r == need - 1) {
        s_key = mk;
        s_pos = mp;
      }
    }
    __syncthreads();
    pre = s_key;
    tpos = (unsigned long long)s_pos;
  } else if (need == group) {  // every region with the threshold key is taken
    if (t == 0) s_max = 0ull;
    __syncthreads();
    unsigned long long mx = 0ull;
    if (inreg) {
#pragma unroll
      for (int q = 0; q < kExactReg; ++q)
        if (kr[q] == pre) mx = max(mx, (unsigned long long)cpos[t + (long long)q * kTopThreads]);
    } else {
      for (long long i = t; i < mc; i += kTopThreads)
        if (ckey[i] == pre) mx = max(mx, (unsigned long long)cpos[i]);
    }
    atomicMax(&s_max, mx);
    __syncthreads();
    tpos = s_max;
  } else {
    // positions are below 2^32 (a store of 2^32 regions would need over
    // 500 GB); thread t counts position digit t, which pick_digit sees as
    // digit 255 - t
    unsigned long long ppre = 0ull, pmask = 0xFFFFFFFF00000000ull;
    long long gc;
    for (int shift = 24; shift >= 0; shift -= 8) {
      if (t < 256) h[t] = 0u;
      __syncthreads();
      for (long long i = t; i < mc; i += kTopThreads) {
        const unsigned long long p = (unsigned long long)cpos[i];
        if (ckey[i] == pre && (p & pmask) == ppre) atomicAdd(&h[(p >> shift) & 255ull], 1u);
      }
      __syncthreads();
      const long long c1[1] = {t < 256 ? (long long)h[t] : 0};
      pick_digit<1>(c1, need, 256, &dig, &need, &gc);
      ppre |= (unsigned long long)(255 - dig) << shift;
      pmask |= 255ull << shift;
    }
    tpos = ppre;
  }
  if (t == 0) {
    prefix[0] = pre;
    krem[0] = (long long)tpos;
  }
}

// totals ---------------------------------------------------------------------

// Sums of I7 and err over the live regions among positions [0, m), per tile
// in a fixed order.
__global__ void __launch_bounds__(kScanBlock) totals_partial_kernel(const double *I7,
                                                                    const double *err,
                                                                    long long m, double *part,
                                                                    const int *done) {
  if (stopped(done)) return;
  const long long base = (long long)blockIdx.x * kScanTile;
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q * kScanBlock + threadIdx.x;
    if (i < m) {
      const double e = err[i];
      if (!retired(e)) {
        a += I7[i];
        b += e;
      }
    }
  }
  const double2 t = block_sum2(a, b);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = t.x;
    part[gridDim.x + blockIdx.x] = t.y;
  }
}

// One workgroup: the tiles' sums in tile order into out[0..1].
__global__ void __launch_bounds__(kScanBlock) totals_final_kernel(const double *part, long long nb,
                                                                  double *out, const int *done) {
  if (stopped(done)) return;
  double x = 0.0, y = 0.0;
  for (long long i = threadIdx.x; i < nb; i += kScanBlock) {
    x += part[i];
    y += part[nb + i];
  }
  const double2 T = block_sum2(x, y);
  if (threadIdx.x == 0) {
    out[0] = T.x;
    out[1] = T.y;
  }
}

// ---------------------------------------------------------------------------
// launchers

long long scratch_blocks(long long n) { return (n + kScanTile - 1) / kScanTile; }
long long split_rows(long long m) { return scratch_blocks(m); }
long long step_rows(long long cap) {
  return scratch_blocks(cap) + std::max<long long>((cap + 63) / 64, kWaveRuleBlocks);
}

template <int FAM, int D>
static void launch_rule_lane_dd(const RuleArgs &A, unsigned grid, bool one_lane, hipStream_t s) {
  if (one_lane)
    hipLaunchKernelGGL((gm_rule_lane1_kernel<FAM, D>), dim3(grid), dim3(256), 0, s, A);
  else
    hipLaunchKernelGGL((gm_rule_lane_kernel<FAM, D>), dim3(grid), dim3(256), 0, s, A);
}

template <int FAM>
static void launch_rule_lane_d(const RuleArgs &A, unsigned grid, bool one_lane, hipStream_t s) {
  switch (A.one.ndim) {
    case 2: launch_rule_lane_dd<FAM, 2>(A, grid, one_lane, s); break;
    case 3: launch_rule_lane_dd<FAM, 3>(A, grid, one_lane, s); break;
    case 4: launch_rule_lane_dd<FAM, 4>(A, grid, one_lane, s); break;
    case 5: launch_rule_lane_dd<FAM, 5>(A, grid, one_lane, s); break;
    case 6: launch_rule_lane_dd<FAM, 6>(A, grid, one_lane, s); break;
    case 7: launch_rule_lane_dd<FAM, 7>(A, grid, one_lane, s); break;
    default: launch_rule_lane_dd<FAM, 8>(A, grid, one_lane, s); break;
  }
}

hipError_t launch_root_clear(const CRegions &R, int ndim, int *done, hipStream_t s) {
  hipLaunchKernelGGL(cuhre_root_kernel, dim3(1), dim3(64), 0, s, R, ndim, done);
  return hipGetLastError();
}

// A lane per region needs enough regions to fill the device; below that,
// and above 8 dimensions (the registers a lane holds grow with d, and the
// 2^d corners with it), a wavefront per region.
static bool lane_rule(const RuleArgs &A) {
  return A.nseg == 1 && A.one.ndim <= kLaneRuleMaxDim && A.total >= kLaneRuleMinRegions;
}

// From this many regions on, one lane per region fills the device (a wavefront
// per SIMD and more) without the four-way split's combine.
static bool one_lane_rule(const RuleArgs &A) { return A.total >= kOneLaneRuleMinRegions; }

long long rule_blocks(const RuleArgs &A) {
  if (A.total <= 0) return 0;
  if (lane_rule(A)) return one_lane_rule(A) ? (A.total + 255) / 256 : (A.total + 63) / 64;
  return std::min<long long>((A.total + 3) / 4, kWaveRuleBlocks);
}

hipError_t launch_rule(const RuleArgs &A, hipStream_t s) {
  const long long grid = rule_blocks(A);
  if (grid <= 0) return hipSuccess;
  if (lane_rule(A)) {
    const bool one = one_lane_rule(A);
    switch (A.one.family) {
      case GAUSSIAN: launch_rule_lane_d<GAUSSIAN>(A, (unsigned)grid, one, s); break;
      case OSCILLATORY: launch_rule_lane_d<OSCILLATORY>(A, (unsigned)grid, one, s); break;
      case PRODUCT_PEAK: launch_rule_lane_d<PRODUCT_PEAK>(A, (unsigned)grid, one, s); break;
      case CORNER_PEAK: launch_rule_lane_d<CORNER_PEAK>(A, (unsigned)grid, one, s); break;
      default: launch_rule_lane_d<C0>(A, (unsigned)grid, one, s); break;
    }
    return hipGetLastError();
  }
  hipLaunchKernelGGL(gm_rule_kernel, dim3((unsigned)grid), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_select16(const CRegions &R, long long m, long long K, const CScratch &S,
                           hipStream_t s, const CRows *open) {
  // blocks see fewer than 2^16 keys each (the LDS counters are 16-bit)
  const long long per = 32768;
  const int hgrid = (int)std::max<long long>(std::min<long long>(64, (m + kTopThreads - 1) /
                                                                         kTopThreads),
                                             (m + per - 1) / per);
  const CRows none{};
  hipLaunchKernelGGL(topk_hist_kernel, dim3(hgrid), dim3(kTopThreads), (kTopBins / 2 + 256) * 4,
                     s, R.err, m, S.hist16, S.coarse, S.cand_cnt, open ? *open : none, S.done);
  const int ggrid = (int)std::min<long long>(256, (m + kTopThreads - 1) / kTopThreads);
  hipLaunchKernelGGL(topk_gather_kernel, dim3(ggrid), dim3(kTopThreads), 0, s, R.err, m, K,
                     S.hist16, S.coarse, S.prefix, S.krem, S.cand_key, S.cand_pos, S.cand_cnt,
                     (const int *)S.done);
  hipLaunchKernelGGL(topk_exact_kernel, dim3(1), dim3(kTopThreads), 0, s, S.cand_key, S.cand_pos,
                     S.cand_cnt, S.prefix, S.krem, (const int *)S.done);
  return hipGetLastError();
}

hipError_t launch_split(const CRegions &R, long long m, long long K, const CScratch &S,
                        hipStream_t s, const CRows *rows) {
  const long long nb = scratch_blocks(m);
  const CRows none{};
  hipLaunchKernelGGL(sel_count_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, R.err, m,
                     S.prefix, S.krem, S.bsum, S.hist16, S.coarse, (const int *)S.done);
  hipLaunchKernelGGL(split_mark_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, R.err, R.I7,
                     m, S.prefix, S.krem, S.bsum, S.parent, K, rows ? *rows : none,
                     (const int *)S.done);
  return hipGetLastError();
}

hipError_t launch_decide(const CRows &rows, int *done, hipStream_t s) {
  hipLaunchKernelGGL(cuhre_decide_kernel, dim3(1), dim3(256), 0, s, rows, done);
  return hipGetLastError();
}

hipError_t launch_totals(const CRegions &R, long long m, const CScratch &S, double *out,
                         hipStream_t s) {
  const long long nb = scratch_blocks(m);
  hipLaunchKernelGGL(totals_partial_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, R.I7,
                     R.err, m, S.tot, (const int *)S.done);
  hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(kScanBlock), 0, s, S.tot, nb, out,
                     (const int *)S.done);
  return hipGetLastError();
}

hipError_t cuhre_set_kernel_limits() {
  // the top-K histogram keeps 2^16 16-bit counters and 256 32-bit ones in
  // LDS (129 KB)
  return hipFuncSetAttribute((const void *)topk_hist_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (kTopBins / 2 + 256) * 4);
}

}  // namespace ccuba
