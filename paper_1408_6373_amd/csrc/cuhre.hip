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
// a9 (region step): radix select of the K largest errors (8 passes of 8
//    bits over the IEEE bit pattern, which orders non-negative doubles;
//    ties go to the lower position, i.e. the lower region id), then one
//    scan-and-scatter pass that keeps the unselected regions in order and
//    writes the two halves of every selected region at the end, and a
//    fixed-order reduction for the totals.  No step waits on another block.
#include "cuhre.h"
#include "genz.h"

namespace ccuba {

namespace {

constexpr int kLaneRuleMaxDim = 8;          // lane-per-region rule up to this d
constexpr long long kLaneRuleMinRegions = 16384;  // and from this many regions on
constexpr int kScanItems = 4;
constexpr int kScanBlock = 256;
constexpr int kScanTile = kScanItems * kScanBlock;  // elements per scan block

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ unsigned long long key_of(double e) {
  return (unsigned long long)__double_as_longlong(e);
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

template <int FAM>
__device__ void rule_region(const RuleArgs &A, const CSeg &S, long long r, int w, int lane,
                            double (*sc)[kMaxDim], double (*sh)[kMaxDim],
                            double (*sf)[4 * kMaxDim + 1], double (*sx)[2 * kMaxDim]) {
  const int d = S.ndim;
  const long long cap = S.regs.cap;
  if (lane < d) {
    sc[w][lane] = S.regs.c[lane * cap + r];
    sh[w][lane] = S.regs.h[lane * cap + r];
  }
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
  }
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

template <int FAM, int D>
__device__ void rule_region_lane(const RuleArgs &A, const CSeg &S, long long r) {
  const long long cap = S.regs.cap;
  double c[D], h[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    c[j] = S.regs.c[j * cap + r];
    h[j] = S.regs.h[j * cap + r];
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
}

}  // namespace

__global__ void cuhre_root_kernel(CRegions R, int d, int *done) {
  const int j = threadIdx.x;
  if (j < d) {
    R.c[j * R.cap] = 0.5;
    R.h[j * R.cap] = 0.5;
  }
  if (j == 0) {
    R.id[0] = 0;
    if (done) *done = 0;
  }
}

// a run's launches do nothing once its stop flag is set
__device__ __forceinline__ bool stopped(const int *done) { return done && *done != 0; }

// One integral (A.one), dimension D: one lane per region.
template <int FAM, int D>
__global__ void __launch_bounds__(256) gm_rule_lane_kernel(RuleArgs A) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= A.total || stopped(A.done)) return;
  rule_region_lane<FAM, D>(A, A.one, A.one.first + g);
}

__global__ void __launch_bounds__(256) gm_rule_kernel(RuleArgs A) {
  __shared__ double sc[4][kMaxDim], sh[4][kMaxDim];
  __shared__ double sf[4][4 * kMaxDim + 1];
  __shared__ double sx[4][2 * kMaxDim];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long g = (long long)blockIdx.x * 4 + w;
  if (g >= A.total || stopped(A.done)) return;  // only whole waves leave; no block barrier below
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
  switch (S.family) {
    case GAUSSIAN: rule_region<GAUSSIAN>(A, S, r, w, lane, sc, sh, sf, sx); break;
    case OSCILLATORY: rule_region<OSCILLATORY>(A, S, r, w, lane, sc, sh, sf, sx); break;
    case PRODUCT_PEAK: rule_region<PRODUCT_PEAK>(A, S, r, w, lane, sc, sh, sf, sx); break;
    case CORNER_PEAK: rule_region<CORNER_PEAK>(A, S, r, w, lane, sc, sh, sf, sx); break;
    default: rule_region<C0>(A, S, r, w, lane, sc, sh, sf, sx); break;
  }
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

// exclusive scan of nb block sums in one workgroup (sequential carry over
// chunks of 256)
__global__ void __launch_bounds__(kScanBlock) scan_bsum_kernel(long long *bsum, long long nb,
                                                               const int *done) {
  if (stopped(done)) return;
  __shared__ long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (long long c0 = 0; c0 < nb; c0 += kScanBlock) {
    const long long i = c0 + threadIdx.x;
    const long long v = i < nb ? bsum[i] : 0;
    long long tot;
    const long long ex = block_excl_scan(v, &tot);
    const long long cr = carry;
    if (i < nb) bsum[i] = cr + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry = cr + tot;
    __syncthreads();
  }
}

// scatter: keep unselected regions in order, append the halves of selected
__global__ void __launch_bounds__(kScanBlock) split_kernel(CRegions src, CRegions dst, int d,
                                                           long long n, long long K,
                                                           long long next_id, int all,
                                                           const int *flag,
                                                           const long long *bsum,
                                                           const int *done) {
  if (stopped(done)) return;
  const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int f[kScanItems];
  long long c = 0;
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q;
    f[q] = i < n ? (all ? 1 : flag[i]) : 0;
    c += f[q];
  }
  long long tot;
  long long rank = (all ? (long long)blockIdx.x * kScanTile : bsum[blockIdx.x]) +
                   block_excl_scan(c, &tot);
  const long long cbase = n - K;
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q;
    if (i >= n) break;
    if (!f[q]) {
      const long long o = i - rank;
      for (int j = 0; j < d; ++j) {
        dst.c[j * dst.cap + o] = src.c[j * src.cap + i];
        dst.h[j * dst.cap + o] = src.h[j * src.cap + i];
      }
      dst.I7[o] = src.I7[i];
      dst.I5[o] = src.I5[i];
      dst.err[o] = src.err[i];
      dst.axis[o] = src.axis[i];
      dst.id[o] = src.id[i];
    } else {
      const long long o0 = cbase + 2 * rank, o1 = o0 + 1;
      const int s = src.axis[i];
      for (int j = 0; j < d; ++j) {
        const double cj = src.c[j * src.cap + i], hj = src.h[j * src.cap + i];
        if (j == s) {
          const double hh = hj / 2.0;
          dst.c[j * dst.cap + o0] = cj - hh;
          dst.c[j * dst.cap + o1] = cj + hh;
          dst.h[j * dst.cap + o0] = hh;
          dst.h[j * dst.cap + o1] = hh;
        } else {
          dst.c[j * dst.cap + o0] = cj;
          dst.c[j * dst.cap + o1] = cj;
          dst.h[j * dst.cap + o0] = hj;
          dst.h[j * dst.cap + o1] = hj;
        }
      }
      dst.id[o0] = next_id + 2 * rank;
      dst.id[o1] = next_id + 2 * rank + 1;
      ++rank;
    }
  }
}

// top-K by a 16-bit first digit ------------------------------------------------
//
// The same selection as the radix select above (the K largest keys, ties to
// the lower position), in four launches instead of nineteen: the histogram of
// the keys' top 16 bits (sign, exponent and 4 mantissa bits of the error),
// the digit that holds the K-th key, the keys and positions of that digit's
// regions gathered, and the exact K-th (key, position) among them.

constexpr int kTopBins = 1 << 16;
constexpr int kTopThreads = 1024;
constexpr int kTopPerThread = kTopBins / kTopThreads;  // 64

// Per block a histogram of 16-bit counters in LDS (two to a 32-bit word: a
// block sees fewer than 2^16 keys, so a half never carries into the other),
// added into the global histogram.
__global__ void __launch_bounds__(kTopThreads) topk_hist_kernel(const double *err, long long n,
                                                                unsigned *ghist,
                                                                const int *done) {
  if (stopped(done)) return;
  extern __shared__ unsigned lh[];  // kTopBins / 2 words
  for (int q = threadIdx.x; q < kTopBins / 2; q += kTopThreads) lh[q] = 0u;
  __syncthreads();
  for (long long i = (long long)blockIdx.x * kTopThreads + threadIdx.x; i < n;
       i += (long long)gridDim.x * kTopThreads) {
    const unsigned b = (unsigned)(key_of(err[i]) >> 48);
    atomicAdd(&lh[b >> 1], 1u << ((b & 1u) << 4));
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kTopBins / 2; q += kTopThreads) {
    const unsigned w = lh[q];
    if (w & 0xFFFFu) atomicAdd(&ghist[2 * q], w & 0xFFFFu);
    if (w >> 16) atomicAdd(&ghist[2 * q + 1], w >> 16);
  }
}

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

// One workgroup: the digit that holds the K-th largest key (thread t holds
// the 64 digits below 2^16 - 64 t, in descending order), the rank wanted
// within it, and the histogram cleared for the next use.
__global__ void __launch_bounds__(kTopThreads) topk_pick_kernel(unsigned *ghist, long long K,
                                                                unsigned long long *prefix,
                                                                long long *krem,
                                                                unsigned long long *cnt,
                                                                const int *done) {
  if (stopped(done)) return;
  const int t = threadIdx.x;
  unsigned c[kTopPerThread];
  long long sum = 0;
#pragma unroll
  for (int q = 0; q < kTopPerThread; ++q) {
    const int b = kTopBins - 1 - (kTopPerThread * t + q);
    c[q] = ghist[b];
    sum += c[q];
  }
#pragma unroll
  for (int q = 0; q < kTopPerThread; ++q) ghist[kTopBins - 1 - (kTopPerThread * t + q)] = 0u;
  long long tot;
  long long acc = block_excl_scan_1024(sum, &tot);  // keys in digits above this thread's
  if (acc < K && acc + sum >= K) {  // exactly one thread
#pragma unroll
    for (int q = 0; q < kTopPerThread; ++q) {
      if (acc + (long long)c[q] >= K) {
        prefix[0] = (unsigned long long)(kTopBins - 1 - (kTopPerThread * t + q));
        krem[0] = K - acc;  // rank (from 1) wanted within the digit
        cnt[0] = 0ull;
        break;
      }
      acc += c[q];
    }
  }
}

// The keys and positions of the boundary digit's regions (any order), one
// atomic add per wavefront.
__global__ void __launch_bounds__(256) topk_gather_kernel(const double *err, long long n,
                                                          const unsigned long long *prefix,
                                                          unsigned long long *ckey,
                                                          long long *cpos,
                                                          unsigned long long *cnt,
                                                          const int *done) {
  if (stopped(done)) return;
  const unsigned long long dg = prefix[0];
  const int lane = threadIdx.x & 63;
  for (long long i0 = (long long)blockIdx.x * 256; i0 < n; i0 += (long long)gridDim.x * 256) {
    const long long i = i0 + threadIdx.x;
    const unsigned long long k = i < n ? key_of(err[i]) : 0ull;
    const bool m = i < n && (k >> 48) == dg;
    const unsigned long long bal = __ballot(m);
    if (bal == 0ull) continue;
    unsigned long long base = 0;
    if (lane == (int)__ffsll((long long)bal) - 1) base = atomicAdd(cnt, (unsigned long long)__popcll(bal));
    base = __shfl(base, __ffsll((long long)bal) - 1, 64);
    if (m) {
      const unsigned long long o = base + __popcll(bal & ((1ull << lane) - 1ull));
      ckey[o] = k;
      cpos[o] = i;
    }
  }
}

// One workgroup: among the gathered regions, the one of rank krem[0] (from 1)
// in the order key descending, position ascending, by radix passes of 8 bits
// over the key's low 48 bits (descending) and then over the position's low
// 32 bits (ascending).  Writes its key to prefix[0] and its position to
// krem[0].
__global__ void __launch_bounds__(kTopThreads) topk_exact_kernel(const unsigned long long *ckey,
                                                                 const long long *cpos,
                                                                 const unsigned long long *cnt,
                                                                 unsigned long long *prefix,
                                                                 long long *krem,
                                                                 const int *done) {
  if (stopped(done)) return;
  __shared__ unsigned h[256];
  __shared__ long long s_need;
  __shared__ int s_dg;
  const int t = threadIdx.x;
  const long long m = (long long)cnt[0];
  long long need = krem[0];
  unsigned long long pre = prefix[0] << 48, mask = 0xFFFFull << 48;  // key bits fixed so far
  // key passes: descending digits
  for (int shift = 40; shift >= 0; shift -= 8) {
    if (t < 256) h[t] = 0u;
    __syncthreads();
    for (long long i = t; i < m; i += kTopThreads) {
      const unsigned long long k = ckey[i];
      if ((k & mask) == pre) atomicAdd(&h[(k >> shift) & 255ull], 1u);
    }
    __syncthreads();
    if (t < 64) {  // one wavefront scans the 256 counts from the top digit down
      unsigned c4[4];
      long long s4 = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c4[q] = h[255 - (4 * t + q)];
        s4 += c4[q];
      }
      long long incl = s4;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const long long v = __shfl_up(incl, o, 64);
        if (t >= o) incl += v;
      }
      long long acc = incl - s4;
      if (acc < need && incl >= need) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (acc + (long long)c4[q] >= need) {
            s_dg = 255 - (4 * t + q);
            s_need = need - acc;
            break;
          }
          acc += c4[q];
        }
      }
    }
    __syncthreads();
    need = s_need;
    pre |= (unsigned long long)s_dg << shift;
    mask |= 255ull << shift;
    __syncthreads();
  }
  // position passes among the regions with the threshold key: ascending
  // (positions are below 2^32: a region store of 2^32 regions would need
  // over 500 GB)
  unsigned long long ppre = 0ull, pmask = 0xFFFFFFFF00000000ull;
  for (int shift = 24; shift >= 0; shift -= 8) {
    if (t < 256) h[t] = 0u;
    __syncthreads();
    for (long long i = t; i < m; i += kTopThreads) {
      const unsigned long long p = (unsigned long long)cpos[i];
      if (ckey[i] == pre && (p & pmask) == ppre) atomicAdd(&h[(p >> shift) & 255ull], 1u);
    }
    __syncthreads();
    if (t < 64) {  // from the lowest digit up
      unsigned c4[4];
      long long s4 = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c4[q] = h[4 * t + q];
        s4 += c4[q];
      }
      long long incl = s4;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const long long v = __shfl_up(incl, o, 64);
        if (t >= o) incl += v;
      }
      long long acc = incl - s4;
      if (acc < need && incl >= need) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (acc + (long long)c4[q] >= need) {
            s_dg = 4 * t + q;
            s_need = need - acc;
            break;
          }
          acc += c4[q];
        }
      }
    }
    __syncthreads();
    need = s_need;
    ppre |= (unsigned long long)s_dg << shift;
    pmask |= 255ull << shift;
    __syncthreads();
  }
  if (t == 0) {
    prefix[0] = pre;
    krem[0] = (long long)ppre;
  }
}

// flag[i] = (key, position) at or above the threshold in the selection order,
// and the per-tile counts of launch_split
__global__ void __launch_bounds__(kScanBlock) thr_flag_count_kernel(const double *err, long long n,
                                                                    const unsigned long long *prefix,
                                                                    const long long *krem,
                                                                    int *flag, long long *bsum,
                                                                    const int *done) {
  if (stopped(done)) return;
  const unsigned long long thr = prefix[0];
  const long long tpos = krem[0];
  const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  long long c = 0;
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q;
    if (i < n) {
      const unsigned long long k = key_of(err[i]);
      const int f = k > thr || (k == thr && i <= tpos);
      flag[i] = f;
      c += f;
    }
  }
  long long tot;
  (void)block_excl_scan(c, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// totals ---------------------------------------------------------------------

__global__ void __launch_bounds__(kScanBlock) totals_partial_kernel(const double *I7,
                                                                    const double *err,
                                                                    long long n, double *part,
                                                                    long long nb,
                                                                    const int *done) {
  if (stopped(done)) return;
  __shared__ double s7[kScanBlock], se[kScanBlock];
  const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  double a = 0.0, b = 0.0;
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q;
    if (i < n) {
      a += I7[i];
      b += err[i];
    }
  }
  s7[threadIdx.x] = a;
  se[threadIdx.x] = b;
  __syncthreads();
  for (int o = kScanBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s7[threadIdx.x] += s7[threadIdx.x + o];
      se[threadIdx.x] += se[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s7[0];
    part[nb + blockIdx.x] = se[0];
  }
}

__global__ void __launch_bounds__(kScanBlock) totals_final_kernel(const double *part, long long nb,
                                                                  double *out) {
  __shared__ double s7[kScanBlock], se[kScanBlock];
  double a = 0.0, b = 0.0;
  for (long long i = threadIdx.x; i < nb; i += kScanBlock) {
    a += part[i];
    b += part[nb + i];
  }
  s7[threadIdx.x] = a;
  se[threadIdx.x] = b;
  __syncthreads();
  for (int o = kScanBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s7[threadIdx.x] += s7[threadIdx.x + o];
      se[threadIdx.x] += se[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s7[0];
    out[1] = se[0];
  }
}

// totals_final, then the stop rule (launch_totals_decide)
__global__ void __launch_bounds__(kScanBlock) totals_decide_kernel(const double *part, long long nb,
                                                                   double *out, int *done,
                                                                   CStop stop) {
  if (stopped(done)) return;
  __shared__ double s7[kScanBlock], se[kScanBlock];
  double a = 0.0, b = 0.0;
  for (long long i = threadIdx.x; i < nb; i += kScanBlock) {
    a += part[i];
    b += part[nb + i];
  }
  s7[threadIdx.x] = a;
  se[threadIdx.x] = b;
  __syncthreads();
  for (int o = kScanBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s7[threadIdx.x] += s7[threadIdx.x + o];
      se[threadIdx.x] += se[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double I = s7[0], E = se[0];
    int code = 0;
    if (!isfinite(I) || !isfinite(E))
      code = 2;
    else if (stop.neval >= stop.mineval && E <= fmax(stop.epsabs, stop.epsrel * fabs(I)))
      code = 1;
    out[0] = I;
    out[1] = E;
    out[2] = (double)code;
    if (code) *done = 1;
  }
}

// ---------------------------------------------------------------------------
// launchers

long long scratch_blocks(long long n) { return (n + kScanTile - 1) / kScanTile; }

template <int FAM>
static void launch_rule_lane_d(const RuleArgs &A, unsigned grid, hipStream_t s) {
  switch (A.one.ndim) {
    case 2: hipLaunchKernelGGL((gm_rule_lane_kernel<FAM, 2>), dim3(grid), dim3(256), 0, s, A); break;
    case 3: hipLaunchKernelGGL((gm_rule_lane_kernel<FAM, 3>), dim3(grid), dim3(256), 0, s, A); break;
    case 4: hipLaunchKernelGGL((gm_rule_lane_kernel<FAM, 4>), dim3(grid), dim3(256), 0, s, A); break;
    case 5: hipLaunchKernelGGL((gm_rule_lane_kernel<FAM, 5>), dim3(grid), dim3(256), 0, s, A); break;
    case 6: hipLaunchKernelGGL((gm_rule_lane_kernel<FAM, 6>), dim3(grid), dim3(256), 0, s, A); break;
    case 7: hipLaunchKernelGGL((gm_rule_lane_kernel<FAM, 7>), dim3(grid), dim3(256), 0, s, A); break;
    default: hipLaunchKernelGGL((gm_rule_lane_kernel<FAM, 8>), dim3(grid), dim3(256), 0, s, A); break;
  }
}

hipError_t launch_root(const CRegions &R, int ndim, hipStream_t s) {
  hipLaunchKernelGGL(cuhre_root_kernel, dim3(1), dim3(64), 0, s, R, ndim, (int *)nullptr);
  return hipGetLastError();
}

hipError_t launch_root_clear(const CRegions &R, int ndim, int *done, hipStream_t s) {
  hipLaunchKernelGGL(cuhre_root_kernel, dim3(1), dim3(64), 0, s, R, ndim, done);
  return hipGetLastError();
}

hipError_t launch_rule(const RuleArgs &A, hipStream_t s) {
  if (A.total <= 0) return hipSuccess;
  // A lane per region needs enough regions to fill the device; below that,
  // and above 8 dimensions (the registers a lane holds grow with d, and the
  // 2^d corners with it), a wavefront per region.
  if (A.nseg == 1 && A.one.ndim <= kLaneRuleMaxDim && A.total >= kLaneRuleMinRegions) {
    const unsigned grid = (unsigned)((A.total + 255) / 256);
    switch (A.one.family) {
      case GAUSSIAN: launch_rule_lane_d<GAUSSIAN>(A, grid, s); break;
      case OSCILLATORY: launch_rule_lane_d<OSCILLATORY>(A, grid, s); break;
      case PRODUCT_PEAK: launch_rule_lane_d<PRODUCT_PEAK>(A, grid, s); break;
      case CORNER_PEAK: launch_rule_lane_d<CORNER_PEAK>(A, grid, s); break;
      default: launch_rule_lane_d<C0>(A, grid, s); break;
    }
    return hipGetLastError();
  }
  const long long grid = (A.total + 3) / 4;
  hipLaunchKernelGGL(gm_rule_kernel, dim3((unsigned)grid), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_select16(const CRegions &R, long long n, long long K, const CScratch &S,
                           hipStream_t s) {
  // blocks see fewer than 2^16 keys each (the LDS counters are 16-bit)
  const long long per = 32768;
  const int hgrid = (int)std::max<long long>(std::min<long long>(256, (n + kTopThreads - 1) /
                                                                          kTopThreads),
                                             (n + per - 1) / per);
  hipLaunchKernelGGL(topk_hist_kernel, dim3(hgrid), dim3(kTopThreads), (kTopBins / 2) * 4, s,
                     R.err, n, S.hist16, (const int *)S.done);
  hipLaunchKernelGGL(topk_pick_kernel, dim3(1), dim3(kTopThreads), 0, s, S.hist16, K, S.prefix,
                     S.krem, S.cand_cnt, (const int *)S.done);
  const int ggrid = (int)std::min<long long>(2048, (n + 255) / 256);
  hipLaunchKernelGGL(topk_gather_kernel, dim3(ggrid), dim3(256), 0, s, R.err, n, S.prefix,
                     S.cand_key, S.cand_pos, S.cand_cnt, (const int *)S.done);
  hipLaunchKernelGGL(topk_exact_kernel, dim3(1), dim3(kTopThreads), 0, s, S.cand_key,
                     S.cand_pos, S.cand_cnt, S.prefix, S.krem, (const int *)S.done);
  return hipGetLastError();
}

hipError_t launch_split(const CRegions &src, const CRegions &dst, int ndim, long long n,
                        long long K, long long next_id, bool all, const CScratch &S,
                        hipStream_t s) {
  const long long nb = scratch_blocks(n);
  if (!all) {
    hipLaunchKernelGGL(thr_flag_count_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, src.err,
                       n, S.prefix, S.krem, S.flag, S.bsum, (const int *)S.done);
    hipLaunchKernelGGL(scan_bsum_kernel, dim3(1), dim3(kScanBlock), 0, s, S.bsum, nb,
                       (const int *)S.done);
  }
  hipLaunchKernelGGL(split_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, src, dst, ndim, n,
                     K, next_id, all ? 1 : 0, S.flag, S.bsum, (const int *)S.done);
  return hipGetLastError();
}

hipError_t launch_totals(const CRegions &R, long long n, const CScratch &S, double *out,
                         hipStream_t s) {
  const long long nb = scratch_blocks(n);
  hipLaunchKernelGGL(totals_partial_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, R.I7,
                     R.err, n, S.tot, nb, (const int *)S.done);
  hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(kScanBlock), 0, s, S.tot, nb, out);
  return hipGetLastError();
}

hipError_t launch_totals_decide(const CRegions &R, long long n, const CScratch &S, double *out,
                                const CStop &stop, hipStream_t s) {
  const long long nb = scratch_blocks(n);
  hipLaunchKernelGGL(totals_partial_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, R.I7,
                     R.err, n, S.tot, nb, (const int *)S.done);
  hipLaunchKernelGGL(totals_decide_kernel, dim3(1), dim3(kScanBlock), 0, s, S.tot, nb, out,
                     S.done, stop);
  return hipGetLastError();
}

hipError_t cuhre_set_kernel_limits() {
  // the top-K histogram keeps 2^16 16-bit counters in LDS (128 KB)
  return hipFuncSetAttribute((const void *)topk_hist_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (kTopBins / 2) * 4);
}

}  // namespace ccuba
