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

__global__ void cuhre_root_kernel(CRegions R, int d) {
  const int j = threadIdx.x;
  if (j < d) {
    R.c[j * R.cap] = 0.5;
    R.h[j * R.cap] = 0.5;
  }
  if (j == 0) R.id[0] = 0;
}

// One integral (A.one), dimension D: one lane per region.
template <int FAM, int D>
__global__ void __launch_bounds__(256) gm_rule_lane_kernel(RuleArgs A) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= A.total) return;
  rule_region_lane<FAM, D>(A, A.one, A.one.first + g);
}

__global__ void __launch_bounds__(256) gm_rule_kernel(RuleArgs A) {
  __shared__ double sc[4][kMaxDim], sh[4][kMaxDim];
  __shared__ double sf[4][4 * kMaxDim + 1];
  __shared__ double sx[4][2 * kMaxDim];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long g = (long long)blockIdx.x * 4 + w;
  if (g >= A.total) return;  // only whole waves leave; no block barrier below
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

// count of flag-like predicate per scan tile
__global__ void __launch_bounds__(kScanBlock) eq_count_kernel(const double *err, long long n,
                                                              const unsigned long long *prefix,
                                                              long long *bsum) {
  const unsigned long long thr = prefix[0];
  const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  long long c = 0;
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q;
    if (i < n && key_of(err[i]) == thr) ++c;
  }
  long long tot;
  (void)block_excl_scan(c, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanBlock) flag_count_kernel(const int *flag, long long n,
                                                                long long *bsum) {
  const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  long long c = 0;
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q;
    if (i < n && flag[i]) ++c;
  }
  long long tot;
  (void)block_excl_scan(c, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of nb block sums in one workgroup (sequential carry over
// chunks of 256)
__global__ void __launch_bounds__(kScanBlock) scan_bsum_kernel(long long *bsum, long long nb) {
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

// radix select ----------------------------------------------------------------

__global__ void sel_init_kernel(unsigned long long *prefix, long long *krem, unsigned *hist,
                                long long K) {
  prefix[0] = 0ull;
  prefix[1] = 0ull;
  krem[0] = K;
  krem[1] = 0;
  for (int q = threadIdx.x; q < 256; q += blockDim.x) hist[q] = 0u;
}

__global__ void __launch_bounds__(256) sel_hist_kernel(const double *err, long long n,
                                                       const unsigned long long *prefix,
                                                       unsigned *hist, int shift) {
  __shared__ unsigned lh[256];
  lh[threadIdx.x] = 0u;
  __syncthreads();
  const unsigned long long pre = prefix[0], mask = prefix[1];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long k = key_of(err[i]);
    if ((k & mask) == pre) atomicAdd(&lh[(k >> shift) & 255ull], 1u);
  }
  __syncthreads();
  if (lh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], lh[threadIdx.x]);
}

// One workgroup of 256 threads: the digit of the K-th largest key among the
// keys with the current prefix, from the pass's histogram.  Thread t holds
// digit 255 - t; an inclusive scan over threads gives, for each digit, the
// count of keys at or above it.  The digit is the top one where that count
// reaches the remaining need, or 0 if none does; the need left within it is
// the need less the keys above it.
__global__ void __launch_bounds__(256) sel_pick_kernel(unsigned long long *prefix,
                                                       long long *krem, unsigned *hist,
                                                       int shift) {
  __shared__ long long wsum[4];
  __shared__ int s_dg;
  __shared__ long long s_need;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int dg = 255 - t;
  const long long need = krem[0];
  const long long c = hist[dg];
  hist[dg] = 0u;  // ready for the next pass
  long long incl = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  for (int q = 0; q < w; ++q) incl += wsum[q];
  const long long excl = incl - c;  // keys above this digit
  if (excl < need && (incl >= need || dg == 0)) {  // exactly one thread
    s_dg = dg;
    s_need = need - excl;
  }
  __syncthreads();
  if (t == 0) {
    krem[0] = s_need;
    prefix[0] |= (unsigned long long)s_dg << shift;
    prefix[1] |= 255ull << shift;
  }
}

// flag[i] = key > threshold, or key == threshold and among the first krem
// such positions
__global__ void __launch_bounds__(kScanBlock) sel_flag_kernel(const double *err, long long n,
                                                              const unsigned long long *prefix,
                                                              const long long *krem,
                                                              const long long *bsum, int *flag) {
  const unsigned long long thr = prefix[0];
  const long long take = krem[0];
  const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  unsigned long long k[kScanItems];
  long long c = 0;
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q;
    k[q] = i < n ? key_of(err[i]) : 0ull;
    if (i < n && k[q] == thr) ++c;
  }
  long long tot;
  long long rank = bsum[blockIdx.x] + block_excl_scan(c, &tot);
  for (int q = 0; q < kScanItems; ++q) {
    const long long i = base + q;
    if (i >= n) break;
    int f = 0;
    if (k[q] > thr) {
      f = 1;
    } else if (k[q] == thr) {
      f = rank < take;
      ++rank;
    }
    flag[i] = f;
  }
}

// scatter: keep unselected regions in order, append the halves of selected
__global__ void __launch_bounds__(kScanBlock) split_kernel(CRegions src, CRegions dst, int d,
                                                           long long n, long long K,
                                                           long long next_id, int all,
                                                           const int *flag,
                                                           const long long *bsum) {
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

// totals ---------------------------------------------------------------------

__global__ void __launch_bounds__(kScanBlock) totals_partial_kernel(const double *I7,
                                                                    const double *err,
                                                                    long long n, double *part,
                                                                    long long nb) {
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
  hipLaunchKernelGGL(cuhre_root_kernel, dim3(1), dim3(64), 0, s, R, ndim);
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

hipError_t launch_select(const CRegions &R, long long n, long long K, const CScratch &S,
                         hipStream_t s) {
  const long long nb = scratch_blocks(n);
  hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(256), 0, s, S.prefix, S.krem, S.hist, K);
  const int hgrid = (int)std::min<long long>(4096, (n + 255) / 256);
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    hipLaunchKernelGGL(sel_hist_kernel, dim3(hgrid), dim3(256), 0, s, R.err, n, S.prefix, S.hist,
                       shift);
    hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(256), 0, s, S.prefix, S.krem, S.hist,
                       shift);
  }
  hipLaunchKernelGGL(eq_count_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, R.err, n,
                     S.prefix, S.bsum);
  hipLaunchKernelGGL(scan_bsum_kernel, dim3(1), dim3(kScanBlock), 0, s, S.bsum, nb);
  hipLaunchKernelGGL(sel_flag_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, R.err, n,
                     S.prefix, S.krem, S.bsum, S.flag);
  return hipGetLastError();
}

hipError_t launch_split(const CRegions &src, const CRegions &dst, int ndim, long long n,
                        long long K, long long next_id, bool all, const CScratch &S,
                        hipStream_t s) {
  const long long nb = scratch_blocks(n);
  if (!all) {
    hipLaunchKernelGGL(flag_count_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, S.flag, n,
                       S.bsum);
    hipLaunchKernelGGL(scan_bsum_kernel, dim3(1), dim3(kScanBlock), 0, s, S.bsum, nb);
  }
  hipLaunchKernelGGL(split_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, src, dst, ndim, n,
                     K, next_id, all ? 1 : 0, S.flag, S.bsum);
  return hipGetLastError();
}

hipError_t launch_totals(const CRegions &R, long long n, const CScratch &S, double *out,
                         hipStream_t s) {
  const long long nb = scratch_blocks(n);
  hipLaunchKernelGGL(totals_partial_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, R.I7,
                     R.err, n, S.tot, nb);
  hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(kScanBlock), 0, s, S.tot, nb, out);
  return hipGetLastError();
}

hipError_t cuhre_set_kernel_limits() { return hipSuccess; }

}  // namespace ccuba
