// suave.hip -- Suave's steps on gfx950.
//
// One step of subregion-adaptive Vegas over the regions of one integral:
//   select  the K regions of largest variance (topk: radix select on the
//           variance bits, then a bitonic sort of the K winners by (variance
//           desc, position asc)); one workgroup
//   fluct   per (selected region, dimension, chunk of its stored sample): the
//           two halves' counts, sums and extremes, then the p-th power sums of
//           the deviations from each half's mean (p = flatness), for the L_p
//           fluctuation F_h = (n_h/n) ((1/n_h) sum |v - m_h|^p)^(1/p)
//   split   per selected region: the dimension of least F_0 + F_1, the two
//           children's bounds, their grids (the parent's map restricted to
//           each half along the cut) and the estimates inherited from the
//           parent's sample; one workgroup each
//   sample  DoSample of every child: nnew Philox points through the child's
//           grid (cells staged in LDS), the integrand, v = w V f, the stored
//           (v, side bits) and per-tile sums and v^2 histograms
//   fold    per child: tile sums in tile order, the child's own estimate, its
//           inverse-variance combination with the inherited one, and the
//           refinement of the child's grid (one wavefront per dimension)
//   totals  sums over all regions and the chi^2 probability; one workgroup
// The host reads the totals after each step and sizes the next one.
#include "engine.h"
#include "genz.h"
#include "philox.h"
#include "refine.h"
#include "suave.h"

namespace ccuba {

namespace {

// sum of one double per thread over the block, in a fixed order; every thread
// gets the result (red: blockDim/64 doubles of LDS)
__device__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < nw; ++q) s += red[q];
  return s;
}

// exclusive prefix sum of one int per thread over the block (block of 1024)
__device__ int block_scan_excl(int v, int *red, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  __syncthreads();
  if (lane == 63) red[w] = incl;
  __syncthreads();
  int before = 0, all = 0;
  for (int q = 0; q < nw; ++q) {
    if (q < w) before += red[q];
    all += red[q];
  }
  *total = all;
  return before + incl - v;
}

__device__ __forceinline__ unsigned long long var_key(double x) {
  return (unsigned long long)__double_as_longlong(x);  // variances are >= 0
}

}  // namespace

__global__ void __launch_bounds__(256) suave_root_kernel(SuaveArgs A) {
  const int d = A.d, N = A.N;
  for (int e = threadIdx.x; e < d * (N + 1); e += blockDim.x)
    A.R.grid[e] = (double)(e % (N + 1)) / N;
  if (threadIdx.x < d) {
    A.R.lo[threadIdx.x] = 0.0;
    A.R.hi[threadIdx.x] = 1.0;
  }
  if (threadIdx.x == 0) {
    A.R.inh_I[0] = 0.0;
    A.R.inh_var[0] = 0.0;
    A.chpos[0] = 0;
    A.chser[0] = 0;
  }
}

constexpr int kKeyBatch = 8;  // key loads issued together by the selection

// The K largest of R non-negative keys, ties to the lower position, in that
// order (the regions of largest variance here, of largest spread in the
// Divonne partition).
__global__ void __launch_bounds__(1024) topk_kernel(const double *key, int R, int K, int *sel) {
  __shared__ unsigned hist[256];
  __shared__ int red[16];
  __shared__ unsigned long long s_prefix, s_mask;
  __shared__ int s_krem;
  __shared__ unsigned long long skey[kSuaveMaxSplit];
  __shared__ int spos[kSuaveMaxSplit];
  const int tid = threadIdx.x;
  const int chunk = (R + 1023) / 1024;
  const int b0 = min(tid * chunk, R), b1 = min(b0 + chunk, R);
  if (tid == 0) {
    s_prefix = 0;
    s_mask = 0;
    s_krem = K;
  }
  // radix select of the K-th largest key, 8 bits at a time from the top
  for (int shift = 56; shift >= 0; shift -= 8) {
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
    const unsigned long long pre = s_prefix, mask = s_mask;
    for (int i0 = b0; i0 < b1; i0 += kKeyBatch) {  // a batch of loads in flight
      unsigned long long kk[kKeyBatch];
#pragma unroll
      for (int q = 0; q < kKeyBatch; ++q) kk[q] = i0 + q < b1 ? var_key(key[i0 + q]) : 0;
#pragma unroll
      for (int q = 0; q < kKeyBatch; ++q)
        if (i0 + q < b1 && (kk[q] & mask) == pre) atomicAdd(&hist[(kk[q] >> shift) & 255], 1u);
    }
    __syncthreads();
    if (tid < 64) {  // one wavefront: lane l owns digits 4l .. 4l+3
      const int lane = tid;
      const unsigned h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2],
                     h3 = hist[4 * lane + 3];
      const unsigned mine = h0 + h1 + h2 + h3;
      // count of keys with a larger digit: the lanes above, inclusive scan downwards
      unsigned above = mine;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const unsigned t = __shfl_down(above, o, 64);
        if (lane + o < 64) above += t;
      }
      above -= mine;
      const int krem = s_krem;
      const unsigned hh[4] = {h0, h1, h2, h3};
      unsigned cum = above;
      for (int q = 3; q >= 0; --q) {
        if (cum < (unsigned)krem && (unsigned)krem <= cum + hh[q]) {
          s_krem = krem - (int)cum;
          s_prefix = pre | ((unsigned long long)(4 * lane + q) << shift);
          s_mask = mask | (255ull << shift);
        }
        cum += hh[q];
      }
    }
    __syncthreads();
  }
  const unsigned long long T = s_prefix;
  const int take_eq = s_krem;  // keys equal to T taken, the lowest positions first
  int ngt = 0, neq = 0;
  for (int i0 = b0; i0 < b1; i0 += kKeyBatch) {
    unsigned long long kk[kKeyBatch];
#pragma unroll
    for (int q = 0; q < kKeyBatch; ++q) kk[q] = i0 + q < b1 ? var_key(key[i0 + q]) : 0;
#pragma unroll
    for (int q = 0; q < kKeyBatch; ++q)
      if (i0 + q < b1) {
        ngt += kk[q] > T;
        neq += kk[q] == T;
      }
  }
  int tot;
  int gbase = block_scan_excl(ngt, red, &tot);
  int ebase = block_scan_excl(neq, red, &tot);
  for (int i0 = b0; i0 < b1; i0 += kKeyBatch) {
    unsigned long long kk[kKeyBatch];
#pragma unroll
    for (int q = 0; q < kKeyBatch; ++q) kk[q] = i0 + q < b1 ? var_key(key[i0 + q]) : 0;
    for (int q = 0; q < kKeyBatch && i0 + q < b1; ++q) {
      const unsigned long long k = kk[q];
      const int i = i0 + q;
      if (k > T) {
        skey[gbase] = k;
        spos[gbase] = i;
        ++gbase;
      } else if (k == T) {
        if (ebase < take_eq) {
          skey[K - take_eq + ebase] = k;
          spos[K - take_eq + ebase] = i;
        }
        ++ebase;
      }
    }
  }
  int P = 1;
  while (P < K) P <<= 1;
  for (int i = K + tid; i < P; i += 1024) {
    skey[i] = 0;
    spos[i] = 0x7fffffff;
  }
  __syncthreads();
  // bitonic sort: larger key first, then lower position
  for (int size = 2; size <= P; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < P; i += 1024) {
        const int jx = i ^ stride;
        if (jx > i) {
          const bool up = (i & size) == 0;
          const unsigned long long ka = skey[i], kb = skey[jx];
          const int pa = spos[i], pb = spos[jx];
          const bool a_first = ka > kb || (ka == kb && pa < pb);
          if (a_first != up) {
            skey[i] = kb;
            skey[jx] = ka;
            spos[i] = pb;
            spos[jx] = pa;
          }
        }
      }
      __syncthreads();
    }
  for (int i = tid; i < K; i += 1024) sel[i] = spos[i];
}

// Split statistics in two passes over each selected region's sample, both
// spread over chunks of kSuaveChunk points (grid: chunk x dimension group x
// region):
//   pass 1, per (dimension, half): count, S1 = sum v, S2 = sum v^2, min v and
//           max v; the largest deviation from the half's mean m_h is then
//           exactly M_h = max(vmax - m_h, m_h - vmin);
//   pass 2, per (dimension, half): sum (|v - m_h| / M_h)^p.
// Chunk partials are reduced in chunk order wherever they are needed.
constexpr int kP1 = 9;       // per (chunk, dimension): cnt1, S1_0, S2_0, S1_1, S2_1, min0, max0, min1, max1

// Both passes stage their chunk in LDS once; then G threads per dimension
// (G = kFlBlock over d rounded up to a power of two, at most 64) accumulate over
// it, two points at a time into independent partial sums, and reduce with
// shuffles within their G-lane group.
constexpr int kFlBlock = 512;  // threads of the split-statistics workgroups
static_assert(kSuaveChunk % kFlBlock == 0, "a chunk stages evenly over the workgroup");

__device__ __forceinline__ int lanes_per_dim(int d) {
  int dp = 1;
  while (dp < d) dp <<= 1;
  return min(64, kFlBlock / dp);
}

__device__ __forceinline__ int stage_chunk(const double *vall, const uint16_t *sall, int pos,
                                           long long n, int ch, double *sv, uint16_t *sb) {
  const long long i0 = (long long)ch * kSuaveChunk;
  const int cnt = (int)min((long long)kSuaveChunk, n - i0);
  const double *v = vall + (size_t)pos * n + i0;
  const uint16_t *sd = sall + (size_t)pos * n + i0;
  // all of a thread's loads in flight at once (kSuaveChunk / kFlBlock each)
  constexpr int kPer = kSuaveChunk / kFlBlock;
  double tv[kPer];
  uint16_t tb[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + kFlBlock * k;
    tv[k] = i < cnt ? v[i] : 0.0;
    tb[k] = i < cnt ? sd[i] : (uint16_t)0;
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    sv[threadIdx.x + kFlBlock * k] = tv[k];
    sb[threadIdx.x + kFlBlock * k] = tb[k];
  }
  __syncthreads();
  return cnt;
}

// pass-1 partial sums: cnt1, S1_0, S2_0, S1_1, S2_1, min0, max0, min1, max1
__device__ __forceinline__ void p1_init(double (&a)[kP1]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) a[q] = 0.0;
  a[5] = a[7] = INFINITY;
  a[6] = a[8] = -INFINITY;
}
__device__ __forceinline__ void p1_add(double (&a)[kP1], double x, bool up) {
  // branch-free (a branch here sends both partials to scratch); adding 0.0
  // to the other half's sums leaves them unchanged
  const double xu = up ? x : 0.0, xl = up ? 0.0 : x;
  a[0] += up ? 1.0 : 0.0;
  a[1] += xl;
  a[2] += xl * xl;
  a[3] += xu;
  a[4] += xu * xu;
  a[5] = up ? a[5] : fmin(a[5], x);
  a[6] = up ? a[6] : fmax(a[6], x);
  a[7] = up ? fmin(a[7], x) : a[7];
  a[8] = up ? fmax(a[8], x) : a[8];
}
__device__ __forceinline__ double p1_merge(int q, double x, double y) {
  return (q == 5 || q == 7) ? fmin(x, y) : (q == 6 || q == 8) ? fmax(x, y) : x + y;
}

// Pass 1 over one chunk: grid (chunk, selected region).
__global__ void __launch_bounds__(kFlBlock) suave_fluct1_kernel(SuaveArgs A) {
  __shared__ double sv[kSuaveChunk];
  __shared__ uint16_t sb[kSuaveChunk];
  const int ch = blockIdx.x, s = blockIdx.y, tid = threadIdx.x, d = A.d;
  const int cnt = stage_chunk(A.R.v, A.R.side, A.sel[s], A.nnew, ch, sv, sb);
  const int G = lanes_per_dim(d);
  const int j = tid / G, sub = tid % G;
  if (j >= d) return;
  double x0[kP1], x1[kP1];
  p1_init(x0);
  p1_init(x1);
  int i = sub;
  for (; i + G < cnt; i += 2 * G) {
    p1_add(x0, sv[i], (sb[i] >> j) & 1u);
    p1_add(x1, sv[i + G], (sb[i + G] >> j) & 1u);
  }
  if (i < cnt) p1_add(x0, sv[i], (sb[i] >> j) & 1u);
#pragma unroll
  for (int q = 0; q < kP1; ++q) {
    double r = p1_merge(q, x0[q], x1[q]);
    for (int o = G >> 1; o > 0; o >>= 1) r = p1_merge(q, r, __shfl_xor(r, o, G));
    x0[q] = r;
  }
  if (sub == 0) {
    double *r = A.fl1 + (((size_t)s * A.nchunks + ch) * d + j) * kP1;
#pragma unroll
    for (int q = 0; q < kP1; ++q) r[q] = x0[q];
  }
}

namespace {

// pass 1 of (region s, dimension j) over all chunks, in chunk order
struct HalfStats {
  double cnt[2], S1[2], S2[2], m[2], M[2];
};
__device__ HalfStats half_stats(const SuaveArgs &A, int s, int j) {
  double c1 = 0.0, a0 = 0.0, q0 = 0.0, a1 = 0.0, q1 = 0.0;
  double mn0 = INFINITY, mx0 = -INFINITY, mn1 = INFINITY, mx1 = -INFINITY;
#pragma unroll 8
  for (int ch = 0; ch < A.nchunks; ++ch) {
    const double *r = A.fl1 + (((size_t)s * A.nchunks + ch) * A.d + j) * kP1;
    c1 += r[0];
    a0 += r[1];
    q0 += r[2];
    a1 += r[3];
    q1 += r[4];
    mn0 = fmin(mn0, r[5]);
    mx0 = fmax(mx0, r[6]);
    mn1 = fmin(mn1, r[7]);
    mx1 = fmax(mx1, r[8]);
  }
  HalfStats h;
  h.cnt[0] = (double)A.nnew - c1;
  h.cnt[1] = c1;
  h.S1[0] = a0;
  h.S2[0] = q0;
  h.S1[1] = a1;
  h.S2[1] = q1;
  h.m[0] = h.cnt[0] > 0.0 ? a0 / h.cnt[0] : 0.0;
  h.m[1] = c1 > 0.0 ? a1 / c1 : 0.0;
  h.M[0] = h.cnt[0] > 0.0 ? fmax(mx0 - h.m[0], h.m[0] - mn0) : 0.0;
  h.M[1] = c1 > 0.0 ? fmax(mx1 - h.m[1], h.m[1] - mn1) : 0.0;
  return h;
}

}  // namespace

namespace {

// r^p for r in [0, 1] (0^p = 0): by squaring for a whole p
__device__ __forceinline__ double pow01(double r, double p, int ip) {
  if (ip > 0) {
    double t = 1.0, b = r;
    for (int e = ip; e; e >>= 1) {
      if (e & 1) t *= b;
      b *= b;
    }
    return t;
  }
  return r > 0.0 ? exp2(p * log2(r)) : 0.0;
}

}  // namespace

// Pass 1 reduced over the chunks, once per (selected region, dimension):
// grid (selected region), lane j < d.
constexpr int kHs = 10;  // per (region, dimension): cnt, S1, S2, m, M of each half
__global__ void __launch_bounds__(64) suave_fluct_reduce_kernel(SuaveArgs A) {
  const int s = blockIdx.x, j = threadIdx.x;
  if (j >= A.d) return;
  const HalfStats h = half_stats(A, s, j);
  double *o = A.hs + ((size_t)s * A.d + j) * kHs;
  for (int k = 0; k < 2; ++k) {
    o[5 * k + 0] = h.cnt[k];
    o[5 * k + 1] = h.S1[k];
    o[5 * k + 2] = h.S2[k];
    o[5 * k + 3] = h.m[k];
    o[5 * k + 4] = h.M[k];
  }
}

// Pass 2 over one chunk: grid (chunk, selected region).
__global__ void __launch_bounds__(kFlBlock) suave_fluct2_kernel(SuaveArgs A) {
  __shared__ double sv[kSuaveChunk];
  __shared__ uint16_t sb[kSuaveChunk];
  __shared__ double sm[kMaxDim][2], sinv[kMaxDim][2];
  const int ch = blockIdx.x, s = blockIdx.y, tid = threadIdx.x, d = A.d;
  if (tid < d) {
    const double *h = A.hs + ((size_t)s * d + tid) * kHs;
    for (int k = 0; k < 2; ++k) {
      sm[tid][k] = h[5 * k + 3];
      sinv[tid][k] = h[5 * k + 4] > 0.0 ? 1.0 / h[5 * k + 4] : 0.0;
    }
  }
  const int cnt = stage_chunk(A.R.v, A.R.side, A.sel[s], A.nnew, ch, sv, sb);
  const int G = lanes_per_dim(d);
  const int j = tid / G, sub = tid % G;
  if (j >= d) return;
  const double p = A.flatness;
  const int ip = A.ipow;
  const double m0 = sm[j][0], m1 = sm[j][1], i0v = sinv[j][0], i1v = sinv[j][1];
  double q00 = 0.0, q01 = 0.0, q10 = 0.0, q11 = 0.0;  // [partial][half]
  int i = sub;
  for (; i + G < cnt; i += 2 * G) {
    const bool ua = (sb[i] >> j) & 1u, ub = (sb[i + G] >> j) & 1u;
    const double ta = pow01(fabs(sv[i] - (ua ? m1 : m0)) * (ua ? i1v : i0v), p, ip);
    const double tb = pow01(fabs(sv[i + G] - (ub ? m1 : m0)) * (ub ? i1v : i0v), p, ip);
    if (ua) q01 += ta; else q00 += ta;
    if (ub) q11 += tb; else q10 += tb;
  }
  if (i < cnt) {
    const bool ua = (sb[i] >> j) & 1u;
    const double ta = pow01(fabs(sv[i] - (ua ? m1 : m0)) * (ua ? i1v : i0v), p, ip);
    if (ua) q01 += ta; else q00 += ta;
  }
  double q0 = q00 + q10, q1 = q01 + q11;
  for (int o = G >> 1; o > 0; o >>= 1) {
    q0 += __shfl_xor(q0, o, G);
    q1 += __shfl_xor(q1, o, G);
  }
  if (sub == 0) {
    double *r = A.fl2 + (((size_t)s * A.nchunks + ch) * d + j) * 2;
    r[0] = q0;
    r[1] = q1;
  }
}

namespace {

// the parent's map along one dimension, X(y), piecewise linear through (k/N, E_k)
__device__ __forceinline__ double map_at(const double *E, int N, double y) {
  const double z = y * N;
  int k = (int)floor(z);
  k = min(max(k, 0), N - 1);
  return fma(z - k, E[k + 1] - E[k], E[k]);
}

// running maximum over e[0..n) by one wavefront (lanes own contiguous runs)
__device__ void wave_prefix_max(double *e, int n, int lane) {
  const int per = (n + 63) >> 6;
  const int k0 = min(lane * per, n), k1 = min(k0 + per, n);
  double run = -INFINITY;
  for (int k = k0; k < k1; ++k) run = fmax(run, e[k]);
  double incl = run;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double t = __shfl_up(incl, o, 64);
    if (lane >= o) incl = fmax(incl, t);
  }
  double acc = __shfl_up(incl, 1, 64);
  if (lane == 0) acc = -INFINITY;
  for (int k = k0; k < k1; ++k) {
    acc = fmax(acc, e[k]);
    e[k] = acc;
  }
}

}  // namespace

// Per selected region: the cut and the two children.
__global__ void __launch_bounds__(256) suave_split_kernel(SuaveArgs A, int R, long long Q) {
  __shared__ double sE[kMaxBins + 1];
  __shared__ double sOut[2][kMaxBins + 1];
  __shared__ int s_cut, s_ks;
  const int s = blockIdx.x, tid = threadIdx.x;
  const int d = A.d, N = A.N, row = N + 1;
  const int pos = A.sel[s], up = R + s;
  __shared__ double s_score[kMaxDim], s_S[kMaxDim][4];
  if (tid < d) {  // F_0 + F_1 of a cut along dimension tid
    const double *h = A.hs + ((size_t)s * d + tid) * kHs;
    const double nd = (double)A.nnew, p = A.flatness;
    double score = 0.0;
    for (int k = 0; k < 2; ++k) {
      double q = 0.0;
#pragma unroll 8
      for (int ch = 0; ch < A.nchunks; ++ch)
        q += A.fl2[(((size_t)s * A.nchunks + ch) * d + tid) * 2 + k];
      const double cnt = h[5 * k], M = h[5 * k + 4];
      if (cnt > 0.0 && M > 0.0) score += (cnt / nd) * M * pow(q / cnt, 1.0 / p);
    }
    s_score[tid] = score;
    s_S[tid][0] = h[1];
    s_S[tid][1] = h[2];
    s_S[tid][2] = h[6];
    s_S[tid][3] = h[7];
  }
  __syncthreads();
  if (tid == 0) {
    int best = 0;
    double b = s_score[0];
    for (int c = 1; c < d; ++c)
      if (s_score[c] < b) {
        b = s_score[c];
        best = c;
      }
    s_cut = best;
    A.cut[Q + s] = best;
  }
  __syncthreads();
  const int c = s_cut;
  double *Gp = A.R.grid + (size_t)pos * d * row;
  double *Gu = A.R.grid + (size_t)up * d * row;
  for (int e = tid; e < d * row; e += 256) Gu[e] = Gp[e];
  for (int e = tid; e <= N; e += 256) sE[e] = Gp[c * row + e];
  if (tid < d) {
    A.R.lo[(size_t)up * d + tid] = A.R.lo[(size_t)pos * d + tid];
    A.R.hi[(size_t)up * d + tid] = A.R.hi[(size_t)pos * d + tid];
  }
  __syncthreads();
  if (tid == 0) {
    const double mid = 0.5 * (A.R.lo[(size_t)pos * d + c] + A.R.hi[(size_t)pos * d + c]);
    A.R.hi[(size_t)pos * d + c] = mid;
    A.R.lo[(size_t)up * d + c] = mid;
    const double n = (double)A.nnew;
    for (int h = 0; h < 2; ++h) {
      const double I = s_S[c][2 * h] / n;
      const double var = fmax(0.0, s_S[c][2 * h + 1] / n - I * I) / (n - 1.0);
      const int p = h == 0 ? pos : up;
      A.R.inh_I[p] = var > 0.0 ? I : 0.0;
      A.R.inh_var[p] = var > 0.0 ? var : 0.0;
    }
    A.chpos[2 * s] = pos;
    A.chpos[2 * s + 1] = up;
    A.chser[2 * s] = (int)(2 * (Q + s) + 1);
    A.chser[2 * s + 1] = (int)(2 * (Q + s) + 2);
  }
  // the bin holding 1/2: the first k with E_k+1 > 1/2 (at most N - 1)
  if (tid == 0) s_ks = N - 1;
  __syncthreads();
  for (int k = tid; k < N; k += 256)
    if (sE[k + 1] > 0.5) atomicMin(&s_ks, k);
  __syncthreads();
  const int ks = s_ks;
  const double ystar = (ks + (0.5 - sE[ks]) / (sE[ks + 1] - sE[ks])) / N;
  for (int k = tid; k <= N; k += 256) {
    const double t = (double)k / N;
    sOut[0][k] = 2.0 * map_at(sE, N, ystar * t);
    sOut[1][k] = 2.0 * map_at(sE, N, fma(1.0 - ystar, t, ystar)) - 1.0;
  }
  __syncthreads();
  if (tid == 0) {
    sOut[0][0] = sOut[1][0] = 0.0;
    sOut[0][N] = sOut[1][N] = 1.0;
  }
  __syncthreads();
  if (tid < 128) wave_prefix_max(sOut[tid >> 6], N + 1, tid & 63);
  __syncthreads();
  for (int k = tid; k <= N; k += 256) {
    Gp[c * row + k] = sOut[0][k];
    Gu[c * row + k] = sOut[1][k];
  }
}

// DoSample of every child: one workgroup per (tile of kSuaveTile points, child).
template <int FAM, int NB>
__global__ void __launch_bounds__(kSuaveBlock) suave_sample_kernel(SuaveArgs A) {
  extern __shared__ double lds[];
  __shared__ double sBlo[kMaxDim], sBw[kMaxDim], sP0[kMaxDim], sP1[kMaxDim];
  __shared__ double red[kSuaveBlock / 64];
  const int c = blockIdx.y, tile = blockIdx.x, tid = threadIdx.x;
  const int pos = A.chpos[c], serial = A.chser[c];
  const int d = A.d, N = A.N, dN = d * N;
  double *sLo = lds, *sSp = lds + dN, *sH = lds + 2 * dN;
  const double *G = A.R.grid + (size_t)pos * d * (N + 1);
  for (int e = tid; e < dN; e += kSuaveBlock) {
    const int j = e / N, k = e - j * N;
    const double l = G[j * (N + 1) + k], h = G[j * (N + 1) + k + 1];
    sLo[e] = l;
    sSp[e] = h - l;
    sH[e] = 0.0;
  }
  if (tid < d) {
    const double lo = A.R.lo[(size_t)pos * d + tid];
    sBlo[tid] = lo;
    sBw[tid] = A.R.hi[(size_t)pos * d + tid] - lo;
    sP0[tid] = A.p64[tid];
    sP1[tid] = A.p64[kParamRow + tid];
  }
  __syncthreads();
  double V = 1.0;
  for (int j = 0; j < d; ++j) V *= sBw[j];
  const double phase0 = sP1[0];
  const double Nd = (double)N;
  const long long n = A.nnew;
  const long long i0 = (long long)tile * kSuaveTile;
  const long long i1 = min(i0 + (long long)kSuaveTile, n);
  double *vout = A.R.v + (size_t)pos * n;
  uint16_t *sout = A.R.side + (size_t)pos * n;
  double S1 = 0.0, S2 = 0.0;
  for (long long i = i0 + tid; i < i1; i += kSuaveBlock) {
    double w = 1.0;
    double acc = Genz<double, FAM>::init(phase0);
    uint32_t bits = 0;
    int cell[4 * NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      {
        const U4 W = philox4x32_10(
            U4{(uint32_t)i, ((uint32_t)serial << 8) | (uint32_t)b, A.sid, 0u}, A.key0, A.key1);
        const uint32_t wd[4] = {W.x, W.y, W.z, W.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = 4 * b + q;
          cell[j] = 0;
          if (j < d) {
            const double y = (double)wd[q] * 0x1p-32 + 0x1p-33;
            const double z = y * Nd;
            int k = (int)z;
            if (k > N - 1) k = N - 1;
            const double fr = z - (double)k;
            const int e = j * N + k;
            const double sp = sSp[e];
            const double xr = fma(fr, sp, sLo[e]);
            w = w * (Nd * sp);
            acc = Genz<double, FAM>::step(acc, fma(xr, sBw[j], sBlo[j]), sP0[j], sP1[j]);
            if (xr >= 0.5) bits |= 1u << j;
            cell[j] = e;
          }
        }
      }
    }
    const double v = (w * V) * Genz<double, FAM>::finish(acc, d);
    vout[i] = v;
    sout[i] = (uint16_t)bits;
    const double v2 = v * v;
    S1 += v;
    S2 += v2;
#pragma unroll
    for (int j = 0; j < 4 * NB; ++j)
      if (j < d) atomicAdd(&sH[cell[j]], v2);
  }
  S1 = block_sum(S1, red);
  S2 = block_sum(S2, red);
  const size_t t = (size_t)c * A.ntiles + tile;
  if (tid == 0) {
    A.tsum[2 * t] = S1;
    A.tsum[2 * t + 1] = S2;
  }
  __syncthreads();
  for (int e = tid; e < dN; e += kSuaveBlock) A.thist[t * dN + e] = sH[e];
}

// Per child: its own estimate, the combination, and the refined grid.
__global__ void __launch_bounds__(1024) suave_fold_kernel(SuaveArgs A) {
  extern __shared__ double lds[];
  __shared__ double red[16];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int pos = A.chpos[c];
  const int d = A.d, N = A.N, dN = d * N, row = N + 1, nt = A.ntiles;
  double *H = lds, *D = lds + dN, *E = lds + 2 * dN;
  double S1 = 0.0, S2 = 0.0;
  for (int t = tid; t < nt; t += 1024) {
    S1 += A.tsum[2 * ((size_t)c * nt + t)];
    S2 += A.tsum[2 * ((size_t)c * nt + t) + 1];
  }
  S1 = block_sum(S1, red);
  S2 = block_sum(S2, red);
  const double *th = A.thist + (size_t)c * nt * dN;
  for (int e = tid; e < dN; e += 1024) {
    double h = 0.0;
#pragma unroll 8
    for (int t = 0; t < nt; ++t) h += th[(size_t)t * dN + e];
    H[e] = h;
  }
  double *G = A.R.grid + (size_t)pos * d * row;
  for (int e = tid; e < d * row; e += 1024) E[e] = G[e];
  if (tid == 0) {
    const double n = (double)A.nnew;
    const double I = S1 / n;
    const double var = fmax(0.0, S2 / n - I * I) / (n - 1.0);
    const double iI = A.R.inh_I[pos], iv = A.R.inh_var[pos];
    const bool inh = iv > 0.0;
    const double Ik[2] = {iI, I}, Vk[2] = {iv, var};
    const int k0 = inh ? 0 : 1;
    int nzero = 0;
    double zsum = 0.0;
    for (int k = k0; k < 2; ++k)
      if (Vk[k] == 0.0) {
        ++nzero;
        zsum += Ik[k];
      }
    double Ir, Vr, chi2 = 0.0;
    if (nzero > 0) {
      Ir = zsum / nzero;
      Vr = 0.0;
    } else {
      double ws = 0.0, wi = 0.0;
      for (int k = k0; k < 2; ++k) {
        ws += 1.0 / Vk[k];
        wi += Ik[k] / Vk[k];
      }
      Ir = wi / ws;
      Vr = 1.0 / ws;
      for (int k = k0; k < 2; ++k) chi2 += (Ik[k] - Ir) * (Ik[k] - Ir) / Vk[k];
    }
    A.R.I[pos] = Ir;
    A.R.var[pos] = Vr;
    A.R.chi2[pos] = chi2;
    A.R.dof[pos] = inh ? 1 : 0;
  }
  __syncthreads();
  if (A.flags & FLAG_FREEZE_GRID) return;
  const int w = tid >> 6, lane = tid & 63;
  if (w < d) rebin_dimension(H + w * N, D + w * N, E + w * row, G + w * row, N, lane);
}

// Totals over the R regions (fixed order) and the chi^2 probability.
__global__ void __launch_bounds__(1024) suave_totals_kernel(SuaveArgs A, int R) {
  __shared__ double red[16];
  const int tid = threadIdx.x;
  const int chunk = (R + 1023) / 1024;
  const int b0 = min(tid * chunk, R), b1 = min(b0 + chunk, R);
  double I = 0.0, V = 0.0, X = 0.0, F = 0.0;
  for (int i = b0; i < b1; ++i) {
    I += A.R.I[i];
    V += A.R.var[i];
    X += A.R.chi2[i];
    F += (double)A.R.dof[i];
  }
  I = block_sum(I, red);
  V = block_sum(V, red);
  X = block_sum(X, red);
  F = block_sum(F, red);
  if (tid == 0) {
    SState st;
    st.I = I;
    st.var = V;
    st.chi2 = X;
    st.dof = (int)F;
    st.pad = 0;
    st.prob = st.dof > 0 ? gamma_p(0.5 * st.dof, 0.5 * X) : 0.0;
    *A.state = st;
  }
}

// ---- launchers ---------------------------------------------------------------

size_t suave_sample_lds(int d, int N) { return (size_t)3 * d * N * sizeof(double); }
size_t suave_fold_lds(int d, int N) {
  return ((size_t)2 * d * N + (size_t)d * (N + 1)) * sizeof(double);
}

hipError_t suave_set_kernel_limits() {
  const int big = 160 * 1024;
  const void *fns[] = {(const void *)suave_fold_kernel,
#define CCUBA_SUAVE_FNS(F)                                                            \
  (const void *)suave_sample_kernel<F, 1>, (const void *)suave_sample_kernel<F, 2>, \
      (const void *)suave_sample_kernel<F, 3>, (const void *)suave_sample_kernel<F, 4>
                       CCUBA_SUAVE_FNS(GAUSSIAN), CCUBA_SUAVE_FNS(OSCILLATORY),
                       CCUBA_SUAVE_FNS(PRODUCT_PEAK), CCUBA_SUAVE_FNS(CORNER_PEAK),
                       CCUBA_SUAVE_FNS(C0)};
#undef CCUBA_SUAVE_FNS
  for (const void *f : fns)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big) != hipSuccess)
      (void)hipGetLastError();
  return hipSuccess;
}

hipError_t launch_suave_root(const SuaveArgs &A, hipStream_t s) {
  hipLaunchKernelGGL(suave_root_kernel, dim3(1), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_topk(const double *key, int R, int K, int *sel, hipStream_t s) {
  hipLaunchKernelGGL(topk_kernel, dim3(1), dim3(1024), 0, s, key, R, K, sel);
  return hipGetLastError();
}

hipError_t launch_suave_select(const SuaveArgs &A, int R, int K, hipStream_t s) {
  return launch_topk(A.R.var, R, K, A.sel, s);
}

hipError_t launch_suave_fluct(const SuaveArgs &A, int K, hipStream_t s) {
  hipLaunchKernelGGL(suave_fluct1_kernel, dim3(A.nchunks, K), dim3(kFlBlock), 0, s, A);
  hipLaunchKernelGGL(suave_fluct_reduce_kernel, dim3(K), dim3(64), 0, s, A);
  hipLaunchKernelGGL(suave_fluct2_kernel, dim3(A.nchunks, K), dim3(kFlBlock), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_suave_split(const SuaveArgs &A, int R, long long Q, int K, hipStream_t s) {
  hipLaunchKernelGGL(suave_split_kernel, dim3(K), dim3(256), 0, s, A, R, Q);
  return hipGetLastError();
}

namespace {

template <int FAM>
void launch_sample_fam(const SuaveArgs &A, dim3 grid, size_t lds, hipStream_t s) {
  switch ((A.d + 3) / 4) {
    case 1:
      hipLaunchKernelGGL((suave_sample_kernel<FAM, 1>), grid, dim3(kSuaveBlock), lds, s, A);
      break;
    case 2:
      hipLaunchKernelGGL((suave_sample_kernel<FAM, 2>), grid, dim3(kSuaveBlock), lds, s, A);
      break;
    case 3:
      hipLaunchKernelGGL((suave_sample_kernel<FAM, 3>), grid, dim3(kSuaveBlock), lds, s, A);
      break;
    default:
      hipLaunchKernelGGL((suave_sample_kernel<FAM, 4>), grid, dim3(kSuaveBlock), lds, s, A);
      break;
  }
}

}  // namespace

hipError_t launch_suave_sample(const SuaveArgs &A, int nchild, hipStream_t s) {
  const dim3 grid(A.ntiles, nchild);
  const size_t lds = suave_sample_lds(A.d, A.N);
  switch (A.family) {
    case GAUSSIAN:
      launch_sample_fam<GAUSSIAN>(A, grid, lds, s);
      break;
    case OSCILLATORY:
      launch_sample_fam<OSCILLATORY>(A, grid, lds, s);
      break;
    case PRODUCT_PEAK:
      launch_sample_fam<PRODUCT_PEAK>(A, grid, lds, s);
      break;
    case CORNER_PEAK:
      launch_sample_fam<CORNER_PEAK>(A, grid, lds, s);
      break;
    default:
      launch_sample_fam<C0>(A, grid, lds, s);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_suave_fold(const SuaveArgs &A, int nchild, hipStream_t s) {
  hipLaunchKernelGGL(suave_fold_kernel, dim3(nchild), dim3(1024), suave_fold_lds(A.d, A.N), s, A);
  return hipGetLastError();
}

hipError_t launch_suave_totals(const SuaveArgs &A, int R, hipStream_t s) {
  hipLaunchKernelGGL(suave_totals_kernel, dim3(1), dim3(1024), 0, s, A, R);
  return hipGetLastError();
}

}  // namespace ccuba
