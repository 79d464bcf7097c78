// vegas.hip -- Vegas DoSample and grid refinement on gfx950.
//
// DoSample (Sect. 2.1) samples n points; the paper splits them n/N over N
// worker processes.  Here the split is over tiles of consecutive point
// indices, processed by persistent workgroups.  Each point is produced in
// registers from its Philox counter, so no sample ever crosses HBM:
//   a1 words   W_b = philox(ctr = (i, (t<<8)|b, sid, 0), key = seed)
//   a2 uniform FP64 y = r 2^-32 + 2^-33 | FP32 y = (r>>9) 2^-23 + 2^-24
//   a3 map     z = y N, k = min(floor z, N-1), x = E[k] + (z-k)(E[k+1]-E[k]),
//              w *= N (E[k+1]-E[k])     (grid staged in LDS per tile)
//   a4 f       Genz family, accumulated one dimension at a time
//   a5 sums    v = w f: S1 += v, S2 += v^2 in FP64 per lane, wave shuffles,
//              then a fixed-order block sum -> one FP64 partial per tile
//   a6 hist    H_j[k_j] += v^2 with LDS atomics, flushed per tile as FP64
// Tiles are folded 32 at a time by the last block to finish (fixed tile
// order, so the fold is deterministic), and the refine kernel (one
// workgroup per integral) finishes the sums in fixed order and does a7:
// iteration statistics, the inverse-variance combination with chi^2 and its
// probability, the convergence test and Lepage's grid refinement, all in FP64.
// Iteration t and its point count are read from device state, so a captured
// iteration replays unchanged.
#include "engine.h"
#include "genz.h"
#include "philox.h"
#include "vegas.h"

#include <vector>

namespace ccuba {

// ---------------------------------------------------------------------------
// a2 + a3: one coordinate

__device__ __forceinline__ void map_coord(uint32_t r, int N, double Nd, const double *E,
                                          double &x, double &jac, int &k) {
  const double y = (double)r * 0x1p-32 + 0x1p-33;
  const double z = y * Nd;
  int kk = (int)z;
  kk = kk > N - 1 ? N - 1 : kk;
  const double frac = z - (double)kk;
  const double lo = E[kk];
  const double width = E[kk + 1] - lo;
  x = fma(frac, width, lo);
  jac = Nd * width;
  k = kk;
}

__device__ __forceinline__ void map_coord(uint32_t r, int N, float Nf, const float *E,
                                          float &x, float &jac, int &k) {
  const float y = (float)(r >> 9) * 0x1p-23f + 0x1p-24f;
  const float z = y * Nf;
  int kk = (int)z;
  kk = kk > N - 1 ? N - 1 : kk;
  const float frac = z - (float)kk;
  const float lo = E[kk];
  const float width = E[kk + 1] - lo;
  x = fmaf(frac, width, lo);
  jac = Nf * width;
  k = kk;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ const T *param_ptr(const VJob &J, int which);
template <>
__device__ __forceinline__ const double *param_ptr<double>(const VJob &J, int which) {
  return J.p64 + which * kParamRow;
}
template <>
__device__ __forceinline__ const float *param_ptr<float>(const VJob &J, int which) {
  return J.p32 + which * kParamRow;
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }

// Bin and fractional position of one coordinate (a2 + the first half of
// a3).  For N = 2^L the bin is the top L bits of the word and the fraction
// the bits below them, which is exactly what the floating-point formula
// z = y N, k = floor(z), z - k gives (every step there is exact), so both
// forms yield identical values.
__device__ __forceinline__ void bin_frac_pow2(uint32_t r, int L, double &frac, int &k) {
  k = (int)(r >> (32 - L));
  const uint32_t m = (r << L) | (1u << (L - 1));  // (r N mod 2^32) + N/2
  frac = (double)m * 0x1p-32;
}
__device__ __forceinline__ void bin_frac_pow2(uint32_t r, int L, float &frac, int &k) {
  k = (int)(r >> (32 - L));
  const uint32_t m = (((r >> 9) << L) & 0x7FFFFFu) | (1u << (L - 1));
  frac = (float)m * 0x1p-23f;
}
__device__ __forceinline__ void bin_frac_any(uint32_t r, int N, double Nd, double &frac, int &k) {
  const double y = (double)r * 0x1p-32 + 0x1p-33;
  const double z = y * Nd;
  int kk = (int)z;
  kk = kk > N - 1 ? N - 1 : kk;
  frac = z - (double)kk;
  k = kk;
}
__device__ __forceinline__ void bin_frac_any(uint32_t r, int N, float Nf, float &frac, int &k) {
  const float y = (float)(r >> 9) * 0x1p-23f + 0x1p-24f;
  const float z = y * Nf;
  int kk = (int)z;
  kk = kk > N - 1 ? N - 1 : kk;
  frac = z - (float)kk;
  k = kk;
}

// Sample the points [i0, i0 + cnt) of one tile; lane sums go to S1, S2.
// NB = ceil(d/4) Philox blocks per point is a template argument so that the
// per-dimension loop is fully unrolled with only the last block guarded.
// Each lane carries ILP independent points per trip (q, q + blockDim, ...),
// so that several Philox chains are in flight; a point past the tile end is
// computed (its LDS reads stay in range) but contributes nothing.  All lanes
// run the same number of trips (a build in which lanes left the loop on
// different trips, holding deferred updates, produced wrong histograms in
// partially filled tiles).  The
// histogram updates of a trip are issued in the next trip, after its grid
// reads, so that those reads never wait behind the atomics in the LDS queue.
template <typename T, typename HT, int FAM, int NB, int ILP, bool POW2>
__device__ __forceinline__ void sample_tile(const VJob &J, int t, long long i0, int cnt,
                                            const T *__restrict__ sE, HT *sH,
                                            const T *__restrict__ p0,
                                            const T *__restrict__ p1, double &S1,
                                            double &S2) {
  constexpr int ND = 4 * NB;
  const int d = J.ndim, N = J.nbins, row = N + 1;
  const T Nt = (T)N;
  const int L = POW2 ? 31 - __clz(N) : 0;
  const uint32_t c1 = (uint32_t)t << 8;
  const uint32_t sid = J.sid, k0 = J.key0, k1 = J.key1;
  T pp0[ND], pp1[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) {  // parameter rows are zero-padded to 16
    pp0[j] = p0[j];
    pp1[j] = p1[j];
  }
  const T phase0 = p1[0];
  const int bs = blockDim.x;
  int pidx[ILP][ND];  // pending histogram slots of the previous trip
  HT pv[ILP];         // and their value (v^2), 0 for no update
  bool pending = false;
  // every lane runs the same number of trips; points past the tile end are
  // predicated off, so no lane leaves the loop while it holds pending updates
  const int trips = (cnt + ILP * bs - 1) / (ILP * bs);
  for (int tr = 0; tr < trips; ++tr) {
    const int q0 = tr * ILP * bs + (int)threadIdx.x;
    T fr[ILP][ND], lo[ILP][ND], hi[ILP][ND];
    int idx[ILP][ND];
    // words, bins and the grid edges they select
#pragma unroll
    for (int e = 0; e < ILP; ++e) {
      const uint32_t i = (uint32_t)(i0 + q0 + e * bs);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const U4 r = philox4x32_10(U4{i, c1 | (uint32_t)b, sid, 0u}, k0, k1);
        const uint32_t rr[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int j = 4 * b + c;
          if (b < NB - 1 || j < d) {
            int k;
            if (POW2)
              bin_frac_pow2(rr[c], L, fr[e][j], k);
            else
              bin_frac_any(rr[c], N, Nt, fr[e][j], k);
            idx[e][j] = j * N + k;
            lo[e][j] = sE[j * row + k];
            hi[e][j] = sE[j * row + k + 1];
          }
        }
      }
    }
    // the previous trip's histogram updates
    if (pending) {
#pragma unroll
      for (int e = 0; e < ILP; ++e) {
        if (pv[e] != (HT)0) {
#pragma unroll
          for (int j = 0; j < ND; ++j)
            if (j < 4 * (NB - 1) || j < d) unsafeAtomicAdd(&sH[pidx[e][j]], pv[e]);
        }
      }
    }
    // weights, integrand, sums
#pragma unroll
    for (int e = 0; e < ILP; ++e) {
      T w = (T)1;
      T acc = Genz<T, FAM>::init(phase0);
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        if (j < 4 * (NB - 1) || j < d) {
          const T width = hi[e][j] - lo[e][j];
          const T x = fma_t(fr[e][j], width, lo[e][j]);
          w = w * (Nt * width);
          acc = Genz<T, FAM>::step(acc, x, pp0[j], pp1[j]);
          pidx[e][j] = idx[e][j];
        }
      }
      const T v = w * Genz<T, FAM>::finish(acc, d);
      const bool valid = q0 + e * bs < cnt;  // also false for q0 >= cnt
      const double vd = valid ? (double)v : 0.0;
      S1 += vd;
      S2 = fma(vd, vd, S2);
      pv[e] = valid ? (HT)(v * v) : (HT)0;
    }
    pending = true;
  }
  if (pending) {
#pragma unroll
    for (int e = 0; e < ILP; ++e) {
      if (pv[e] != (HT)0) {
#pragma unroll
        for (int j = 0; j < ND; ++j)
          if (j < 4 * (NB - 1) || j < d) unsafeAtomicAdd(&sH[pidx[e][j]], pv[e]);
      }
    }
  }
}

// One kernel per (precision, histogram type, ILP, NB): every instance only
// holds the registers its own dimension class needs.  A launch walks the
// slice [tile_first, tile_first + tile_count) of the tile list, which holds
// the tiles of the jobs of that class.
template <typename T, typename HT, int ILP, int NB, bool POW2>
__global__ void __launch_bounds__(256) vegas_dosample_kernel(VegasArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[2][4];
  T *sE = (T *)smem;
  HT *sH = (HT *)(smem + A.lds_hist_byte_off);
  const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wid = tid >> 6;
  const int myprec = sizeof(T) == 8 ? FP64 : FP32;

  const int tend = A.tile_first + A.tile_count;
  for (int tt = A.tile_first + blockIdx.x; tt < tend; tt += gridDim.x) {
    const int jb = A.tile_job[tt];
    const VJob J = A.jobs[jb];
    if (J.prec != myprec || ((J.ndim + 3) >> 2) != NB || ((J.nbins & (J.nbins - 1)) == 0) != POW2)
      continue;
    const VState st = *J.state;
    if (st.done) continue;
    const int d = J.ndim, N = J.nbins, dN = d * N, row = N + 1;
    const int lt = tt - J.tile0;
    const long long n_t = J.nstart + (long long)st.T * J.nincrease;
    const long long i0 = (long long)lt * J.tile_pts;
    long long c = n_t - i0;
    c = c < 0 ? 0 : (c > J.tile_pts ? J.tile_pts : c);
    const int cnt = (int)c;

    const double *E = J.grid + (long long)(st.T & 1) * d * row;
    for (int e = tid; e < d * row; e += bs) sE[e] = (T)E[e];
    for (int e = tid; e < dN; e += bs) sH[e] = (HT)0;
    __syncthreads();

    const T *p0 = param_ptr<T>(J, 0);
    const T *p1 = param_ptr<T>(J, 1);
    double S1 = 0.0, S2 = 0.0;
    switch (J.family) {
      case GAUSSIAN: sample_tile<T, HT, GAUSSIAN, NB, ILP, POW2>(J, st.T, i0, cnt, sE, sH, p0, p1, S1, S2); break;
      case OSCILLATORY: sample_tile<T, HT, OSCILLATORY, NB, ILP, POW2>(J, st.T, i0, cnt, sE, sH, p0, p1, S1, S2); break;
      case PRODUCT_PEAK: sample_tile<T, HT, PRODUCT_PEAK, NB, ILP, POW2>(J, st.T, i0, cnt, sE, sH, p0, p1, S1, S2); break;
      case CORNER_PEAK: sample_tile<T, HT, CORNER_PEAK, NB, ILP, POW2>(J, st.T, i0, cnt, sE, sH, p0, p1, S1, S2); break;
      default: sample_tile<T, HT, C0, NB, ILP, POW2>(J, st.T, i0, cnt, sE, sH, p0, p1, S1, S2); break;
    }
    S1 = wave_sum(S1);
    S2 = wave_sum(S2);
    if (lane == 0) {
      red[0][wid] = S1;
      red[1][wid] = S2;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int q = 0; q < (bs >> 6); ++q) {
        a += red[0][q];
        b += red[1][q];
      }
      J.tsums[2 * lt] = a;
      J.tsums[2 * lt + 1] = b;
    }
    double *th = J.thist + (long long)lt * dN;
    for (int e = tid; e < dN; e += bs) th[e] = (double)sH[e];

    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// a7: lower regularized incomplete gamma P(a, x) for the chi^2 probability,
// by its power series below a+1 and Legendre's continued fraction for Q = 1-P
// above (Abramowitz & Stegun 6.5.29, 6.5.31; Lentz's evaluation).

__device__ double gamma_p(double a, double x) {
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

// Fold the per-tile partials of every running integral: one wavefront per
// (integral, group of kGroupTiles tiles, 64-bin chunk) sums the group's tile
// rows in tile order; the chunk-0 wave of a group also folds the tile sums.
__global__ void __launch_bounds__(256) vegas_fold_kernel(FoldArgs F) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long g = (long long)blockIdx.x * 4 + w;
  if (g >= F.total) return;  // whole waves only; no block barrier here
  int lo = 0, hi = F.njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (F.task_end[mid] > g)
      hi = mid;
    else
      lo = mid + 1;
  }
  const VJob &J = F.jobs[lo];
  if (J.state->done) return;
  const long long local = g - (lo > 0 ? F.task_end[lo - 1] : 0);
  const int dN = J.ndim * J.nbins, nch = (dN + 63) >> 6;
  const int grp = (int)(local / nch), ch = (int)(local - (long long)grp * nch);
  const int t0 = grp * kGroupTiles, t1 = min(t0 + kGroupTiles, J.ntiles);
  const int bin = ch * 64 + lane;
  if (bin < dN) {
    const double *src = J.thist + (long long)t0 * dN + bin;
    double s = 0.0;
#pragma unroll 8
    for (int t = t0; t < t1; ++t, src += dN) s += *src;
    J.ghist[(long long)grp * dN + bin] = s;
  }
  if (ch == 0 && lane < 2) {
    double s = 0.0;
    for (int t = t0; t < t1; ++t) s += J.tsums[2 * t + lane];
    J.gsums[2 * grp + lane] = s;
  }
}

// Second fold level: one wavefront per (integral, 64-bin chunk) sums the
// group rows in group order into hsum = (S1, S2, H[d*N]).
__global__ void __launch_bounds__(256) vegas_fold2_kernel(FoldArgs F) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long g = (long long)blockIdx.x * 4 + w;
  if (g >= F.total2) return;
  int lo = 0, hi = F.njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (F.task_end2[mid] > g)
      hi = mid;
    else
      lo = mid + 1;
  }
  const VJob &J = F.jobs[lo];
  if (J.state->done) return;
  const int ch = (int)(g - (lo > 0 ? F.task_end2[lo - 1] : 0));
  const int dN = J.ndim * J.nbins, ng = ngroups_of(J.ntiles);
  const int bin = ch * 64 + lane;
  if (bin < dN) {
    const double *src = J.ghist + bin;
    double s = 0.0;
#pragma unroll 8
    for (int q = 0; q < ng; ++q, src += dN) s += *src;
    J.hsum[2 + bin] = s;
  }
  if (ch == 0 && lane < 2) {
    double s = 0.0;
    for (int q = 0; q < ng; ++q) s += J.gsums[2 * q + lane];
    J.hsum[lane] = s;
  }
}

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

// One workgroup per integral: finish the iteration (a7).  Thread 0 forms the
// iteration's estimate and variance, the inverse-variance combination and
// the convergence decision; chi^2 and its probability are formed only once
// the integral is done (no intermediate value is ever observed).  Then, if
// the grid is to be refined, each wavefront takes whole dimensions: the
// histogram row is smoothed, damped and prefix-summed with wave-wide scans
// (lanes own contiguous runs of bins), and every new edge is placed by a
// binary search of the prefix sums.
__global__ void __launch_bounds__(1024) vegas_refine_kernel(VegasArgs A) {
  extern __shared__ __align__(16) double rsm[];
  __shared__ int s_mode;
  const int jb = blockIdx.x, tid = threadIdx.x, bs = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nwv = bs >> 6;
  const VJob J = A.jobs[jb];
  VState st = *J.state;
  if (st.done) return;
  const int d = J.ndim, N = J.nbins, dN = d * N, row = N + 1;
  const int t = st.T;
  double *H = rsm;       // histogram, later prefix sums of m
  double *D = rsm + dN;  // smoothed histogram, later m
  for (int e = tid; e < dN; e += bs) H[e] = J.hsum[2 + e];
  if (tid == 0) {
    const long long n = J.nstart + (long long)t * J.nincrease;
    const double S1 = J.hsum[0], S2 = J.hsum[1];
    const double I = S1 / (double)n;
    double var = S2 / (double)n - I * I;
    if (var < 0.0) var = 0.0;
    var /= (double)(n - 1);
    double *hI = J.iter_I, *hV = J.iter_var;
    hI[t] = I;
    hV[t] = var;
    const int T = t + 1;
    st.T = T;
    st.neval += n;
    // inverse-variance combination over all iterations (running sums, added
    // in iteration order)
    if (var == 0.0) {
      st.nzero += 1;
      st.sum_zI += I;
    } else {
      st.sum_w += 1.0 / var;
      st.sum_wI += I / var;
    }
    const int nz = st.nzero;
    st.dof = T - 1;
    if (nz > 0) {
      st.integral = st.sum_zI / nz;
      st.error = 0.0;
    } else {
      st.integral = st.sum_wI / st.sum_w;
      st.error = sqrt(1.0 / st.sum_w);
    }
    const double tol = fmax(J.epsabs, J.epsrel * fabs(st.integral));
    const bool conv = st.neval >= J.mineval && st.error <= tol;
    const long long nnext = J.nstart + (long long)T * J.nincrease;
    if (conv) {
      st.done = 1;
      st.fail = 0;
    } else if (st.neval + nnext > J.maxeval || T >= J.hist_cap || nnext >= (1ll << 32)) {
      st.done = 1;
      st.fail = 1;
    }
    st.chi2 = 0.0;
    st.prob = 0.0;
    if (st.done && nz == 0) {
      double chi2 = 0.0;
      for (int q = 0; q < T; ++q) {
        const double dl = hI[q] - st.integral;
        chi2 += dl * dl / hV[q];
      }
      st.chi2 = chi2;
      st.prob = st.dof > 0 ? gamma_p(0.5 * st.dof, 0.5 * chi2) : 0.0;
    }
    *J.state = st;
    s_mode = conv ? 0 : ((J.flags & FLAG_FREEZE_GRID) ? 2 : 1);
  }
  __syncthreads();
  const int mode = s_mode;
  if (mode == 0) return;
  const double *Eold = J.grid + (long long)(t & 1) * d * row;
  double *Enew = J.grid + (long long)((t + 1) & 1) * d * row;
  if (mode == 2) {
    for (int e = tid; e < d * row; e += bs) Enew[e] = Eold[e];
    return;
  }
  const int per = (N + 63) >> 6;  // contiguous bins per lane
  for (int j = wv; j < d; j += nwv) {
    double *h = H + j * N, *dd = D + j * N;
    const double *Eo = Eold + j * row;
    double *En = Enew + j * row;
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
    if (!(hs > 0.0)) {
      for (int i = lane; i <= N; i += 64) En[i] = Eo[i];
      continue;
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
      else
        m = pow((r - 1.0) / log(r), 1.5);
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
    // new edge i: smallest old bin k with C_k >= i * share
    for (int i = lane; i <= N; i += 64) {
      if (i == 0 || i == N) {
        En[i] = i == 0 ? 0.0 : 1.0;
        continue;
      }
      const double target = i * share;
      int lo = 0, hi = N - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (h[mid] < target)
          lo = mid + 1;
        else
          hi = mid;
      }
      const double before = lo > 0 ? h[lo - 1] : 0.0;
      En[i] = Eo[lo] + (target - before) / dd[lo] * (Eo[lo + 1] - Eo[lo]);
    }
  }
}

// Copy out every job's folded iteration totals: sums[2] and hist[d*N]; used by
// the raw DoSample entry point.
__global__ void __launch_bounds__(256) vegas_collect_kernel(VegasArgs A, double *sums,
                                                            double *hist) {
  const int jb = blockIdx.x, tid = threadIdx.x;
  const VJob J = A.jobs[jb];
  const int dN = J.ndim * J.nbins;
  if (tid < 2) sums[2 * jb + tid] = J.hsum[tid];
  for (int e = tid; e < dN; e += blockDim.x) hist[e] = J.hsum[2 + e];
}

// Debug/parity kernel: the points of one iteration (a1-a3), with the grid
// staged in LDS in the working precision exactly as DoSample stages it.
template <typename T>
__global__ void __launch_bounds__(256) vegas_points_kernel(PointsArgs P) {
  extern __shared__ __align__(16) unsigned char psm[];
  T *sE = (T *)psm;
  const int d = P.ndim, N = P.nbins, row = N + 1, nblk = (d + 3) >> 2;
  for (int e = threadIdx.x; e < d * row; e += blockDim.x) sE[e] = (T)P.grid[e];
  __syncthreads();
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P.npts) return;
  const uint32_t i = (uint32_t)(P.i0 + p);
  const T Nt = (T)N;
  T w = (T)1;
  for (int b = 0; b < nblk; ++b) {
    const U4 r = philox4x32_10(U4{i, ((uint32_t)P.iteration << 8) | (uint32_t)b, P.sid, 0u},
                               P.key0, P.key1);
    const uint32_t rr[4] = {r.x, r.y, r.z, r.w};
    for (int c = 0; c < 4; ++c) {
      P.words[(p * nblk + b) * 4 + c] = rr[c];
      const int j = 4 * b + c;
      if (j >= d) continue;
      T x, jac;
      int k;
      map_coord(rr[c], N, Nt, sE + j * row, x, jac, k);
      w = w * jac;
      P.x[p * d + j] = (double)x;
      P.bin[p * d + j] = k;
    }
  }
  P.w[p] = (double)w;
}

// ---------------------------------------------------------------------------
// launchers

template <int ILP, int NB, bool POW2>
static void launch_dosample_nb(const VegasArgs &A, int prec, int grid, int block, size_t lds,
                               hipStream_t s) {
  if (prec == FP64) {
    hipLaunchKernelGGL((vegas_dosample_kernel<double, double, ILP, NB, POW2>), dim3(grid),
                       dim3(block), lds, s, A);
  } else if (A.hist64) {
    hipLaunchKernelGGL((vegas_dosample_kernel<float, double, ILP, NB, POW2>), dim3(grid),
                       dim3(block), lds, s, A);
  } else {
    hipLaunchKernelGGL((vegas_dosample_kernel<float, float, ILP, NB, POW2>), dim3(grid),
                       dim3(block), lds, s, A);
  }
}

template <int ILP, bool POW2>
static void launch_dosample_ilp(const VegasArgs &A, int prec, int nb, int grid, int block,
                                size_t lds, hipStream_t s) {
  switch (nb) {
    case 1: launch_dosample_nb<ILP, 1, POW2>(A, prec, grid, block, lds, s); break;
    case 2: launch_dosample_nb<ILP, 2, POW2>(A, prec, grid, block, lds, s); break;
    case 3: launch_dosample_nb<ILP, 3, POW2>(A, prec, grid, block, lds, s); break;
    default: launch_dosample_nb<ILP, 4, POW2>(A, prec, grid, block, lds, s); break;
  }
}

hipError_t launch_dosample(const VegasArgs &A, int prec, int nb, bool pow2, int grid, int block,
                           size_t lds, hipStream_t s) {
  if (A.tile_count <= 0 || grid <= 0) return hipSuccess;
  if (A.ilp == 2) {
    if (pow2)
      launch_dosample_ilp<2, true>(A, prec, nb, grid, block, lds, s);
    else
      launch_dosample_ilp<2, false>(A, prec, nb, grid, block, lds, s);
  } else {
    if (pow2)
      launch_dosample_ilp<1, true>(A, prec, nb, grid, block, lds, s);
    else
      launch_dosample_ilp<1, false>(A, prec, nb, grid, block, lds, s);
  }
  return hipGetLastError();
}

hipError_t launch_fold(const FoldArgs &F, hipStream_t s) {
  if (F.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(vegas_fold_kernel, dim3((unsigned)((F.total + 3) / 4)), dim3(256), 0, s, F);
  hipLaunchKernelGGL(vegas_fold2_kernel, dim3((unsigned)((F.total2 + 3) / 4)), dim3(256), 0, s,
                     F);
  return hipGetLastError();
}

hipError_t launch_refine(const VegasArgs &A, int njobs, size_t lds, hipStream_t s) {
  // one wavefront per dimension (up to 16)
  hipLaunchKernelGGL(vegas_refine_kernel, dim3(njobs), dim3(1024), lds, s, A);
  return hipGetLastError();
}

hipError_t launch_collect(const VegasArgs &A, int njobs, double *sums, double *hist,
                          hipStream_t s) {
  hipLaunchKernelGGL(vegas_collect_kernel, dim3(njobs), dim3(256), 0, s, A, sums, hist);
  return hipGetLastError();
}

hipError_t launch_points(const PointsArgs &P, hipStream_t s) {
  const int block = 256;
  const long long grid = (P.npts + block - 1) / block;
  if (grid == 0) return hipSuccess;
  const size_t row = (size_t)P.ndim * (P.nbins + 1);
  if (P.prec == FP64)
    hipLaunchKernelGGL(vegas_points_kernel<double>, dim3((unsigned)grid), dim3(block),
                       row * sizeof(double), s, P);
  else
    hipLaunchKernelGGL(vegas_points_kernel<float>, dim3((unsigned)grid), dim3(block),
                       row * sizeof(float), s, P);
  return hipGetLastError();
}

hipError_t set_kernel_limits() {
  // allow the large-grid cases (d = 16, 256 bins: ~65 KB) the LDS gfx950 has;
  // a runtime that refuses keeps its default limit and such launches report
  // an error instead of running
  const int big = 160 * 1024;
  std::vector<const void *> fns = {
      (const void *)vegas_dosample_kernel<double, double, 1, 4, true>,
      (const void *)vegas_dosample_kernel<float, double, 1, 4, true>,
      (const void *)vegas_dosample_kernel<float, float, 1, 4, true>,
      (const void *)vegas_dosample_kernel<double, double, 2, 4, true>,
      (const void *)vegas_dosample_kernel<float, double, 2, 4, true>,
      (const void *)vegas_dosample_kernel<float, float, 2, 4, true>,
      (const void *)vegas_dosample_kernel<double, double, 1, 4, false>,
      (const void *)vegas_dosample_kernel<float, double, 1, 4, false>,
      (const void *)vegas_dosample_kernel<float, float, 1, 4, false>,
      (const void *)vegas_dosample_kernel<double, double, 2, 4, false>,
      (const void *)vegas_dosample_kernel<float, double, 2, 4, false>,
      (const void *)vegas_dosample_kernel<float, float, 2, 4, false>,
      (const void *)vegas_refine_kernel};
  for (const void *f : fns)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big) != hipSuccess)
      (void)hipGetLastError();
  return hipSuccess;
}

}  // namespace ccuba
