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

// Sample the points [i0, i0 + cnt) of one tile; lane sums go to S1, S2.
// NB = ceil(d/4) Philox blocks per point is a template argument so that the
// per-dimension loop is fully unrolled with only the last block guarded.
template <typename T, typename HT, int FAM, int NB>
__device__ __forceinline__ void sample_tile(const VJob &J, int t, long long i0, int cnt,
                                            const T *__restrict__ sE, HT *sH,
                                            const T *__restrict__ p0,
                                            const T *__restrict__ p1, double &S1,
                                            double &S2) {
  const int d = J.ndim, N = J.nbins, row = N + 1;
  const T Nt = (T)N;
  const uint32_t c1 = (uint32_t)t << 8;
  const uint32_t sid = J.sid, k0 = J.key0, k1 = J.key1;
  T pp0[4 * NB], pp1[4 * NB];
#pragma unroll
  for (int j = 0; j < 4 * NB; ++j) {  // parameter rows are zero-padded to 16
    pp0[j] = p0[j];
    pp1[j] = p1[j];
  }
  const T phase0 = p1[0];
  for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
    const uint32_t i = (uint32_t)(i0 + q);
    T w = (T)1;
    T acc = Genz<T, FAM>::init(phase0);
    uint32_t kp[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      kp[b] = 0;
      const U4 r = philox4x32_10(U4{i, c1 | (uint32_t)b, sid, 0u}, k0, k1);
      const uint32_t rr[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int j = 4 * b + c;
        if (b < NB - 1 || j < d) {
          T x, jac;
          int k;
          map_coord(rr[c], N, Nt, sE + j * row, x, jac, k);
          w = w * jac;
          acc = Genz<T, FAM>::step(acc, x, pp0[j], pp1[j]);
          kp[b] |= (uint32_t)k << (8 * c);
        }
      }
    }
    const T f = Genz<T, FAM>::finish(acc, d);
    const T v = w * f;
    const double vd = (double)v;
    S1 += vd;
    S2 = fma(vd, vd, S2);
    const HT v2 = (HT)(v * v);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int j = 4 * b + c;
        if (b < NB - 1 || j < d) unsafeAtomicAdd(&sH[j * N + ((kp[b] >> (8 * c)) & 255u)], v2);
      }
    }
  }
}

template <typename T, typename HT, int FAM>
__device__ __forceinline__ void sample_tile_nb(const VJob &J, int t, long long i0, int cnt,
                                               const T *sE, HT *sH, const T *p0, const T *p1,
                                               double &S1, double &S2) {
  switch ((J.ndim + 3) >> 2) {
    case 1: sample_tile<T, HT, FAM, 1>(J, t, i0, cnt, sE, sH, p0, p1, S1, S2); break;
    case 2: sample_tile<T, HT, FAM, 2>(J, t, i0, cnt, sE, sH, p0, p1, S1, S2); break;
    case 3: sample_tile<T, HT, FAM, 3>(J, t, i0, cnt, sE, sH, p0, p1, S1, S2); break;
    default: sample_tile<T, HT, FAM, 4>(J, t, i0, cnt, sE, sH, p0, p1, S1, S2); break;
  }
}

template <typename T, typename HT>
__global__ void __launch_bounds__(256) vegas_dosample_kernel(VegasArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[2][4];
  __shared__ int s_last;
  T *sE = (T *)smem;
  HT *sH = (HT *)(smem + A.lds_hist_byte_off);
  const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wid = tid >> 6;
  const int myprec = sizeof(T) == 8 ? FP64 : FP32;

  for (int tt = blockIdx.x; tt < A.ntiles; tt += gridDim.x) {
    const int jb = A.tile_job[tt];
    const VJob J = A.jobs[jb];
    if (J.prec != myprec) continue;
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
      case GAUSSIAN: sample_tile_nb<T, HT, GAUSSIAN>(J, st.T, i0, cnt, sE, sH, p0, p1, S1, S2); break;
      case OSCILLATORY: sample_tile_nb<T, HT, OSCILLATORY>(J, st.T, i0, cnt, sE, sH, p0, p1, S1, S2); break;
      case PRODUCT_PEAK: sample_tile_nb<T, HT, PRODUCT_PEAK>(J, st.T, i0, cnt, sE, sH, p0, p1, S1, S2); break;
      case CORNER_PEAK: sample_tile_nb<T, HT, CORNER_PEAK>(J, st.T, i0, cnt, sE, sH, p0, p1, S1, S2); break;
      default: sample_tile_nb<T, HT, C0>(J, st.T, i0, cnt, sE, sH, p0, p1, S1, S2); break;
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

    // fold the 32-tile group once its last tile is written
    const int g = lt / kGroupTiles, gfirst = g * kGroupTiles;
    const int gsize = min(kGroupTiles, J.ntiles - gfirst);
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      const unsigned old = atomicAdd(&J.gcnt[g], 1u);
      s_last = (old == (unsigned)(gsize - 1));
    }
    __syncthreads();
    if (s_last) {
      __threadfence();
      if (tid == 0) {
        atomicExch(&J.gcnt[g], 0u);
        double a = 0.0, b = 0.0;
        for (int q = 0; q < gsize; ++q) {
          const long long ti = gfirst + q;
          a += __hip_atomic_load(&J.tsums[2 * ti], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          b += __hip_atomic_load(&J.tsums[2 * ti + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        J.gsums[2 * g] = a;
        J.gsums[2 * g + 1] = b;
      }
      const double *src = J.thist + (long long)gfirst * dN;
      double *dst = J.ghist + (long long)g * dN;
      for (int e = tid; e < dN; e += bs) {
        double s = 0.0;
        for (int q = 0; q < gsize; ++q)
          s += __hip_atomic_load(&src[(long long)q * dN + e], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        dst[e] = s;
      }
    }
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

// One workgroup per integral: finish the iteration, combine, decide, refine.
__global__ void __launch_bounds__(256) vegas_refine_kernel(VegasArgs A) {
  extern __shared__ __align__(16) double rsm[];
  __shared__ int s_refine;
  __shared__ double s_share[kMaxDim], s_dsum[kMaxDim];
  __shared__ int s_has[kMaxDim];
  const int jb = blockIdx.x, tid = threadIdx.x, bs = blockDim.x;
  const VJob J = A.jobs[jb];
  VState st = *J.state;
  if (st.done) return;
  const int d = J.ndim, N = J.nbins, dN = d * N, row = N + 1;
  const int t = st.T;
  const int ng = ngroups_of(J.ntiles);

  if (tid == 0) {
    const long long n = J.nstart + (long long)t * J.nincrease;
    double S1 = 0.0, S2 = 0.0;
    for (int g = 0; g < ng; ++g) {
      S1 += J.gsums[2 * g];
      S2 += J.gsums[2 * g + 1];
    }
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
    // inverse-variance combination over all iterations
    int nz = 0;
    double zs = 0.0;
    for (int q = 0; q < T; ++q)
      if (hV[q] == 0.0) {
        ++nz;
        zs += hI[q];
      }
    st.dof = T - 1;
    if (nz > 0) {
      st.integral = zs / nz;
      st.error = 0.0;
      st.chi2 = 0.0;
      st.prob = 0.0;
    } else {
      double ws = 0.0, wis = 0.0;
      for (int q = 0; q < T; ++q) {
        ws += 1.0 / hV[q];
        wis += hI[q] / hV[q];
      }
      st.integral = wis / ws;
      st.error = sqrt(1.0 / ws);
      double chi2 = 0.0;
      for (int q = 0; q < T; ++q) {
        const double dl = hI[q] - st.integral;
        chi2 += dl * dl / hV[q];
      }
      st.chi2 = chi2;
      st.prob = st.dof > 0 ? gamma_p(0.5 * st.dof, 0.5 * chi2) : 0.0;
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
    *J.state = st;
    s_refine = conv ? 0 : ((J.flags & FLAG_FREEZE_GRID) ? 2 : 1);
  }
  __syncthreads();
  const int mode = s_refine;
  if (mode == 0) return;
  const double *Eold = J.grid + (long long)(t & 1) * d * row;
  double *Enew = J.grid + (long long)((t + 1) & 1) * d * row;
  if (mode == 2) {
    for (int e = tid; e < d * row; e += bs) Enew[e] = Eold[e];
    return;
  }
  double *H = rsm;        // histogram, later prefix sums of m
  double *D = rsm + dN;   // smoothed histogram, later m
  for (int e = tid; e < dN; e += bs) {
    double s = 0.0;
    for (int g = 0; g < ng; ++g) s += J.ghist[(long long)g * dN + e];
    H[e] = s;
  }
  __syncthreads();
  // 3-point smoothing
  for (int e = tid; e < dN; e += bs) {
    const int j = e / N, k = e - j * N;
    const double *h = H + j * N;
    double v;
    if (k == 0)
      v = (h[0] + h[1]) / 2.0;
    else if (k == N - 1)
      v = (h[N - 2] + h[N - 1]) / 2.0;
    else
      v = (h[k - 1] + h[k] + h[k + 1]) / 3.0;
    D[e] = v;
  }
  __syncthreads();
  if (tid < d) {
    double hs = 0.0, ds = 0.0;
    for (int k = 0; k < N; ++k) hs += H[tid * N + k];
    for (int k = 0; k < N; ++k) ds += D[tid * N + k];
    s_has[tid] = hs > 0.0;
    s_dsum[tid] = ds;
  }
  __syncthreads();
  // damping m_k = ((r-1)/ln r)^1.5, r = normalised smoothed histogram
  for (int e = tid; e < dN; e += bs) {
    const int j = e / N;
    if (!s_has[j]) continue;
    const double r = D[e] / s_dsum[j];
    double m;
    if (r == 0.0)
      m = 0.0;
    else if (r == 1.0)
      m = 1.0;
    else
      m = pow((r - 1.0) / log(r), 1.5);
    D[e] = m;
  }
  __syncthreads();
  if (tid < d && s_has[tid]) {
    double acc = 0.0;
    for (int k = 0; k < N; ++k) {
      acc += D[tid * N + k];
      H[tid * N + k] = acc;
    }
    s_share[tid] = acc / N;
  }
  __syncthreads();
  // new edge i of dimension j: smallest old bin k with C_k >= i * share
  for (int e = tid; e < d * row; e += bs) {
    const int j = e / row, i = e - j * row;
    const double *Eo = Eold + j * row;
    if (!s_has[j] || i == 0 || i == N) {
      Enew[e] = s_has[j] ? (i == 0 ? 0.0 : 1.0) : Eo[i];
      continue;
    }
    const double *C = H + j * N;
    const double target = i * s_share[j];
    int lo = 0, hi = N - 1;  // C[hi] >= target or hi == N-1
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (C[mid] < target)
        lo = mid + 1;
      else
        hi = mid;
    }
    const int k = lo;
    const double before = k > 0 ? C[k - 1] : 0.0;
    Enew[e] = Eo[k] + (target - before) / D[j * N + k] * (Eo[k + 1] - Eo[k]);
  }
}

// Copy out the group partials of every job as its iteration total: sums[2]
// and hist[d*N] (fixed order); used by the raw DoSample entry point.
__global__ void __launch_bounds__(256) vegas_collect_kernel(VegasArgs A, double *sums,
                                                            double *hist) {
  const int jb = blockIdx.x, tid = threadIdx.x;
  const VJob J = A.jobs[jb];
  const int dN = J.ndim * J.nbins, ng = ngroups_of(J.ntiles);
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int g = 0; g < ng; ++g) {
      a += J.gsums[2 * g];
      b += J.gsums[2 * g + 1];
    }
    sums[2 * jb] = a;
    sums[2 * jb + 1] = b;
  }
  for (int e = tid; e < dN; e += blockDim.x) {
    double s = 0.0;
    for (int g = 0; g < ng; ++g) s += J.ghist[(long long)g * dN + e];
    hist[e] = s;
  }
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

hipError_t launch_dosample(const VegasArgs &A, int prec, int grid, int block, size_t lds,
                           hipStream_t s) {
  if (prec == FP64) {
    hipLaunchKernelGGL((vegas_dosample_kernel<double, double>), dim3(grid), dim3(block), lds, s,
                       A);
  } else if (A.hist64) {
    hipLaunchKernelGGL((vegas_dosample_kernel<float, double>), dim3(grid), dim3(block), lds, s,
                       A);
  } else {
    hipLaunchKernelGGL((vegas_dosample_kernel<float, float>), dim3(grid), dim3(block), lds, s, A);
  }
  return hipGetLastError();
}

hipError_t launch_refine(const VegasArgs &A, int njobs, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(vegas_refine_kernel, dim3(njobs), dim3(256), lds, s, A);
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
  const void *fns[] = {(const void *)vegas_dosample_kernel<double, double>,
                       (const void *)vegas_dosample_kernel<float, double>,
                       (const void *)vegas_dosample_kernel<float, float>,
                       (const void *)vegas_refine_kernel};
  for (const void *f : fns)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big) != hipSuccess)
      (void)hipGetLastError();
  return hipSuccess;
}

}  // namespace ccuba
