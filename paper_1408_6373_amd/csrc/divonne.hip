// divonne.hip -- Divonne's partitioning phase on gfx950 (Sect. 2.2).
//
// Spread(r) = 1/2 Vol(r) (sup_r f - inf_r f).  One step:
//   topk    the K regions of largest spread (the Suave selection kernel)
//   split   per selected region, one wavefront: d probes f(xmax with
//           x_j := xmin_j); the cut goes through the midpoint of the
//           dimension of largest loss fmax - f_j; the two children
//   search  per child, one workgroup of two wavefronts: both evaluate the
//           nsearch Philox points of the child and reduce to the largest and
//           smallest value (ties to the lower index); then wave 0 climbs to
//           the maximum and wave 1 descends to the minimum by compass search,
//           lane c < 2d evaluating candidate c (x +- h_j e_j, clipped) each
//           iteration; a move is taken when the best candidate (ties to the
//           lower c) beats the current value, else every step halves
//   totals  the largest and the total spread over all regions (fixed order)
// The host reads the totals after each step and sizes the next.
#include "divonne.h"
#include "genz.h"
#include "philox.h"

namespace ccuba {

namespace {

template <int FAM>
__device__ __forceinline__ double eval_at(const double *x, int d, const double *p0,
                                          const double *p1) {
  double acc = Genz<double, FAM>::init(p1[0]);
  for (int j = 0; j < d; ++j) acc = Genz<double, FAM>::step(acc, x[j], p0[j], p1[j]);
  return Genz<double, FAM>::finish(acc, d);
}

// one DPP step of the reduction below: each lane compares itself with the
// lane the control selects (lanes without a source compare with themselves)
template <int CTRL, int ROWS, int BANKS>
__device__ __forceinline__ void best_step(double &v, int &idx, double sign) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, ROWS, BANKS, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, ROWS, BANKS,
                                             false);
  const int oi = __builtin_amdgcn_update_dpp(idx, idx, CTRL, ROWS, BANKS, false);
  const double ov = __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  if (sign * ov > sign * v || (ov == v && oi < idx)) {
    v = ov;
    idx = oi;
  }
}

// (value, index) reduction over a wavefront: the larger sign*value, ties to
// the lower index; every lane gets the winner.  "Best of" is idempotent, so
// the DPP pattern may count a lane twice: row shifts by 1, 2, 4 and 8 leave
// each row's best in its lane 15, the row broadcasts carry it to lane 63,
// whose result readlane hands to every lane.
__device__ __forceinline__ void wave_best(double &v, int &idx, double sign) {
  best_step<0x111, 0xf, 0xf>(v, idx, sign);  // row_shr:1
  best_step<0x112, 0xf, 0xf>(v, idx, sign);  // row_shr:2
  best_step<0x114, 0xf, 0xf>(v, idx, sign);  // row_shr:4
  best_step<0x118, 0xf, 0xf>(v, idx, sign);  // row_shr:8
  best_step<0x142, 0xa, 0xf>(v, idx, sign);  // row_bcast:15 into rows 1 and 3
  best_step<0x143, 0xc, 0xf>(v, idx, sign);  // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  v = __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  idx = __builtin_amdgcn_readlane(idx, 63);
}

}  // namespace

__global__ void __launch_bounds__(64) div_root_kernel(DivArgs A) {
  if (threadIdx.x < A.d) {
    A.R.lo[threadIdx.x] = 0.0;
    A.R.hi[threadIdx.x] = 1.0;
  }
  if (threadIdx.x == 0) {
    A.chpos[0] = 0;
    A.chser[0] = 0;
  }
}

// a double of lane l (l wave-uniform) to every lane
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// D = 4 NB coordinates in registers (d <= D): the point and the steps of the
// compass search live in every lane, and a move is broadcast from the
// winning lane, so an iteration needs no LDS and no barrier.
template <int FAM, int NB>
__global__ void __launch_bounds__(kDivBlock) div_search_kernel(DivArgs A) {
  constexpr int D = 4 * NB;
  __shared__ double sLo[kMaxDim], sW[kMaxDim], sP0[kMaxDim], sP1[kMaxDim];
  __shared__ double sv[2][2], sF[2];
  __shared__ int si[2][2];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int pos = A.chpos[c], q = A.chser[c], d = A.d;
  if (tid < d) {
    const double lo = A.R.lo[(size_t)pos * d + tid];
    sLo[tid] = lo;
    sW[tid] = A.R.hi[(size_t)pos * d + tid] - lo;
    sP0[tid] = A.p64[tid];
    sP1[tid] = A.p64[kParamRow + tid];
  }
  __syncthreads();
  double p0[D], p1[D], lo[D], wd[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    p0[j] = j < d ? sP0[j] : 0.0;
    p1[j] = j < d ? sP1[j] : 0.0;
    lo[j] = j < d ? sLo[j] : 0.0;
    wd[j] = j < d ? sW[j] : 0.0;
  }
  // the point of search-sample index i
  auto point = [&](int i, double (&x)[D]) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const U4 W = philox4x32_10(U4{(uint32_t)i, ((uint32_t)q << 8) | (uint32_t)b, A.sid, 0u},
                                 A.key0, A.key1);
      const uint32_t r[4] = {W.x, W.y, W.z, W.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) x[4 * b + k] = fma((double)r[k] * 0x1p-32 + 0x1p-33,
                                                      wd[4 * b + k], lo[4 * b + k]);
    }
  };
  auto value = [&](const double (&x)[D]) {
    double acc = Genz<double, FAM>::init(p1[0]);
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) acc = Genz<double, FAM>::step(acc, x[j], p0[j], p1[j]);
    return Genz<double, FAM>::finish(acc, d);
  };
  // the search sample
  double bmax = -INFINITY, bmin = INFINITY;
  int imax = 0x7fffffff, imin = 0x7fffffff;
  for (int i = tid; i < A.nsearch; i += kDivBlock) {
    double x[D];
    point(i, x);
    const double f = value(x);
    if (f > bmax) {  // i grows, so a tie keeps the lower index
      bmax = f;
      imax = i;
    }
    if (f < bmin) {
      bmin = f;
      imin = i;
    }
  }
  wave_best(bmax, imax, 1.0);
  wave_best(bmin, imin, -1.0);
  if (lane == 0) {
    sv[w][0] = bmax;
    si[w][0] = imax;
    sv[w][1] = bmin;
    si[w][1] = imin;
  }
  __syncthreads();
  // wave 0 searches the maximum, wave 1 the minimum, from the sample's best
  const int k = w;
  const double sign = k == 0 ? 1.0 : -1.0;
  double fx;
  int i0;
  {
    const double v0 = sv[0][k], v1 = sv[1][k];
    const int j0 = si[0][k], j1 = si[1][k];
    const bool second = sign * v1 > sign * v0 || (v1 == v0 && j1 < j0);
    fx = second ? v1 : v0;
    i0 = __builtin_amdgcn_readfirstlane(second ? j1 : j0);
  }
  double x[D], h[D];
  point(i0, x);
#pragma unroll
  for (int j = 0; j < D; ++j) h[j] = wd[j] / 4.0;
  // lane c < 2d owns candidate c: coordinate jc = c/2, + for even c
  const int jc = lane >> 1;
  const bool plus = (lane & 1) == 0, live = lane < 2 * d;
  double loj = 0.0, hij = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (j == jc) {
      loj = lo[j];
      hij = lo[j] + wd[j];
    }
  for (int t = 0; t < A.niter; ++t) {
    double xj = 0.0, hj = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j == jc) {
        xj = x[j];
        hj = h[j];
      }
    const double zc = fmin(fmax(plus ? xj + hj : xj - hj, loj), hij);
    double acc = Genz<double, FAM>::init(p1[0]);
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) acc = Genz<double, FAM>::step(acc, j == jc ? zc : x[j], p0[j], p1[j]);
    double bv = live ? Genz<double, FAM>::finish(acc, d) : sign * -INFINITY;
    int bi = live ? lane : 0x7fffffff;
    wave_best(bv, bi, sign);
    if (sign * bv > sign * fx) {
      const int win = __builtin_amdgcn_readfirstlane(bi);
      const double znew = readlane_d(zc, win);
      const int jw = win >> 1;
      fx = bv;
#pragma unroll
      for (int j = 0; j < D; ++j) x[j] = j == jw ? znew : x[j];
    } else {
#pragma unroll
      for (int j = 0; j < D; ++j) h[j] *= 0.5;
    }
  }
  double* xo = (k == 0 ? A.R.xmax : A.R.xmin) + (size_t)pos * d;
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (j < d && lane == j) xo[j] = x[j];
  if (lane == 0) {
    (k == 0 ? A.R.fmax : A.R.fmin)[pos] = fx;
    sF[k] = fx;
  }
  __syncthreads();
  if (tid == 0) {
    double V = 1.0;
    for (int j = 0; j < d; ++j) V *= sW[j];
    A.R.spread[pos] = 0.5 * V * (sF[0] - sF[1]);
  }
}

// Per selected region (one wavefront): the cut and the two children.
template <int FAM>
__global__ void __launch_bounds__(64) div_split_kernel(DivArgs A, int R, long long Q) {
  __shared__ double sXmax[kMaxDim], sXmin[kMaxDim], sP0[kMaxDim], sP1[kMaxDim];
  const int s = blockIdx.x, lane = threadIdx.x, d = A.d;
  const int pos = A.sel[s], up = R + s;
  if (lane < d) {
    sXmax[lane] = A.R.xmax[(size_t)pos * d + lane];
    sXmin[lane] = A.R.xmin[(size_t)pos * d + lane];
    sP0[lane] = A.p64[lane];
    sP1[lane] = A.p64[kParamRow + lane];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const double fmax = A.R.fmax[pos];
  double loss = -INFINITY;
  int idx = 0x7fffffff;
  if (lane < d) {
    double acc = Genz<double, FAM>::init(sP1[0]);
    for (int j = 0; j < d; ++j)
      acc = Genz<double, FAM>::step(acc, j == lane ? sXmin[j] : sXmax[j], sP0[j], sP1[j]);
    loss = fmax - Genz<double, FAM>::finish(acc, d);
    idx = lane;
  }
  wave_best(loss, idx, 1.0);
  const int c = idx;
  if (lane < d) {
    const double lo = A.R.lo[(size_t)pos * d + lane], hi = A.R.hi[(size_t)pos * d + lane];
    const double mid = 0.5 * (lo + hi);
    A.R.lo[(size_t)up * d + lane] = lane == c ? mid : lo;
    A.R.hi[(size_t)up * d + lane] = hi;
    if (lane == c) A.R.hi[(size_t)pos * d + lane] = mid;
  }
  if (lane == 0) {
    A.cut[Q + s] = c;
    A.chpos[2 * s] = pos;
    A.chpos[2 * s + 1] = up;
    A.chser[2 * s] = (int)(2 * (Q + s) + 1);
    A.chser[2 * s + 1] = (int)(2 * (Q + s) + 2);
  }
}

// The largest and the total spread over the R regions (fixed order).
__global__ void __launch_bounds__(1024) div_totals_kernel(DivArgs A, int R) {
  __shared__ double rs[16], rm[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int chunk = (R + 1023) / 1024;
  const int b0 = min(tid * chunk, R), b1 = min(b0 + chunk, R);
  double sum = 0.0, mx = 0.0;
  for (int i = b0; i < b1; ++i) {
    const double v = A.R.spread[i];
    sum += v;
    mx = fmax(mx, v);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_xor(sum, o, 64);
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  if (lane == 0) {
    rs[w] = sum;
    rm[w] = mx;
  }
  __syncthreads();
  if (tid == 0) {
    double S = 0.0, M = 0.0;
    for (int q = 0; q < 16; ++q) {
      S += rs[q];
      M = fmax(M, rm[q]);
    }
    A.state->max_spread = M;
    A.state->total_spread = S;
  }
}

// ---- launchers ---------------------------------------------------------------

hipError_t launch_div_root(const DivArgs &A, hipStream_t s) {
  hipLaunchKernelGGL(div_root_kernel, dim3(1), dim3(64), 0, s, A);
  return hipGetLastError();
}

#define CCUBA_DIV_FAMILY_SWITCH(KERNEL, GRID, BLOCK, ...)                               \
  switch (A.family) {                                                                   \
    case GAUSSIAN:                                                                      \
      hipLaunchKernelGGL(KERNEL<GAUSSIAN>, GRID, BLOCK, 0, s, __VA_ARGS__);             \
      break;                                                                            \
    case OSCILLATORY:                                                                   \
      hipLaunchKernelGGL(KERNEL<OSCILLATORY>, GRID, BLOCK, 0, s, __VA_ARGS__);          \
      break;                                                                            \
    case PRODUCT_PEAK:                                                                  \
      hipLaunchKernelGGL(KERNEL<PRODUCT_PEAK>, GRID, BLOCK, 0, s, __VA_ARGS__);         \
      break;                                                                            \
    case CORNER_PEAK:                                                                   \
      hipLaunchKernelGGL(KERNEL<CORNER_PEAK>, GRID, BLOCK, 0, s, __VA_ARGS__);          \
      break;                                                                            \
    default:                                                                            \
      hipLaunchKernelGGL(KERNEL<C0>, GRID, BLOCK, 0, s, __VA_ARGS__);                   \
      break;                                                                            \
  }

template <int NB>
static void launch_search_nb(const DivArgs &A, int nchild, hipStream_t s) {
  switch (A.family) {
    case GAUSSIAN:
      hipLaunchKernelGGL((div_search_kernel<GAUSSIAN, NB>), dim3(nchild), dim3(kDivBlock), 0, s, A);
      break;
    case OSCILLATORY:
      hipLaunchKernelGGL((div_search_kernel<OSCILLATORY, NB>), dim3(nchild), dim3(kDivBlock), 0, s,
                         A);
      break;
    case PRODUCT_PEAK:
      hipLaunchKernelGGL((div_search_kernel<PRODUCT_PEAK, NB>), dim3(nchild), dim3(kDivBlock), 0, s,
                         A);
      break;
    case CORNER_PEAK:
      hipLaunchKernelGGL((div_search_kernel<CORNER_PEAK, NB>), dim3(nchild), dim3(kDivBlock), 0, s,
                         A);
      break;
    default:
      hipLaunchKernelGGL((div_search_kernel<C0, NB>), dim3(nchild), dim3(kDivBlock), 0, s, A);
      break;
  }
}

hipError_t launch_div_search(const DivArgs &A, int nchild, hipStream_t s) {
  switch ((A.d + 3) / 4) {
    case 1:
      launch_search_nb<1>(A, nchild, s);
      break;
    case 2:
      launch_search_nb<2>(A, nchild, s);
      break;
    case 3:
      launch_search_nb<3>(A, nchild, s);
      break;
    default:
      launch_search_nb<4>(A, nchild, s);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_div_split(const DivArgs &A, int R, long long Q, int K, hipStream_t s) {
  CCUBA_DIV_FAMILY_SWITCH(div_split_kernel, dim3(K), dim3(64), A, R, Q)
  return hipGetLastError();
}

#undef CCUBA_DIV_FAMILY_SWITCH

hipError_t launch_div_totals(const DivArgs &A, int R, hipStream_t s) {
  hipLaunchKernelGGL(div_totals_kernel, dim3(1), dim3(1024), 0, s, A, R);
  return hipGetLastError();
}

}  // namespace ccuba
