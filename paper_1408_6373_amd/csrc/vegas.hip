// vegas.hip -- Vegas DoSample and grid refinement on gfx950.
//
// DoSample (Sect. 2.1) samples n points; the paper splits them n/N over N
// worker processes.  Here the split is over tiles of consecutive point
// indices, processed by persistent workgroups.  Each point is produced in
// registers from its Philox counter, so no sample ever crosses HBM:
//   a1 words   W_b = philox(ctr = (i, (t<<8)|b, sid, 0), key = seed)
//   a2 uniform FP64 y = r 2^-32 + 2^-33 | FP32 y = (r>>9) 2^-23 + 2^-24
//   a3 map     z = y N, k = min(floor z, N-1), x = E[k] + (z-k)(E[k+1]-E[k]),
//              w *= N (E[k+1]-E[k])     (grid cells staged in LDS per tile)
//   a4 f       Genz family, accumulated one dimension at a time
//   a5 sums    v = w f: S1 += v, S2 += v^2 in FP64 per lane, wave shuffles,
//              then a fixed-order block sum -> one FP64 partial per tile
//   a6 hist    H_j[k_j] += v^2 with LDS atomics, written per tile as FP64
// A fold kernel sums the tile rows 32 at a time in tile order and a second
// one sums those group rows in group order (so the sums are deterministic);
// the refine kernel (one workgroup per integral) then does a7: iteration
// statistics, the inverse-variance combination with chi^2 and its
// probability, the convergence test and Lepage's grid refinement, all in FP64.
// Iteration t and its point count are read from device state, so a captured
// iteration replays unchanged.
#include "engine.h"
#include "genz.h"
#include "philox.h"
#include "vegas.h"
#include "vegas_sample.h"
#include "refine.h"

#include <vector>

namespace ccuba {

static_assert(kGroupTiles % 32 == 0, "a group's tile sums fill whole wavefronts");
constexpr int kFoldBatch = kGroupTiles < 64 ? kGroupTiles : 64;  // rows in flight per lane
constexpr int kTsPer = 2 * kGroupTiles / 64;  // a group's tile sums per lane

// Fold the per-tile partials of every running integral: one wavefront per
// (integral, group of kGroupTiles tiles, 64-bin chunk) sums the group's tile
// rows in tile order; the chunk-0 wave of a group also folds the tile sums.
__global__ void __launch_bounds__(256) vegas_fold_kernel(FoldArgs F) {
  // the task index is the same for the whole wavefront: saying so makes the
  // job lookups scalar loads, issued together
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
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
  const long long base = lo > 0 ? F.task_end[lo - 1] : 0;
  const uint32_t jw = load_words<kJobWords>(F.jobs + lo, lane);
  const int dN = JOB_FIELD(jw, ndim) * JOB_FIELD(jw, nbins), nch = (dN + 63) >> 6;
  const int local = (int)(g - base);  // a job has fewer than 2^31 tasks
  const int grp = local / nch, ch = local - grp * nch;
  const int t0 = grp * kGroupTiles, nt = min(t0 + kGroupTiles, JOB_FIELD(jw, ntiles)) - t0;
  const int bin = ch * 64 + lane;
  // Every load of the wave's first batch -- the done flag, the group's tile
  // rows and, in chunk 0, the group's tile sums (kTsPer values per lane) --
  // is issued before any of them is used, so that together they are one
  // round trip to memory.  (The rows are allocated whether or not the
  // integral is done.)
  const int done = *gload(&JOB_FIELD(jw, state)->done);
  // the state as this iteration's sampling left it, for the refine launch
  VState *snap = JOB_FIELD(jw, snap);
  const uint32_t stw = (snap && grp == 0 && ch == 0)
                           ? load_words<kStateWords>(JOB_FIELD(jw, state), lane) : 0u;
  const gbl<double> *src = gload(JOB_FIELD(jw, thist)) + (long long)t0 * dN + (bin < dN ? bin : 0);
  const gbl<double> *tsp = gload(JOB_FIELD(jw, tsums)) + 2ll * t0;
  double ts[kTsPer];
#pragma unroll
  for (int k = 0; k < kTsPer; ++k)
    ts[k] = (ch == 0 && 64 * k + lane < 2 * nt) ? tsp[64 * k + lane] : 0.0;
  double s = 0.0;
  for (int q0 = 0; q0 < nt; q0 += kFoldBatch) {
    double v[kFoldBatch];
#pragma unroll
    for (int q = 0; q < kFoldBatch; ++q)
      v[q] = (bin < dN && q0 + q < nt) ? src[(long long)(q0 + q) * dN] : 0.0;
    // keeps the compiler from folding each add into its load's branch, which
    // would wait for every load before issuing the next
    asm volatile("" ::: "memory");
    if (q0 == 0 && snap && grp == 0 && ch == 0 && lane < kStateWords)
      ((uint32_t *)snap)[lane] = stw;  // (also once the integral is done)
    if (done) return;
    // tile order; the first row starts the sum (a group has at least one
    // tile; starting from 0.0 would put the first add, and a wait, inside
    // the loads)
    if (q0 == 0) s = v[0];
#pragma unroll
    for (int q = 0; q < kFoldBatch; ++q)
      if ((q0 > 0 || q > 0) && q0 + q < nt) s += v[q];
  }
  if (bin < dN) gstore(JOB_FIELD(jw, ghist))[(long long)grp * dN + bin] = s;
  if (ch == 0) {  // the tile sums in tile order, read across the lanes
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int k = 0; k < kTsPer; ++k)
      for (int q = 32 * k; q < min(nt, 32 * k + 32); ++q) {
        s1 += lane_value(ts[k], 2 * q - 64 * k);
        s2 += lane_value(ts[k], 2 * q + 1 - 64 * k);
      }
    if (lane == 0) {
      gbl<double> *gs = gstore(JOB_FIELD(jw, gsums));
      gs[2 * grp] = s1;
      gs[2 * grp + 1] = s2;
    }
  }
}

// Second fold level, for callers that want the iteration totals themselves
// (the refine kernel does this level on its own): one wavefront per
// (integral, 64-bin chunk) sums the group rows in group order into
// hsum = (S1, S2, H[d*N]).
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

// a7, the iteration's statistics for one component: the estimate I_t and
// variance sigma_t^2 of iteration t = st.T from its sums over n points,
// folded into the running inverse-variance combination (sums added in
// iteration order).  The sums are taken about c = st.shift, S1 = sum (v - c)
// and S2 = sum (v - c)^2, so I_t = c + S1/n and sigma_t^2 =
// max(0, S2/n - (S1/n)^2)/(n - 1), the same quantities as from plain sums;
// the estimate becomes the next iteration's shift.  The stop rule and chi^2
// are applied by finish_state.
__device__ __forceinline__ void settle_component(VState &st, double S1, double S2, long long n,
                                                 double &I, double &var) {
  const double m = S1 / (double)n;
  I = st.shift + m;
  var = S2 / (double)n - m * m;
  if (var < 0.0) var = 0.0;
  var /= (double)(n - 1);
  st.shift = I;
  const int T = st.T + 1;
  st.T = T;
  st.neval += n;
  if (var == 0.0) {
    st.nzero += 1;
    st.sum_zI += I;
  } else {
    st.sum_w += 1.0 / var;
    st.sum_wI += I / var;
  }
  st.dof = T - 1;
  if (st.nzero > 0) {
    st.integral = st.sum_zI / st.nzero;
    st.error = 0.0;
  } else {
    st.integral = st.sum_wI / st.sum_w;
    st.error = sqrt(1.0 / st.sum_w);
  }
}

// The stop rule's outcome (bad: the iteration's sums are not finite, which
// ends the integral with fail -4 and zero results; conv: the accuracy test
// passed; budget: the next iteration would pass maxeval) and, once done,
// chi^2 over the history hI/hV of the st.T iterations and its probability.
__device__ __forceinline__ void finish_state(VState &st, bool bad, bool conv, bool budget,
                                             const double *hI, const double *hV) {
  if (bad) {
    st.done = 1;
    st.fail = -4;
    st.integral = st.error = st.chi2 = st.prob = 0.0;
    return;
  }
  if (conv) {
    st.done = 1;
    st.fail = 0;
  } else if (budget) {
    st.done = 1;
    st.fail = 1;
  }
  st.chi2 = 0.0;
  st.prob = 0.0;
  if (st.done && st.nzero == 0) {
    double chi2 = 0.0;
    for (int q = 0; q < st.T; ++q) {
      const double dl = hI[q] - st.integral;
      chi2 += dl * dl / hV[q];
    }
    st.chi2 = chi2;
    st.prob = st.dof > 0 ? gamma_p(0.5 * st.dof, 0.5 * chi2) : 0.0;
  }
}

// One workgroup per (integral, dimension): finish the iteration (a7).  Every
// workgroup reads the state as the iteration's fold left it (the snapshot:
// the live state is rewritten by this launch) and the iteration's sums, and
// thread 0 forms the iteration's estimate and variance, the inverse-variance
// combination and the convergence decision -- the same in every workgroup of
// the integral; only dimension 0's writes the state and the history, with
// chi^2 and its probability once the integral is done (no intermediate value
// is ever observed).  Meanwhile wavefront 1 refines its dimension of the grid
// into LDS: the histogram row is smoothed, damped
// and prefix-summed with wave-wide scans (lanes own contiguous runs of
// bins), and every new edge is placed in the old bin whose prefix-sum
// interval holds its share.  The new edges are written out if the decision
// is to refine.
constexpr int kRefineThreads = 256;  // the refine kernel's block (launch_refine)

__global__ void __launch_bounds__(kRefineThreads) vegas_refine_kernel(VegasArgs A) {
  __shared__ double H[kMaxBins];      // histogram row, later prefix sums of m
  __shared__ double D[kMaxBins];      // smoothed row, later m
  __shared__ double G[kMaxBins + 1];  // the current edges
  __shared__ double Gn[kMaxBins + 1];  // the refined edges
  __shared__ int s_mode;
  __shared__ double s_sums[2];
  __shared__ __align__(16) uint32_t s_stw[kStateWords];  // the state, word by word
  // (a constant block size: reading blockDim would be one more wait)
  constexpr int bs = kRefineThreads;
  const int jb = blockIdx.x, dim = blockIdx.y, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  // Every wavefront holds the job descriptor, one word per lane.
  const uint32_t jw = load_words<kJobWords>(A.jobs + jb, lane);
  const int d = JOB_FIELD(jw, ndim), N = JOB_FIELD(jw, nbins);
  if (dim >= d) return;  // (a launch covers the largest d of its integrals)
  const int dN = d * N, row = N + 1;
  const int ng = ngroups_of(JOB_FIELD(jw, ntiles));
  double *grow = JOB_FIELD(jw, grid) + (long long)dim * row;
  const double *gsums = JOB_FIELD(jw, gsums);
  // One round trip to memory for all of: the state (a word per lane of the
  // first wavefront), the first 32 groups' sums (a value per lane), this
  // dimension's edges and its bins' group rows.  (The edges are staged in
  // LDS before any of them is rewritten.)
  const uint32_t stw = wv == 0 ? load_words<kStateWords>(JOB_FIELD(jw, snap), lane) : 0u;
  const double gsv = (tid < 2 * min(ng, 32)) ? gload(gsums)[tid] : 0.0;
  const double e0 = tid < row ? gload(grow)[tid] : 0.0;
  const double e1 = (tid == 0 && row > bs) ? gload(grow)[bs] : 0.0;
  // the last fold level: the group rows in group order (the order of the
  // separate second-level fold, so both give the same sums)
  constexpr int kBatch = 32;  // loads in flight per thread before the adds
  if (tid < N) {
    const gbl<double> *src = gload(JOB_FIELD(jw, ghist)) + (long long)dim * N + tid;
    double h = 0.0;
    for (int q0 = 0; q0 < ng; q0 += kBatch) {
      double v[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) v[q] = q0 + q < ng ? src[(long long)(q0 + q) * dN] : 0.0;
      asm volatile("" ::: "memory");  // every load of the batch before the adds
      // (the first group row starts the sum: there is at least one group)
      if (q0 == 0) h = v[0];
#pragma unroll
      for (int q = 0; q < kBatch; ++q)
        if ((q0 > 0 || q > 0) && q0 + q < ng) h += v[q];
    }
    H[tid] = h;
  }
  if (wv == 0) {
    if (lane < kStateWords) s_stw[lane] = stw;
    // the group sums in group order: the first 32 read across the lanes
    double h1 = 0.0, h2 = 0.0;
    for (int q = 0; q < min(ng, 32); ++q) {
      h1 += lane_value(gsv, 2 * q);
      h2 += lane_value(gsv, 2 * q + 1);
    }
    for (int q0 = 32; q0 < ng; q0 += kBatch) {
      double v[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q)
        v[q] = (lane < 2 && q0 + q < ng) ? gload(gsums)[2 * (q0 + q) + lane] : 0.0;
#pragma unroll
      for (int q = 0; q < kBatch; ++q)
        if (q0 + q < ng) {
          h1 += lane_value(v[q], 0);
          h2 += lane_value(v[q], 1);
        }
    }
    if (lane == 0) {
      s_sums[0] = h1;
      s_sums[1] = h2;
    }
  }
  __syncthreads();
  // (state words read as written, uint32_t; the whole state by memcpy below)
  if (s_stw[offsetof(VState, done) / 4] != 0u) return;  // the same for the whole block
  const int t = (int)s_stw[offsetof(VState, T) / 4];
  if (tid < row) G[tid] = e0;
  if (tid == 0 && row > bs) G[bs] = e1;
  __syncthreads();  // G complete
  if (wv == 1) rebin_dimension(H, D, G, Gn, N, lane);
  if (tid == 0) {
    VState st;
    __builtin_memcpy(&st, s_stw, sizeof(VState));
    const long long nstart = JOB_FIELD(jw, nstart), ninc = JOB_FIELD(jw, nincrease);
    const long long n = nstart + (long long)t * ninc;
    const double S1 = s_sums[0], S2 = s_sums[1];
    const double c = st.shift;  // the sums' shift (settle_component moves it on)
    double I, var;
    settle_component(st, S1, S2, n, I, var);
    const int T = st.T;
    const double tol = fmax(JOB_FIELD(jw, epsabs), JOB_FIELD(jw, epsrel) * fabs(st.integral));
    const bool conv = st.neval >= JOB_FIELD(jw, mineval) && st.error <= tol;
    const long long nnext = nstart + (long long)T * ninc;
    const bool budget = st.neval + nnext > JOB_FIELD(jw, maxeval) ||
                        T >= JOB_FIELD(jw, hist_cap) || nnext >= (1ll << 32);
    const bool bad = !isfinite(S1) || !isfinite(S2);
    if (dim == 0) {
      double *hI = JOB_FIELD(jw, iter_I), *hV = JOB_FIELD(jw, iter_var);
      hI[t] = I;
      hV[t] = var;
      finish_state(st, bad, conv, budget, hI, hV);
      // the mean v^2 of the iteration, (S2 + 2 c S1)/n + c^2
      st.hcap = (float)(1024.0 * (fma(2.0 * c, S1, S2) / (double)n + c * c));
      *JOB_FIELD(jw, state) = st;
    }
    s_mode = conv || bad ? 0 : ((JOB_FIELD(jw, flags) & FLAG_FREEZE_GRID) ? 2 : 1);
  }
  __syncthreads();
  if (s_mode != 1) return;  // converged, or the grid is frozen (kept as it is)
  for (int e = tid; e < row; e += bs) grow[e] = Gn[e];
}

// Uniform starting grids, E_j[k] = k/N, one workgroup per job (the same
// division the host would do, so the grids are the same).
__global__ void __launch_bounds__(256) vegas_init_grids_kernel(const VJob *jobs) {
  const VJob &J = jobs[blockIdx.x];
  const int N = J.nbins, row = N + 1, tot = J.ndim * row;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) J.grid[e] = (double)(e % row) / N;
}

__global__ void __launch_bounds__(256) vegas_init_grid_kernel(double *grid, int d, int N) {
  const int row = N + 1, tot = d * row;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) grid[e] = (double)(e % row) / N;
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

// Parity kernel: the points of one iteration (a1-a3), computed with the
// staging and the per-coordinate arithmetic of the DoSample kernel.
template <typename T>
__host__ __device__ constexpr size_t points_cells_bytes(int d, int N) {
  return ((size_t)d * N * sizeof(Cell<T>) + 15) / 16 * 16;
}
constexpr int kPointsPerThread = 4;
constexpr int kPointsBlock = 256;

// Each block makes kPointsPerThread rounds of kPointsBlock consecutive points.
// A round's coordinates and bins go through LDS, so that its rows of
// x[p][ndim] and bin[p][ndim] (contiguous in memory) are written with
// coalesced stores, not one strided element per lane.
template <typename T>
__global__ void __launch_bounds__(kPointsBlock) vegas_points_kernel(PointsArgs P) {
  extern __shared__ __align__(16) unsigned char psm[];
  const int d = P.ndim, N = P.nbins, nblk = (d + 3) >> 2;
  Cell<T> *sC = (Cell<T> *)psm;
  double *sX = (double *)(psm + points_cells_bytes<T>(d, N));  // [kPointsBlock][d]
  int *sK = (int *)(sX + kPointsBlock * d);                     // [kPointsBlock][d]
  const bool pow2 = (N & (N - 1)) == 0;
  if (pow2)
    stage_cells<T, true>(P.grid, d, N, sC);
  else
    stage_cells<T, false>(P.grid, d, N, sC);
  __syncthreads();
  const T Nt = (T)N;
  const int L = 31 - __clz(N);
  const T scale = pow2_scale<T>(L);
  const int tid = threadIdx.x;
  const long long first = (long long)blockIdx.x * kPointsBlock * kPointsPerThread;
  const long long end = min(P.npts, first + (long long)kPointsBlock * kPointsPerThread);
  for (long long base = first; base < end; base += kPointsBlock) {  // the same for the block
    const long long p = base + tid;
    if (p < end) {
      const uint32_t i = (uint32_t)(P.i0 + p);
      T w = (T)1;
      for (int b = 0; b < nblk; ++b) {
        const U4 r = philox4x32_10(U4{i, ((uint32_t)P.iteration << 8) | (uint32_t)b, P.sid, 0u},
                                   P.key0, P.key1);
        const uint32_t rr[4] = {r.x, r.y, r.z, r.w};
        for (int c = 0; c < 4; ++c) {
          if (P.words) P.words[(p * nblk + b) * 4 + c] = rr[c];
          const int j = 4 * b + c;
          if (j >= d) continue;
          T fr;
          int k;
          if (pow2)
            bin_frac_pow2(rr[c], L, scale, fr, k);
          else
            bin_frac_any(rr[c], N, Nt, fr, k);
          const Cell<T> cell = sC[j * N + k];
          const T x = fma_t(fr, cell.span, cell.lo);
          w = pow2 ? w * cell.span : w * (Nt * cell.span);
          sX[tid * d + j] = (double)x;
          sK[tid * d + j] = k;
        }
      }
      P.w[p] = (double)w;
    }
    __syncthreads();
    const int cnt = (int)(min(end - base, (long long)kPointsBlock) * d);
    for (int e = tid; e < cnt; e += kPointsBlock) {
      P.x[base * d + e] = sX[e];
      P.bin[base * d + e] = sK[e];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Caller-evaluated integrands: the integrand values f of a batch of points
// (made by the points kernel above) come from the caller; these kernels do
// the rest of the iteration on the device.

// a5/a6 over one batch: one workgroup per tile of tile_pts consecutive
// points writes one row: per component c, S1_c = sum v_c and S2_c = sum v_c^2
// with v_c = w f_c (per lane in point order, then wave and block sums in a
// fixed order), then H_j[k_j] += v_0^2 (an LDS histogram: the grid follows
// component 0).  With FP32 evaluation v_c is the binary32 product, as the
// points were made in binary32.
constexpr int kAccumThreads = 1024;

__global__ void __launch_bounds__(kAccumThreads) vegas_batched_accumulate_kernel(BatchedArgs B) {
  extern __shared__ double hs[];  // ndim * nbins
  __shared__ double red[kAccumThreads / 64][2 * kMaxComp];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int d = B.ndim, N = B.nbins, dN = d * N, nc = B.ncomp;
  const long long p0 = (long long)blockIdx.x * B.tile_pts;
  const long long p1 = min(p0 + (long long)B.tile_pts, B.npts);
  for (int e = tid; e < dN; e += blockDim.x) hs[e] = 0.0;
  __syncthreads();
  double s1[kMaxComp], s2[kMaxComp], sh[kMaxComp];
#pragma unroll
  for (int c = 0; c < kMaxComp; ++c) {
    s1[c] = s2[c] = 0.0;
    sh[c] = c < nc ? B.state[c].shift : 0.0;  // every component's sums have their own shift
  }
  for (long long p = p0 + tid; p < p1; p += blockDim.x) {
    const double w = B.w[p];
    double v0 = 0.0;
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c)
      if (c < nc) {
        const double f = B.f[p * nc + c];
        const double v = B.prec == FP32 ? (double)((float)w * (float)f) : w * f;
        const double dv = v - sh[c];
        s1[c] += dv;
        s2[c] = fma(dv, dv, s2[c]);
        if (c == 0) v0 = v;
      }
    const double v2 = v0 * v0;
    for (int j = 0; j < d; ++j) unsafeAtomicAdd(&hs[j * N + B.bin[p * d + j]], v2);
  }
#pragma unroll
  for (int c = 0; c < kMaxComp; ++c)
    if (c < nc) {
      const double a = wave_sum(s1[c]), b = wave_sum(s2[c]);
      if (lane == 0) {
        red[wid][2 * c] = a;
        red[wid][2 * c + 1] = b;
      }
    }
  __syncthreads();
  double *row = B.rows + (long long)(B.tile_base + blockIdx.x) * (2 * nc + dN);
  if (tid < 2 * nc) {
    double a = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) a += red[q][tid];
    row[tid] = a;
  }
  for (int e = tid; e < dN; e += blockDim.x) row[2 * nc + e] = hs[e];
}

// a7 for caller-evaluated integrands: one workgroup sums the iteration's
// group rows in group order, settles every component (its own estimate,
// combination and chi^2), applies the stop rule to all components together
// (accuracy needs every one) and refines the grid in place from component 0's
// histogram, one wavefront per dimension.
__global__ void __launch_bounds__(1024) vegas_batched_finish_kernel(BatchedFinishArgs F) {
  extern __shared__ double fsm[];
  __shared__ int s_conv[kMaxComp], s_bad[kMaxComp];
  __shared__ int s_mode;
  const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wv = tid >> 6, nwv = bs >> 6;
  const int d = F.ndim, N = F.nbins, dN = d * N, nc = F.ncomp, row = N + 1, drow = d * row;
  const int R = 2 * nc + dN;
  if (F.state[0].done) return;  // the same for every thread (and every component)
  double *S = fsm;              // the folded row: sums, then H
  double *D = fsm + R;          // smoothed histogram, later m
  double *G = fsm + R + dN;     // the grid
  constexpr int kB = 16;        // group rows in flight per thread
  for (int e = tid; e < R; e += bs) {
    const double *src = F.ghist + e;
    double h = 0.0;
    for (int g0 = 0; g0 < F.ngroups; g0 += kB) {
      double v[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) v[q] = g0 + q < F.ngroups ? src[(long long)(g0 + q) * R] : 0.0;
      asm volatile("" ::: "memory");  // every load of the batch before the adds
      if (g0 == 0) h = v[0];          // group order; the first row starts the sum
#pragma unroll
      for (int q = 0; q < kB; ++q)
        if ((g0 > 0 || q > 0) && g0 + q < F.ngroups) h += v[q];
    }
    S[e] = h;
  }
  for (int e = tid; e < drow; e += bs) G[e] = F.grid[e];
  __syncthreads();
  VState st;
  double I = 0.0, var = 0.0;
  const int t = F.state[0].T;
  const long long n = F.nstart + (long long)t * F.nincrease;
  if (tid < nc) {
    st = F.state[tid];
    settle_component(st, S[2 * tid], S[2 * tid + 1], n, I, var);
    F.iter_I[(long long)tid * F.hist_cap + t] = I;
    F.iter_var[(long long)tid * F.hist_cap + t] = var;
    const double tol = fmax(F.epsabs, F.epsrel * fabs(st.integral));
    s_conv[tid] = st.neval >= F.mineval && st.error <= tol;
    s_bad[tid] = !isfinite(S[2 * tid]) || !isfinite(S[2 * tid + 1]);
  }
  __syncthreads();
  if (tid < nc) {
    bool conv = true, bad = false;
    for (int c = 0; c < nc; ++c) {
      conv = conv && s_conv[c] != 0;
      bad = bad || s_bad[c] != 0;
    }
    const int T = st.T;
    const long long nnext = F.nstart + (long long)T * F.nincrease;
    const bool budget = st.neval + nnext > F.maxeval || T >= F.hist_cap || nnext >= (1ll << 32);
    finish_state(st, bad, conv, budget, F.iter_I + (long long)tid * F.hist_cap,
                 F.iter_var + (long long)tid * F.hist_cap);
    F.state[tid] = st;
    if (tid == 0) s_mode = conv || bad ? 0 : ((F.flags & FLAG_FREEZE_GRID) ? 2 : 1);
  }
  __syncthreads();
  if (s_mode != 1) return;  // converged, or the grid is frozen (kept as it is)
  double *H = S + 2 * nc;
  for (int j = wv; j < d; j += nwv)
    rebin_dimension(H + j * N, D + j * N, G + j * row, F.grid + j * row, N, lane);
}

// ---------------------------------------------------------------------------
// launchers

hipError_t launch_dosample(const VegasArgs &A, int prec, int nb, bool pow2, bool full,
                           int grid, int block, size_t lds, hipStream_t s) {
  if (A.tile_count <= 0 || grid <= 0) return hipSuccess;
  if (prec == FP64)
    return A.hist64 ? launch_dosample_f64(A, nb, pow2, full, grid, block, lds, s)
                    : launch_dosample_f64hfx(A, nb, pow2, full, grid, block, lds, s);
  if (A.hist64) return launch_dosample_f32h64(A, nb, pow2, full, grid, block, lds, s);
  return launch_dosample_f32hfx(A, nb, pow2, full, grid, block, lds, s);
}

hipError_t launch_fold(const FoldArgs &F, bool level2, hipStream_t s) {
  if (F.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(vegas_fold_kernel, dim3((unsigned)((F.total + 3) / 4)), dim3(256), 0, s, F);
  if (level2)
    hipLaunchKernelGGL(vegas_fold2_kernel, dim3((unsigned)((F.total2 + 3) / 4)), dim3(256), 0,
                       s, F);
  return hipGetLastError();
}

hipError_t launch_refine(const VegasArgs &A, int njobs, int dmax, hipStream_t s) {
  // one workgroup per (integral, dimension)
  hipLaunchKernelGGL(vegas_refine_kernel, dim3(njobs, dmax), dim3(kRefineThreads), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_init_grids(const VJob *jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(vegas_init_grids_kernel, dim3(njobs), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_init_grid(double *grid, int ndim, int nbins, hipStream_t s) {
  hipLaunchKernelGGL(vegas_init_grid_kernel, dim3(1), dim3(256), 0, s, grid, ndim, nbins);
  return hipGetLastError();
}

hipError_t launch_collect(const VegasArgs &A, int njobs, double *sums, double *hist,
                          hipStream_t s) {
  hipLaunchKernelGGL(vegas_collect_kernel, dim3(njobs), dim3(256), 0, s, A, sums, hist);
  return hipGetLastError();
}

hipError_t launch_points(const PointsArgs &P, hipStream_t s) {
  const long long per = (long long)kPointsBlock * kPointsPerThread;
  const long long grid = (P.npts + per - 1) / per;
  if (grid == 0) return hipSuccess;
  const size_t stage = (size_t)kPointsBlock * P.ndim * (sizeof(double) + sizeof(int));
  if (P.prec == FP64)
    hipLaunchKernelGGL(vegas_points_kernel<double>, dim3((unsigned)grid), dim3(kPointsBlock),
                       points_cells_bytes<double>(P.ndim, P.nbins) + stage, s, P);
  else
    hipLaunchKernelGGL(vegas_points_kernel<float>, dim3((unsigned)grid), dim3(kPointsBlock),
                       points_cells_bytes<float>(P.ndim, P.nbins) + stage, s, P);
  return hipGetLastError();
}

hipError_t launch_batched_accumulate(const BatchedArgs &B, hipStream_t s) {
  const long long tiles = (B.npts + B.tile_pts - 1) / B.tile_pts;
  if (tiles <= 0) return hipSuccess;
  const size_t lds = (size_t)B.ndim * B.nbins * sizeof(double);
  hipLaunchKernelGGL(vegas_batched_accumulate_kernel, dim3((unsigned)tiles), dim3(kAccumThreads),
                     lds, s, B);
  return hipGetLastError();
}

hipError_t launch_batched_finish(const BatchedFinishArgs &F, hipStream_t s) {
  const size_t dN = (size_t)F.ndim * F.nbins;
  const size_t lds = (2 * (size_t)F.ncomp + 2 * dN + (size_t)F.ndim * (F.nbins + 1)) * 8;
  hipLaunchKernelGGL(vegas_batched_finish_kernel, dim3(1), dim3(1024), lds, s, F);
  return hipGetLastError();
}

hipError_t set_kernel_limits() {
  // allow the large-grid cases (d = 16, 256 bins: up to 128 KB of cells and
  // histogram) the LDS gfx950 has; a runtime that refuses keeps its default
  // limit and such launches report an error instead of running
  const int big = 160 * 1024;
  std::vector<const void *> fns = {(const void *)vegas_batched_finish_kernel,
                                   (const void *)vegas_points_kernel<double>,
                                   (const void *)vegas_points_kernel<float>};
  dosample_fns_f64(fns);
  dosample_fns_f32h64(fns);
  dosample_fns_f32hfx(fns);
  dosample_fns_f64hfx(fns);
  for (const void *f : fns)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big) != hipSuccess)
      (void)hipGetLastError();
  return hipSuccess;
}

}  // namespace ccuba
