// vegas_batched.cpp -- Vegas with a caller-evaluated integrand.
//
// The accelerator strategy of Sect. 3.2.4: the integrand receives batches of
// exactly nvec points, fewer only in an iteration's last batch, as
// x[nvec][ndim] with f[nvec][ncomp] to fill (the integrand declaration of
// Sect. 3.2.2, core < 0 for an accelerator).  The library makes each batch's
// points on the GPU with the points kernel (the Philox words, uniforms and
// grid map of DoSample) and hands them over in host memory or, for an
// integrand that runs its own GPU code, in device memory.  The rest of the
// iteration stays on the GPU: per-tile sums of every component and component
// 0's histogram, the fold kernel over those rows, and one workgroup for the
// statistics, the stop rule and the grid.
#include "vegas_batched.h"

#include <algorithm>
#include <vector>

#include "vegas.h"
#include "vegas_engine.h"

namespace ccuba {

namespace {

constexpr int kBatchedTile = 4096;  // points per tile row

struct PinnedHost {
  void *p = nullptr;
  ~PinnedHost() {
    if (p) (void)hipHostFree(p);
  }
};

long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

}  // namespace

int vegas_batched(ccuba_ctx *ctx, const BatchedSpec &sp, ccuba_batch_integrand fn,
                  void *userdata, long long *neval, int *fail, double integral[],
                  double error[], double prob[]) {
  hipStream_t s = ctx->stream;
  const int d = sp.ndim, N = sp.nbins, nc = sp.ncomp, dN = d * N, R = 2 * nc + dN;
  const int row = N + 1;
  for (int c = 0; c < nc; ++c) integral[c] = error[c] = prob[c] = 0.0;
  VegasSpec vs;
  vs.nstart = sp.nstart;
  vs.nincrease = sp.nincrease;
  vs.maxeval = sp.maxeval;
  int iters = 0;
  long long nmax = 0;
  vegas_budget(vs, &iters, &nmax);
  if (iters == 0) {  // not even one iteration fits the budget
    *neval = 0;
    *fail = 1;
    return CCUBA_OK;
  }
  const int cap = iters;
  const long long mmax = std::min<long long>(sp.nvec, nmax);
  const long long tiles_max = ceil_div(nmax, sp.nvec) * ceil_div(mmax, kBatchedTile);
  const long long groups_max = ngroups_of((int)tiles_max);
  DevBuf<double> grid, x, f, w, rows, tzero, ghist, gsums, hist;
  DevBuf<int> bin;
  DevBuf<VState> states, dummy;
  DevBuf<VJob> view;
  DevBuf<long long> task_end;
  int rc;
  if ((rc = grid.alloc(ctx, (size_t)d * row)) || (rc = x.alloc(ctx, mmax * d)) ||
      (rc = f.alloc(ctx, mmax * nc)) || (rc = w.alloc(ctx, mmax)) ||
      (rc = bin.alloc(ctx, mmax * d)) || (rc = rows.alloc(ctx, tiles_max * R)) ||
      (rc = tzero.alloc(ctx, 2 * tiles_max)) || (rc = ghist.alloc(ctx, groups_max * R)) ||
      (rc = gsums.alloc(ctx, 2 * groups_max)) || (rc = hist.alloc(ctx, 2ll * nc * cap)) ||
      (rc = states.alloc(ctx, nc)) || (rc = dummy.alloc(ctx, 1)) || (rc = view.alloc(ctx, 1)) ||
      (rc = task_end.alloc(ctx, 1)))
    return rc;
  PinnedHost xh, fh;
  const bool host = sp.where == CCUBA_POINTS_HOST;
  if (host) {
    CCUBA_HIP(hipHostMalloc(&xh.p, mmax * d * sizeof(double), hipHostMallocDefault));
    CCUBA_HIP(hipHostMalloc(&fh.p, mmax * nc * sizeof(double), hipHostMallocDefault));
  }
  CCUBA_HIP(launch_init_grid(grid.p, d, N, s));
  // a zero VState is the state before the first iteration; the fold's view
  // of the tile rows reads a state that is never done and tile sums of zero
  CCUBA_HIP(hipMemsetAsync(states.p, 0, nc * sizeof(VState), s));
  CCUBA_HIP(hipMemsetAsync(dummy.p, 0, sizeof(VState), s));
  CCUBA_HIP(hipMemsetAsync(tzero.p, 0, 2 * tiles_max * sizeof(double), s));

  PointsArgs pa{};
  pa.ndim = d;
  pa.nbins = N;
  pa.prec = sp.prec;
  pa.key0 = (uint32_t)(sp.seed & 0xffffffffull);
  pa.key1 = (uint32_t)(sp.seed >> 32);
  pa.sid = sp.sid;
  pa.grid = grid.p;
  pa.words = nullptr;
  pa.x = x.p;
  pa.w = w.p;
  pa.bin = bin.p;
  // host copies of the fold's view, alive until the iteration's sync
  VJob jv{};
  long long tend = 0;
  VState st0{};
  long long handed = 0;  // points given to the integrand
  const int core = -1;   // an accelerator (Sect. 3.2.4)
  for (int t = 0; t < iters; ++t) {
    const long long n = sp.nstart + (long long)t * sp.nincrease;
    int tiles = 0;
    for (long long i0 = 0; i0 < n; i0 += sp.nvec) {
      const long long m = std::min<long long>(sp.nvec, n - i0);
      pa.iteration = t;
      pa.i0 = i0;
      pa.npts = m;
      CCUBA_HIP(launch_points(pa, s));
      const int mi = (int)m, nd = d, ncomp = nc;
      int urc;
      if (host) {
        CCUBA_HIP(hipMemcpyAsync(xh.p, x.p, m * d * sizeof(double), hipMemcpyDeviceToHost, s));
        CCUBA_HIP(hipStreamSynchronize(s));
        urc = fn(&nd, (const double *)xh.p, &ncomp, (double *)fh.p, userdata, &mi, &core);
      } else {
        CCUBA_HIP(hipStreamSynchronize(s));
        urc = fn(&nd, x.p, &ncomp, f.p, userdata, &mi, &core);
      }
      handed += m;
      if (urc == -999) {
        for (int c = 0; c < nc; ++c) integral[c] = error[c] = prob[c] = 0.0;
        *neval = handed;
        *fail = -99;
        return CCUBA_OK;
      }
      if (host)
        CCUBA_HIP(hipMemcpyAsync(f.p, fh.p, m * nc * sizeof(double), hipMemcpyHostToDevice, s));
      BatchedArgs ba{d, N, nc, sp.prec, m, kBatchedTile, tiles, w.p, f.p, bin.p, rows.p,
                     states.p};
      CCUBA_HIP(launch_batched_accumulate(ba, s));
      tiles += (int)ceil_div(m, kBatchedTile);
    }
    // the fold kernel sums the tile rows 32 at a time, seeing them as the
    // histogram rows of one job of R = 2 ncomp + ndim nbins bins
    jv = VJob{};
    jv.ndim = 1;
    jv.nbins = R;
    jv.ntiles = tiles;
    jv.state = dummy.p;
    jv.thist = rows.p;
    jv.tsums = tzero.p;
    jv.ghist = ghist.p;
    jv.gsums = gsums.p;
    const int ng = ngroups_of(tiles);
    tend = (long long)ng * ((R + 63) / 64);
    CCUBA_HIP(hipMemcpyAsync(view.p, &jv, sizeof(VJob), hipMemcpyHostToDevice, s));
    CCUBA_HIP(hipMemcpyAsync(task_end.p, &tend, sizeof(long long), hipMemcpyHostToDevice, s));
    FoldArgs fo{view.p, task_end.p, 1, tend, nullptr, 0};
    CCUBA_HIP(launch_fold(fo, false, s));
    BatchedFinishArgs fa{};
    fa.ndim = d;
    fa.nbins = N;
    fa.ncomp = nc;
    fa.flags = sp.flags;
    fa.ngroups = ng;
    fa.ghist = ghist.p;
    fa.grid = grid.p;
    fa.state = states.p;
    fa.iter_I = hist.p;
    fa.iter_var = hist.p + (size_t)nc * cap;
    fa.hist_cap = cap;
    fa.nstart = sp.nstart;
    fa.nincrease = sp.nincrease;
    fa.mineval = sp.mineval;
    fa.maxeval = sp.maxeval;
    fa.epsrel = sp.epsrel;
    fa.epsabs = sp.epsabs;
    CCUBA_HIP(launch_batched_finish(fa, s));
    CCUBA_HIP(hipMemcpyAsync(&st0, states.p, sizeof(VState), hipMemcpyDeviceToHost, s));
    CCUBA_HIP(hipStreamSynchronize(s));
    if (st0.done) break;
  }
  std::vector<VState> st(nc);
  CCUBA_HIP(hipMemcpyAsync(st.data(), states.p, nc * sizeof(VState), hipMemcpyDeviceToHost, s));
  CCUBA_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < nc; ++c) {
    integral[c] = st[c].integral;
    error[c] = st[c].error;
    prob[c] = st[c].prob;
  }
  *neval = st[0].neval;
  *fail = st[0].fail;
  return CCUBA_OK;
}

}  // namespace ccuba
