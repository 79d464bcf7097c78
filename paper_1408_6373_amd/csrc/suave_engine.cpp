// suave_engine.cpp -- host driver of Suave (Sect. 3.2.2 prototype; the steps
// are those listed in suave.hip).
//
// Device memory: per region its bounds, grid and result, plus the nnew values
// and side bits of its own sample (10 bytes a point); the region count is
// bounded by the budget, R <= 1 + (maxeval - nnew) / (2 nnew).  After each
// step the host reads the totals (a few doubles), applies the stop rule and
// sizes the next step: K = min(nsplit, R, (maxeval - neval) / (2 nnew)).
#include "suave_engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "vegas_engine.h"

namespace ccuba {

int validate_suave(const SuaveSpec &s) {
  if (s.ndim < 1 || s.ndim > kMaxDim || s.nbins < 2 || s.nbins > kMaxBins || s.family < 0 ||
      s.family > C0 || s.nnew < 2 || s.nnew >= (1ll << 32) || !(s.flatness > 0.0) ||
      !std::isfinite(s.flatness) || s.nsplit < 1 || s.nsplit > kSuaveMaxSplit || s.mineval < 0 ||
      s.maxeval < 0 || !(s.epsrel >= 0.0) || !(s.epsabs >= 0.0))
    return CCUBA_EINVAL;
  for (int j = 0; j < s.ndim; ++j)
    if (!std::isfinite(s.a[j]) || !std::isfinite(s.u[j])) return CCUBA_EINVAL;
  return CCUBA_OK;
}

namespace {

struct Buffers {
  DevBuf<double> lo, hi, grid, I, var, chi2, inh_I, inh_var, v, fl1, fl2, hs, tsum, thist, p64;
  DevBuf<int> dof, sel, chpos, chser, cut;
  DevBuf<uint16_t> side;
};

}  // namespace

int run_suave(ccuba_ctx *ctx, const SuaveSpec &sp, SuaveResult &res, const SuaveTraceOut *tr,
              hipStream_t s) {
  int rc = validate_suave(sp);
  if (rc) return rc;
  res = SuaveResult();
  if (sp.nnew > sp.maxeval) return CCUBA_OK;  // no point can be afforded: fail 1
  const int d = sp.ndim, N = sp.nbins;
  const long long n = sp.nnew;
  const long long Rmax = 1 + (sp.maxeval - n) / (2 * n);
  if (Rmax > (1ll << 23)) return CCUBA_EINVAL;  // sampling serials are 24 bits
  const int Kmax = (int)std::min<long long>(sp.nsplit, std::max<long long>(1, Rmax - 1));
  const int ntiles = (int)((n + kSuaveTile - 1) / kSuaveTile);
  const int nchunks = (int)((n + kSuaveChunk - 1) / kSuaveChunk);
  const size_t dN = (size_t)d * N, row = (size_t)d * (N + 1);
  Buffers B;
  if ((rc = B.lo.alloc(ctx, Rmax * d)) || (rc = B.hi.alloc(ctx, Rmax * d)) ||
      (rc = B.grid.alloc(ctx, Rmax * row)) || (rc = B.I.alloc(ctx, Rmax)) ||
      (rc = B.var.alloc(ctx, Rmax)) || (rc = B.chi2.alloc(ctx, Rmax)) ||
      (rc = B.inh_I.alloc(ctx, Rmax)) || (rc = B.inh_var.alloc(ctx, Rmax)) ||
      (rc = B.dof.alloc(ctx, Rmax)) || (rc = B.v.alloc(ctx, Rmax * n)) ||
      (rc = B.side.alloc(ctx, Rmax * n)) || (rc = B.fl1.alloc(ctx, (size_t)Kmax * nchunks * d * 9)) ||
      (rc = B.fl2.alloc(ctx, (size_t)Kmax * nchunks * d * 2)) ||
      (rc = B.hs.alloc(ctx, (size_t)Kmax * d * 10)) ||
      (rc = B.tsum.alloc(ctx, (size_t)2 * Kmax * ntiles * 2)) ||
      (rc = B.thist.alloc(ctx, (size_t)2 * Kmax * ntiles * dN)) ||
      (rc = B.p64.alloc(ctx, 2 * kParamRow)) || (rc = B.sel.alloc(ctx, Kmax)) ||
      (rc = B.chpos.alloc(ctx, 2 * Kmax)) || (rc = B.chser.alloc(ctx, 2 * Kmax)) ||
      (rc = B.cut.alloc(ctx, std::max<long long>(1, Rmax - 1))))
    return rc;
  double *pin_host = nullptr, *pin_dev = nullptr;  // the totals land in host memory
  if ((rc = pinned_block(ctx, &pin_host, &pin_dev))) return rc;

  VegasSpec vs;
  vs.ndim = d;
  vs.family = sp.family;
  for (int j = 0; j < d; ++j) {
    vs.a[j] = sp.a[j];
    vs.u[j] = sp.u[j];
  }
  double p64[2][kParamRow];
  float p32[2][kParamRow];
  genz_constants(vs, p64, p32);
  CCUBA_HIP(hipMemcpyAsync(B.p64.p, p64, sizeof(p64), hipMemcpyHostToDevice, s));

  SuaveArgs A{};
  A.R = SRegions{B.lo.p, B.hi.p, B.grid.p, B.I.p, B.var.p, B.chi2.p, B.dof.p,
                 B.inh_I.p, B.inh_var.p, B.v.p, B.side.p};
  A.d = d;
  A.N = N;
  A.family = sp.family;
  A.flags = sp.flags & FLAG_FREEZE_GRID;
  A.nnew = n;
  A.key0 = (uint32_t)(sp.seed & 0xffffffffull);
  A.key1 = (uint32_t)(sp.seed >> 32);
  A.sid = sp.sid;
  A.ntiles = ntiles;
  A.nchunks = nchunks;
  A.flatness = sp.flatness;
  A.ipow = (sp.flatness == std::floor(sp.flatness) && sp.flatness <= 4096.0) ? (int)sp.flatness : 0;
  A.p64 = B.p64.p;
  A.sel = B.sel.p;
  A.chpos = B.chpos.p;
  A.chser = B.chser.p;
  A.fl1 = B.fl1.p;
  A.fl2 = B.fl2.p;
  A.hs = B.hs.p;
  A.tsum = B.tsum.p;
  A.thist = B.thist.p;
  A.cut = B.cut.p;
  A.state = (SState *)pin_dev;

  // the root region
  CCUBA_HIP(launch_suave_root(A, s));
  CCUBA_HIP(launch_suave_sample(A, 1, s));
  CCUBA_HIP(launch_suave_fold(A, 1, s));
  CCUBA_HIP(launch_suave_totals(A, 1, s));
  long long R = 1, Q = 0, neval = n;
  SState st{};
  int fail = 1;
  for (;;) {
    CCUBA_HIP(hipStreamSynchronize(s));
    std::memcpy(&st, pin_host, sizeof(st));
    if (!std::isfinite(st.I) || !std::isfinite(st.var)) {  // a non-finite integrand value
      fail = -4;
      st = SState{};
      break;
    }
    if (neval >= sp.mineval &&
        std::sqrt(st.var) <= std::max(sp.epsabs, sp.epsrel * std::fabs(st.I))) {
      fail = 0;
      break;
    }
    long long K = std::min<long long>(sp.nsplit, R);
    K = std::min<long long>(K, (sp.maxeval - neval) / (2 * n));
    if (K <= 0) break;
    CCUBA_HIP(launch_suave_select(A, (int)R, (int)K, s));
    CCUBA_HIP(launch_suave_fluct(A, (int)K, s));
    CCUBA_HIP(launch_suave_split(A, (int)R, Q, (int)K, s));
    CCUBA_HIP(launch_suave_sample(A, (int)(2 * K), s));
    CCUBA_HIP(launch_suave_fold(A, (int)(2 * K), s));
    R += K;
    Q += K;
    neval += 2 * K * n;
    CCUBA_HIP(launch_suave_totals(A, (int)R, s));
  }
  res.integral = st.I;
  res.error = std::sqrt(st.var);
  res.prob = st.prob;
  res.chi2 = st.chi2;
  res.dof = st.dof;
  res.fail = fail;
  res.nregions = (int)R;
  res.neval = neval;
  res.nsplits = Q;
  if (tr) {
    const size_t m = (size_t)std::min<long long>(R, tr->max_regions);
    if (m > 0) {
      if (tr->lo) CCUBA_HIP(hipMemcpyAsync(tr->lo, B.lo.p, m * d * 8, hipMemcpyDeviceToHost, s));
      if (tr->hi) CCUBA_HIP(hipMemcpyAsync(tr->hi, B.hi.p, m * d * 8, hipMemcpyDeviceToHost, s));
      if (tr->I) CCUBA_HIP(hipMemcpyAsync(tr->I, B.I.p, m * 8, hipMemcpyDeviceToHost, s));
      if (tr->var) CCUBA_HIP(hipMemcpyAsync(tr->var, B.var.p, m * 8, hipMemcpyDeviceToHost, s));
      if (tr->grid)
        CCUBA_HIP(hipMemcpyAsync(tr->grid, B.grid.p, m * row * 8, hipMemcpyDeviceToHost, s));
    }
    const size_t q = (size_t)std::min<long long>(Q, tr->max_splits);
    if (q > 0 && tr->cut)
      CCUBA_HIP(hipMemcpyAsync(tr->cut, B.cut.p, q * sizeof(int), hipMemcpyDeviceToHost, s));
    CCUBA_HIP(hipStreamSynchronize(s));
  }
  return CCUBA_OK;
}

}  // namespace ccuba
