// divonne_engine.cpp -- host driver of Divonne's partitioning phase (Sect. 2.2;
// the steps are those listed in divonne.hip).  The regions, their extrema and
// spreads stay on the device; after each step the host reads the largest and
// the total spread (16 bytes) and sizes the next step:
// K = min(nsplit, regions, maxregions - regions).
#include "divonne_engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "suave.h"
#include "vegas_engine.h"

namespace ccuba {

int validate_partition(const PartitionSpec &s) {
  if (s.ndim < 1 || s.ndim > kMaxDim || s.family < 0 || s.family > C0 || s.nsearch < 1 ||
      s.nsearch > (1 << 30) ||  // the search loops step an int index
      s.niter < 0 || s.niter > 4096 || s.maxregions < 1 || s.maxregions > (1 << 23) ||
      s.nsplit < 1 || s.nsplit > kSuaveMaxSplit || !(s.spread_tol >= 0.0))
    return CCUBA_EINVAL;
  for (int j = 0; j < s.ndim; ++j)
    if (!std::isfinite(s.a[j]) || !std::isfinite(s.u[j])) return CCUBA_EINVAL;
  return CCUBA_OK;
}

int run_partition(ccuba_ctx *ctx, const PartitionSpec &sp, PartitionResult &res,
                  const PartitionTraceOut *tr, hipStream_t s) {
  int rc = validate_partition(sp);
  if (rc) return rc;
  res = PartitionResult();
  const int d = sp.ndim;
  const long long Rmax = sp.maxregions;
  const int Kmax = (int)std::min<long long>(sp.nsplit, std::max<long long>(1, Rmax - 1));
  DevBuf<double> lo, hi, xmin, xmax, fmin, fmax, spread, p64;
  DevBuf<int> sel, chpos, chser, cut;
  if ((rc = lo.alloc(ctx, Rmax * d)) || (rc = hi.alloc(ctx, Rmax * d)) ||
      (rc = xmin.alloc(ctx, Rmax * d)) || (rc = xmax.alloc(ctx, Rmax * d)) ||
      (rc = fmin.alloc(ctx, Rmax)) || (rc = fmax.alloc(ctx, Rmax)) ||
      (rc = spread.alloc(ctx, Rmax)) || (rc = p64.alloc(ctx, 2 * kParamRow)) ||
      (rc = sel.alloc(ctx, Kmax)) || (rc = chpos.alloc(ctx, 2 * Kmax)) ||
      (rc = chser.alloc(ctx, 2 * Kmax)) || (rc = cut.alloc(ctx, std::max<long long>(1, Rmax - 1))))
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
  double c64[2][kParamRow];
  float c32[2][kParamRow];
  genz_constants(vs, c64, c32);
  CCUBA_HIP(hipMemcpyAsync(p64.p, c64, sizeof(c64), hipMemcpyHostToDevice, s));

  DivArgs A{};
  A.R = DRegions{lo.p, hi.p, xmin.p, xmax.p, fmin.p, fmax.p, spread.p};
  A.d = d;
  A.family = sp.family;
  A.key0 = (uint32_t)(sp.seed & 0xffffffffull);
  A.key1 = (uint32_t)(sp.seed >> 32);
  A.sid = sp.sid;
  A.nsearch = sp.nsearch;
  A.niter = sp.niter;
  A.p64 = p64.p;
  A.sel = sel.p;
  A.chpos = chpos.p;
  A.chser = chser.p;
  A.cut = cut.p;
  A.state = (DState *)pin_dev;
  const long long per_search = sp.nsearch + 4ll * d * sp.niter;

  CCUBA_HIP(launch_div_root(A, s));
  CCUBA_HIP(launch_div_search(A, 1, s));
  CCUBA_HIP(launch_div_totals(A, 1, s));
  long long R = 1, Q = 0, neval = per_search;
  DState st{};
  int fail = 1;
  for (;;) {
    CCUBA_HIP(hipStreamSynchronize(s));
    std::memcpy(&st, pin_host, sizeof(st));
    if (!std::isfinite(st.total_spread)) {  // a non-finite integrand value
      fail = -4;
      st = DState{};
      break;
    }
    if (st.max_spread <= sp.spread_tol) {
      fail = 0;
      break;
    }
    const long long K = std::min<long long>({(long long)sp.nsplit, R, Rmax - R});
    if (K <= 0) break;
    CCUBA_HIP(launch_topk(spread.p, (int)R, (int)K, sel.p, s));
    CCUBA_HIP(launch_div_split(A, (int)R, Q, (int)K, s));
    CCUBA_HIP(launch_div_search(A, (int)(2 * K), s));
    R += K;
    Q += K;
    neval += K * (2 * per_search + d);
    CCUBA_HIP(launch_div_totals(A, (int)R, s));
  }
  res.nregions = (int)R;
  res.fail = fail;
  res.neval = neval;
  res.nsplits = Q;
  res.total_spread = st.total_spread;
  res.max_spread = st.max_spread;
  if (tr) {
    const size_t m = (size_t)std::min<long long>(R, tr->max_regions);
    auto get = [&](double *dst, const double *src, size_t n) {
      return dst ? hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToHost, s) : hipSuccess;
    };
    if (m > 0) {
      CCUBA_HIP(get(tr->lo, lo.p, m * d));
      CCUBA_HIP(get(tr->hi, hi.p, m * d));
      CCUBA_HIP(get(tr->xmin, xmin.p, m * d));
      CCUBA_HIP(get(tr->xmax, xmax.p, m * d));
      CCUBA_HIP(get(tr->fmin, fmin.p, m));
      CCUBA_HIP(get(tr->fmax, fmax.p, m));
      CCUBA_HIP(get(tr->spread, spread.p, m));
    }
    const size_t q = (size_t)std::min<long long>(Q, tr->max_splits);
    if (q > 0 && tr->cut)
      CCUBA_HIP(hipMemcpyAsync(tr->cut, cut.p, q * sizeof(int), hipMemcpyDeviceToHost, s));
    CCUBA_HIP(hipStreamSynchronize(s));
  }
  return CCUBA_OK;
}

}  // namespace ccuba
