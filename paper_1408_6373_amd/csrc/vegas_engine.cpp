// vegas_engine.cpp -- host driver of the batched Vegas DoSample engine.
#include "vegas_engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace ccuba {

namespace {

const double kTwoPi = 6.283185307179586476925286766559;
const double kLog2e = 1.4426950408889634073599246810019;

long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }
size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

template <typename T>
int upload(DevBuf<T> &b, const std::vector<T> &h, hipStream_t s) {
  if (h.empty()) return 0;
  CCUBA_HIP(hipMemcpyAsync(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return 0;
}

}  // namespace

int validate_vegas(const VegasSpec &s) {
  if (s.ndim < 1 || s.ndim > kMaxDim || s.nbins < 2 || s.nbins > kMaxBins ||
      s.nstart < 2 || s.nincrease < 0 || s.family < 0 || s.family > C0 ||
      (s.prec != FP64 && s.prec != FP32) || s.maxeval < 0 || s.nstart >= (1ll << 32) ||
      !(s.epsrel >= 0) || !(s.epsabs >= 0))
    return CCUBA_EINVAL;
  for (int j = 0; j < s.ndim; ++j)
    if (!std::isfinite(s.a[j]) || !std::isfinite(s.u[j])) return CCUBA_EINVAL;
  return CCUBA_OK;
}

void vegas_budget(const VegasSpec &s, int *iters, long long *nmax) {
  long long used = 0, nm = s.nstart;
  int t = 0;
  while (t < kIterCap) {
    const long long n = s.nstart + (long long)t * s.nincrease;
    if (n >= (1ll << 32) || used + n > s.maxeval) break;
    used += n;
    nm = n;
    ++t;
  }
  *iters = t;
  *nmax = nm;
}

void genz_constants(const VegasSpec &s, double p64[2][kParamRow], float p32[2][kParamRow]) {
  for (int w = 0; w < 2; ++w)
    for (int j = 0; j < kParamRow; ++j) {
      p64[w][j] = 0.0;
      p32[w][j] = 0.0f;
    }
  for (int j = 0; j < s.ndim; ++j) {
    const double a = s.a[j], u = s.u[j];
    switch (s.family) {
      case GAUSSIAN:
        p64[0][j] = a * a;
        p64[1][j] = u;
        p32[0][j] = (float)(a * a * kLog2e);
        p32[1][j] = (float)u;
        break;
      case OSCILLATORY:
        p64[0][j] = a;
        p32[0][j] = (float)(a / kTwoPi);
        break;
      case PRODUCT_PEAK:
        p64[0][j] = 1.0 / (a * a);
        p64[1][j] = u;
        p32[0][j] = (float)(1.0 / (a * a));
        p32[1][j] = (float)u;
        break;
      case CORNER_PEAK:
        p64[0][j] = a;
        p32[0][j] = (float)a;
        break;
      case USER:  // a caller's function gets its a and u as given
        p64[0][j] = a;
        p64[1][j] = u;
        p32[0][j] = (float)a;
        p32[1][j] = (float)u;
        break;
      default:  // C0
        p64[0][j] = a;
        p64[1][j] = u;
        p32[0][j] = (float)(a * kLog2e);
        p32[1][j] = (float)u;
        break;
    }
  }
  if (s.family == OSCILLATORY) {
    p64[1][0] = kTwoPi * s.u[0];
    p32[1][0] = (float)s.u[0];
  }
}

size_t batch_cut(const std::vector<VegasSpec> &specs) {
  if (specs.size() < 2) return specs.size();
  std::vector<double> work(specs.size());
  double total = 0.0;
  for (size_t j = 0; j < specs.size(); ++j) {
    int it = 0;
    long long nmax = 0;
    vegas_budget(specs[j], &it, &nmax);
    const VegasSpec &sp = specs[j];
    work[j] = (double)it * (double)sp.nstart +
              (double)sp.nincrease * (double)it * (double)(it - 1) / 2.0;
    total += work[j];
  }
  size_t best = 1;
  double acc = 0.0, gap = -1.0;
  for (size_t k = 1; k < specs.size(); ++k) {
    acc += work[k - 1];
    const double g = std::fabs(2.0 * acc - total);
    if (gap < 0.0 || g < gap) {
      gap = g;
      best = k;
    }
  }
  return best;
}

bool fixed_hist(int prec, int hist64, long long dN) {
  // the DoSample kernel's static LDS (block sums, per-dimension maxima) is
  // well below the 1 KB left for it
  constexpr long long kLds = 160 * 1024 - 1024;
  return !hist64 && (prec == FP32 || dN * (16 + 3 * 8) <= kLds);
}

void plan_tile_groups(std::vector<VJob> &jobs, std::vector<int> &tiles,
                      std::vector<TileGroup> &groups, const int hist64[2], size_t *refine_lds) {
  tiles.clear();
  groups.clear();
  size_t ref = 0;
  // one class per (precision, Philox blocks, power-of-two bins, d = 4 nb)
  for (int cls = 0; cls < 32; ++cls) {
    const int p = cls >> 4, nb = ((cls >> 2) & 3) + 1, pw = (cls >> 1) & 1, full = cls & 1;
    TileGroup g{p, nb, pw, full, (int)tiles.size(), 0, 0, 0, 0};
    auto mine = [&](const VJob &J) {
      const int jp = (J.nbins & (J.nbins - 1)) == 0, jf = J.ndim == 4 * nb;
      return J.prec == p && ((J.ndim + 3) >> 2) == nb && jp == pw && jf == full;
    };
    long long dNmax = 0;
    for (const VJob &J : jobs)
      if (mine(J)) dNmax = std::max(dNmax, (long long)J.ndim * J.nbins);
    g.hfx = fixed_hist(p, hist64[p], dNmax) ? 1 : 0;
    for (int j = 0; j < (int)jobs.size(); ++j) {
      VJob &J = jobs[j];
      if (!mine(J)) continue;
      J.tile0 = (int)tiles.size();
      for (int q = 0; q < J.ntiles; ++q) tiles.push_back(j);
      const size_t dN = (size_t)J.ndim * J.nbins;
      // refine: histogram, smoothed histogram and the current grid
      ref = std::max(ref, (2 * dN + (size_t)J.ndim * (J.nbins + 1)) * 8);
    }
    // LDS: one (lower edge, span) cell per bin, then the histogram (the
    // fixed-point one holds one integer sum per bin, two with FP64
    // evaluation, and an FP64 histogram beside them for the other values)
    const size_t csz = p == FP64 ? 16 : 8;
    const size_t hsz = !g.hfx ? 8 : (p == FP64 ? 24 : 16);
    g.grid_bytes = align16((size_t)dNmax * csz);
    g.count = (int)tiles.size() - g.first;
    g.lds = g.grid_bytes + (size_t)dNmax * hsz;
    if (g.count > 0) groups.push_back(g);
  }
  *refine_lds = ref;
}

int launch_tile_groups(ccuba_ctx *ctx, VegasArgs A, const std::vector<TileGroup> &groups,
                       hipStream_t s, hipFunction_t user) {
  for (const TileGroup &g : groups) {
    A.tile_first = g.first;
    A.tile_count = g.count;
    A.ilp = ctx->tune[g.prec].ilp;
    A.hist64 = g.hfx ? 0 : 1;
    A.lds_hist_byte_off = (long long)g.grid_bytes;
    const long long B = (long long)ctx->ncu * ctx->tune[g.prec].blocks_per_cu;
    const int grid = (int)std::min<long long>(B, g.count);
    if (user) {
      void *args[] = {&A};
      CCUBA_HIP(hipModuleLaunchKernel(user, grid, 1, 1, ctx->tune[g.prec].block, 1, 1,
                                      (unsigned)g.lds, s, args, nullptr));
    } else {
      CCUBA_HIP(launch_dosample(A, g.prec, g.nb, g.pow2 != 0, g.full != 0, grid,
                                ctx->tune[g.prec].block, g.lds, s));
    }
  }
  return CCUBA_OK;
}

void fold_tasks(const std::vector<VJob> &jobs, std::vector<long long> &ends, long long *total,
                long long *total2) {
  const size_t n = jobs.size();
  ends.resize(2 * n);
  long long t1 = 0, t2 = 0;
  for (size_t j = 0; j < n; ++j) {
    const long long dN = (long long)jobs[j].ndim * jobs[j].nbins, nch = (dN + 63) / 64;
    t1 += (long long)ngroups_of(jobs[j].ntiles) * nch;
    t2 += nch;
    ends[j] = t1;
    ends[n + j] = t2;
  }
  *total = t1;
  *total2 = t2;
}

VegasEngine::~VegasEngine() {
  for (auto &g : graphs_) (void)hipGraphExecDestroy(g.exec);
}

int VegasEngine::setup(const std::vector<VegasSpec> &specs, bool single, hipStream_t s) {
  specs_ = specs;
  const int n = (int)specs.size();
  if (n == 0) return CCUBA_EINVAL;
  for (const auto &sp : specs) {
    VegasSpec chk = sp;  // a caller's integrand needs its compiled kernel
    if (chk.family == USER && user_fn_ && specs.size() == 1) chk.family = GAUSSIAN;
    if (validate_vegas(chk) != CCUBA_OK) return CCUBA_EINVAL;
  }
  for (int p = 0; p < 2; ++p) {
    hist64_[p] = ctx_->tune[p].hist64;
    block_[p] = ctx_->tune[p].block;
    has_prec_[p] = 0;
  }
  std::vector<int> iters(n);
  std::vector<long long> nmax(n);
  long long total[2] = {0, 0};
  max_iters_ = 0;
  evals_iter_ = 0;
  dmax_ = 1;
  for (int j = 0; j < n; ++j) dmax_ = std::max(dmax_, specs[j].ndim);
  for (int j = 0; j < n; ++j) {
    vegas_budget(specs[j], &iters[j], &nmax[j]);
    max_iters_ = std::max(max_iters_, iters[j]);
    total[specs[j].prec] += nmax[j];
    has_prec_[specs[j].prec] = 1;
    if (iters[j] > 0) evals_iter_ += specs[j].nstart;
  }
  // Tile size of a batch, per precision: the tuned minimum, or larger when
  // that would give more than 8 tiles per block; then, within 3/4 to 5/4 of
  // that size, the one that makes the most tiles a compute unit gets
  // smallest.  The blocks take the tiles in turn, so a compute unit works
  // through about ceil(tiles / CUs) of them and the launch takes as long as
  // the busiest one: 1222 tiles of 16384 points leave some units 5 tiles
  // (81920 points) where 4.8 is the mean, 1262 of 15872 leave at most 5 of
  // the smaller tiles (79360).
  long long batch_P[2] = {0, 0};
  for (int p = 0; p < 2 && !single; ++p) {
    if (!has_prec_[p]) continue;
    const int bs = block_[p];
    const long long B = (long long)ctx_->ncu * ctx_->tune[p].blocks_per_cu;
    const long long target = round_up((total[p] + B * 8 - 1) / (B * 8), bs);
    const long long P0 = std::max<long long>(
        std::max(round_up(ctx_->tune[p].min_tile, bs), target), bs);
    long long best = P0, best_load = -1;
    for (long long P = std::max<long long>(bs, round_up(3 * P0 / 4, bs)); P <= 5 * P0 / 4;
         P += bs) {
      long long tiles = 0;
      for (int j = 0; j < n; ++j)
        if (specs[j].prec == p) tiles += std::max<long long>(1, (nmax[j] + P - 1) / P);
      const long long load = (tiles + ctx_->ncu - 1) / ctx_->ncu * P;
      if (best_load < 0 || load < best_load || (load == best_load && P > best)) {
        best = P;
        best_load = load;
      }
    }
    batch_P[p] = best;
  }
  // tile plan
  hjobs_.assign(n, VJob{});
  struct Offsets {
    long long grid, thist, ghist, iter;
    int tile0, group0;
    long long hsum;
  };
  std::vector<Offsets> off(n);
  std::vector<int> tile_job;
  long long goff = 0, thoff = 0, ghoff = 0, ioff = 0, hsoff = 0;
  int tile0 = 0, group0 = 0;
  for (int j = 0; j < n; ++j) {
    const VegasSpec &sp = specs[j];
    const int p = sp.prec;
    const int bs = block_[p];
    const long long B = (long long)ctx_->ncu * ctx_->tune[p].blocks_per_cu;
    long long P = single ? round_up((nmax[j] + B - 1) / B, bs) : batch_P[p];
    P = std::max<long long>(P, bs);
    const int nt = (int)std::max<long long>(1, (nmax[j] + P - 1) / P);
    VJob &J = hjobs_[j];
    J.ndim = sp.ndim;
    J.nbins = sp.nbins;
    J.family = sp.family;
    J.prec = p;
    J.flags = sp.flags;
    J.key0 = (uint32_t)(sp.seed & 0xffffffffull);
    J.key1 = (uint32_t)(sp.seed >> 32);
    J.sid = sp.sid;
    J.nstart = sp.nstart;
    J.nincrease = sp.nincrease;
    J.mineval = sp.mineval;
    J.maxeval = sp.maxeval;
    J.epsrel = sp.epsrel;
    J.epsabs = sp.epsabs;
    J.tile0 = tile0;
    J.ntiles = nt;
    J.tile_pts = P;
    J.hist_cap = std::max(1, iters[j]);
    const long long dN = (long long)sp.ndim * sp.nbins, row = (long long)sp.ndim * (sp.nbins + 1);
    off[j] = Offsets{goff, thoff, ghoff, ioff, tile0, group0, hsoff};
    hsoff += 2 + dN;
    goff += row;
    thoff += nt * dN;
    ghoff += ngroups_of(nt) * dN;
    ioff += J.hist_cap;
    tile0 += nt;
    group0 += ngroups_of(nt);
  }
  ntiles_ = tile0;
  ngroups_ = group0;
  plan_tile_groups(hjobs_, tile_job, tgroups_, hist64_, &lds_refine_);
  for (int p = 0; p < 2; ++p) {
    const long long B = (long long)ctx_->ncu * ctx_->tune[p].blocks_per_cu;
    nblocks_[p] = (int)std::min<long long>(B, ntiles_);
  }

  // buffers of an earlier setup are kept when large enough (an engine that
  // is set up again for the same shape keeps its device addresses)
  int rc;
  // (the states, then their snapshots for the refine kernel)
  if ((rc = jobs_.reserve(ctx_, n)) || (rc = state_.reserve(ctx_, 2 * (size_t)n)) ||
      (rc = tile_job_.reserve(ctx_, ntiles_)) || (rc = grids_.reserve(ctx_, goff)) ||
      (rc = p64_.reserve(ctx_, (size_t)n * 2 * kParamRow)) ||
      (rc = p32_.reserve(ctx_, (size_t)n * 2 * kParamRow)) ||
      (rc = tile_sums_.reserve(ctx_, 2 * (size_t)ntiles_)) ||
      (rc = tile_hist_.reserve(ctx_, thoff)) ||
      (rc = group_sums_.reserve(ctx_, 2 * (size_t)ngroups_)) ||
      (rc = group_hist_.reserve(ctx_, ghoff)) || (rc = fold_end_.reserve(ctx_, 2 * n)) ||
      (rc = hsum_.reserve(ctx_, hsoff)) ||
      (rc = iter_I_.reserve(ctx_, ioff)) || (rc = iter_var_.reserve(ctx_, ioff)))
    return rc;

  for (int j = 0; j < n; ++j) {
    VJob &J = hjobs_[j];
    J.state = state_.p + j;
    J.snap = state_.p + n + j;
    J.grid = grids_.p + off[j].grid;
    J.tsums = tile_sums_.p + 2ll * off[j].tile0;
    J.thist = tile_hist_.p + off[j].thist;
    J.gsums = group_sums_.p + 2ll * off[j].group0;
    J.ghist = group_hist_.p + off[j].ghist;
    J.hsum = hsum_.p + off[j].hsum;
    J.iter_I = iter_I_.p + off[j].iter;
    J.iter_var = iter_var_.p + off[j].iter;
    J.p64 = p64_.p + (size_t)j * 2 * kParamRow;
    J.p32 = p32_.p + (size_t)j * 2 * kParamRow;
  }
  std::vector<double> p64((size_t)n * 2 * kParamRow);
  std::vector<float> p32((size_t)n * 2 * kParamRow);
  std::vector<VState> st(n);
  for (int j = 0; j < n; ++j) {
    const VegasSpec &sp = specs[j];
    double a64[2][kParamRow];
    float a32[2][kParamRow];
    genz_constants(sp, a64, a32);
    std::memcpy(&p64[(size_t)j * 2 * kParamRow], a64, sizeof(a64));
    std::memcpy(&p32[(size_t)j * 2 * kParamRow], a32, sizeof(a32));
    st[j] = VState{};
    if (iters[j] == 0) {
      st[j].done = 1;
      st[j].fail = 1;
    }
  }
  if ((rc = upload(jobs_, hjobs_, s)) || (rc = upload(tile_job_, tile_job, s)) ||
      (rc = upload(p64_, p64, s)) || (rc = upload(p32_, p32, s)) ||
      (rc = upload(state_, st, s)))
    return rc;
  CCUBA_HIP(launch_init_grids(jobs_.p, n, s));
  std::vector<long long> ends;
  fold_tasks(hjobs_, ends, &fold_total_, &fold_total2_);
  if ((rc = upload(fold_end_, ends, s))) return rc;

  args_.jobs = jobs_.p;
  args_.tile_job = tile_job_.p;
  args_.tile_first = 0;
  args_.tile_count = ntiles_;
  args_.hist64 = 0;  // set per tile group at launch
  args_.njobs = n;
  pending_.clear();
  iter_launched_ = 0;
  // captured graphs stay valid only while every kernel argument they hold
  // is unchanged
  std::vector<long long> sig = {(long long)(intptr_t)jobs_.p, (long long)(intptr_t)state_.p,
                                (long long)(intptr_t)tile_job_.p,
                                (long long)(intptr_t)fold_end_.p, (long long)(intptr_t)user_fn_,
                                fold_total_, fold_total2_,
                                n, ntiles_, (long long)lds_refine_, hist64_[0], hist64_[1]};
  for (int p = 0; p < 2; ++p) {
    const VegasTune &t = ctx_->tune[p];
    sig.insert(sig.end(), {t.block, t.blocks_per_cu, t.ilp, t.hist64, ctx_->ncu});
  }
  for (const TileGroup &g : tgroups_)
    sig.insert(sig.end(), {g.prec, g.nb, g.pow2, g.full, g.first, g.count,
                           (long long)g.grid_bytes, (long long)g.lds, g.hfx});
  if (sig != graph_sig_) {
    for (auto &g : graphs_) (void)hipGraphExecDestroy(g.exec);
    graphs_.clear();
    graph_sig_ = sig;
  }
  // host copies of the tables must outlive the async uploads
  CCUBA_HIP(hipStreamSynchronize(s));
  return CCUBA_OK;
}

int VegasEngine::dosample_only(hipStream_t s, bool level2, hipEvent_t between) {
  const int rc = launch_tile_groups(ctx_, args_, tgroups_, s, user_fn_);
  if (rc) return rc;
  if (between) CCUBA_HIP(hipEventRecord(between, s));
  FoldArgs F{jobs_.p, fold_end_.p, njobs(), fold_total_, fold_end_.p + njobs(), fold_total2_};
  CCUBA_HIP(launch_fold(F, level2, s));
  return CCUBA_OK;
}

int VegasEngine::launch_iteration(hipStream_t s) {
  if (ctx_->profile && !capturing_) {
    // time the sampling kernels, the fold and the refine with events on the
    // stream they run on
    hipEvent_t ev[4];
    for (auto &e : ev) CCUBA_HIP(hipEventCreate(&e));
    CCUBA_HIP(hipEventRecord(ev[0], s));
    int rc = dosample_only(s, false, ev[1]);
    if (rc) return rc;
    CCUBA_HIP(hipEventRecord(ev[2], s));
    CCUBA_HIP(launch_refine(args_, njobs(), dmax_, s));
    CCUBA_HIP(hipEventRecord(ev[3], s));
    pending_.push_back({ev[0], ev[1], ev[2], ev[3], iter_launched_++});
    return CCUBA_OK;
  }
  int rc = dosample_only(s);
  if (rc) return rc;
  CCUBA_HIP(launch_refine(args_, njobs(), dmax_, s));
  ++iter_launched_;
  return CCUBA_OK;
}

int VegasEngine::flush_timing() {
  for (auto &p : pending_) {
    float a = 0, b = 0, c = 0, t0 = 0;
    CCUBA_HIP(hipEventSynchronize(p.e3));
    CCUBA_HIP(hipEventElapsedTime(&a, p.e0, p.e1));
    CCUBA_HIP(hipEventElapsedTime(&b, p.e1, p.e2));
    CCUBA_HIP(hipEventElapsedTime(&c, p.e2, p.e3));
    if (ref_) {
      CCUBA_HIP(hipEventElapsedTime(&t0, ref_, p.e0));
      ds_iv_.push_back({(double)t0, (double)t0 + a});
    }
    std::lock_guard<std::mutex> g(ctx_->stats_lock);
    ctx_->stats.dosample_launches += (long long)tgroups_.size();
    ctx_->stats.dosample_ms += a;
    if (!ref_) ctx_->stats.dosample_busy_ms += a;
    ctx_->stats.fold_ms += b;
    ctx_->stats.refine_launches += 1;
    ctx_->stats.refine_ms += c;
    (void)hipEventDestroy(p.e0);
    (void)hipEventDestroy(p.e1);
    (void)hipEventDestroy(p.e2);
    (void)hipEventDestroy(p.e3);
  }
  pending_.clear();
  return CCUBA_OK;
}

int VegasEngine::step(hipStream_t s) { return launch_iteration(s); }

int VegasEngine::graph_for(int k, hipStream_t s, hipGraphExec_t *out) {
  for (const auto &g : graphs_)
    if (g.k == k) {
      *out = g.exec;
      return CCUBA_OK;
    }
  CCUBA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  capturing_ = true;
  int rc = CCUBA_OK;
  for (int q = 0; q < k && rc == CCUBA_OK; ++q) rc = launch_iteration(s);
  capturing_ = false;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (rc == CCUBA_OK && e != hipSuccess) rc = CCUBA_EHIP;
  hipGraphExec_t exec = nullptr;
  if (rc == CCUBA_OK && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess)
    rc = CCUBA_EHIP;
  if (g) (void)hipGraphDestroy(g);
  if (rc) return rc;
  graphs_.push_back({k, exec});
  *out = exec;
  return CCUBA_OK;
}

bool VegasEngine::fixed() const {
  for (const auto &sp : specs_)
    if (sp.epsrel > 0 || sp.epsabs > 0) return false;
  return true;
}

int VegasEngine::run(hipStream_t s) {
  const int rc = launch_run(s);
  return rc ? rc : finish_run(s);
}

int VegasEngine::prepare_run(hipStream_t s) {
  if (!fixed() || ctx_->use_graph == 0 || ctx_->profile) return CCUBA_OK;
  // the chunks launch_run takes when no job can stop early
  for (int remaining = max_iters_; remaining > 0;) {
    const int k = std::min(remaining, kMaxGraphIters);
    hipGraphExec_t exec = nullptr;
    const int rc = graph_for(k, s, &exec);
    if (rc) return rc;
    remaining -= k;
  }
  return CCUBA_OK;
}

int VegasEngine::launch_run(hipStream_t s) {
  const bool fixed = this->fixed();
  int remaining = max_iters_;
  if (remaining == 0) return CCUBA_OK;
  // Iterations are launched in chunks between host checks of the states:
  // all of them at once when no job can stop early, else 2, 4, 8, ... (a
  // finished job's state makes the remaining launches of its chunk skip it).
  // With graphs on, a chunk of k iterations is one graph of 3k kernels, so
  // that consecutive iterations are not separated by graph launches.
  const bool graph = ctx_->use_graph != 0 && !ctx_->profile;
  int chunk = fixed ? std::min(remaining, kMaxGraphIters) : 2;
  std::vector<VState> st;
  while (remaining > 0) {
    const int k = std::min(chunk, remaining);
    if (graph) {
      hipGraphExec_t exec = nullptr;
      const int rc = graph_for(k, s, &exec);
      if (rc) return rc;
      CCUBA_HIP(hipGraphLaunch(exec, s));
    } else {
      for (int q = 0; q < k; ++q) {
        const int rc = launch_iteration(s);
        if (rc) return rc;
      }
    }
    remaining -= k;
    if (remaining > 0 && !fixed) {
      const int rc = read_states(st, s);
      if (rc) return rc;
      bool all = true;
      for (const auto &x : st) all = all && x.done;
      if (all) break;
      chunk = std::min(chunk * 2, kMaxGraphIters);
    }
  }
  return CCUBA_OK;
}

int VegasEngine::finish_run(hipStream_t s) {
  if (max_iters_ == 0) return CCUBA_OK;
  CCUBA_HIP(hipStreamSynchronize(s));
  std::vector<VState> st;
  if (ctx_->profile) {
    // every point a timed DoSample launch sampled is in some job's neval
    int rc = read_states(st, s);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(ctx_->stats_lock);
    for (const auto &x : st) ctx_->stats.evals += x.neval;
  }
  return flush_timing();
}

int VegasEngine::run_each(hipStream_t s, const std::function<int(const VState &)> &after) {
  std::vector<VState> st;
  int rc = read_states(st, s);
  if (rc) return rc;
  // the budget counts every iteration from t = 0, resumed ones included
  for (int t = st[0].T; t < max_iters_ && !st[0].done; ++t) {
    if ((rc = launch_iteration(s))) return rc;
    if ((rc = read_states(st, s))) return rc;
    if ((rc = after(st[0]))) return rc;
  }
  CCUBA_HIP(hipStreamSynchronize(s));
  return flush_timing();
}

int VegasEngine::load_checkpoint(const VState &st, const double *grid, const double *I,
                                 const double *var, hipStream_t s) {
  const VJob &J = hjobs_[0];
  if (st.T > J.hist_cap) return CCUBA_EINVAL;
  int rc = load_grid(0, grid, hipMemcpyHostToDevice, s);
  if (rc) return rc;
  if (st.T > 0) {
    CCUBA_HIP(hipMemcpyAsync(J.iter_I, I, st.T * sizeof(double), hipMemcpyHostToDevice, s));
    CCUBA_HIP(hipMemcpyAsync(J.iter_var, var, st.T * sizeof(double), hipMemcpyHostToDevice, s));
  }
  CCUBA_HIP(hipMemcpyAsync(state_.p, &st, sizeof(VState), hipMemcpyHostToDevice, s));
  CCUBA_HIP(hipStreamSynchronize(s));  // the host copies are the caller's
  return CCUBA_OK;
}

int VegasEngine::read_states(std::vector<VState> &out, hipStream_t s) {
  out.resize(njobs());
  CCUBA_HIP(hipMemcpyAsync(out.data(), state_.p, njobs() * sizeof(VState),
                           hipMemcpyDeviceToHost, s));
  CCUBA_HIP(hipStreamSynchronize(s));
  return CCUBA_OK;
}

int VegasEngine::read_history(int job, int n, double *I, double *var, hipStream_t s) {
  if (job < 0 || job >= njobs()) return CCUBA_EINVAL;
  n = std::min(n, hjobs_[job].hist_cap);
  if (n <= 0) return CCUBA_OK;
  if (I)
    CCUBA_HIP(hipMemcpyAsync(I, hjobs_[job].iter_I, n * sizeof(double),
                             hipMemcpyDeviceToHost, s));
  if (var)
    CCUBA_HIP(hipMemcpyAsync(var, hjobs_[job].iter_var, n * sizeof(double),
                             hipMemcpyDeviceToHost, s));
  CCUBA_HIP(hipStreamSynchronize(s));
  return CCUBA_OK;
}

int VegasEngine::read_grid(int job, double *grid, hipStream_t s) {
  if (job < 0 || job >= njobs()) return CCUBA_EINVAL;
  const VJob &J = hjobs_[job];
  const long long row = (long long)J.ndim * (J.nbins + 1);
  CCUBA_HIP(hipMemcpyAsync(grid, J.grid, row * sizeof(double), hipMemcpyDeviceToHost, s));
  CCUBA_HIP(hipStreamSynchronize(s));
  return CCUBA_OK;
}

int VegasEngine::read_step(int job, int t, double *grid, double *I, double *var,
                           hipStream_t s) {
  if (job < 0 || job >= njobs() || t < 0 || t >= hjobs_[job].hist_cap) return CCUBA_EINVAL;
  const VJob &J = hjobs_[job];
  const long long row = (long long)J.ndim * (J.nbins + 1);
  CCUBA_HIP(hipMemcpyAsync(grid, J.grid, row * sizeof(double), hipMemcpyDeviceToHost, s));
  CCUBA_HIP(hipMemcpyAsync(I, J.iter_I + t, sizeof(double), hipMemcpyDeviceToHost, s));
  CCUBA_HIP(hipMemcpyAsync(var, J.iter_var + t, sizeof(double), hipMemcpyDeviceToHost, s));
  CCUBA_HIP(hipStreamSynchronize(s));
  return CCUBA_OK;
}

int VegasEngine::set_iteration(int job, int t, hipStream_t s) {
  if (job < 0 || job >= njobs()) return CCUBA_EINVAL;
  VState st{};
  st.T = t;
  // the state is a pinned-free host value; copy synchronously to keep it alive
  CCUBA_HIP(hipMemcpyAsync(state_.p + job, &st, sizeof(VState), hipMemcpyHostToDevice, s));
  CCUBA_HIP(hipStreamSynchronize(s));
  return CCUBA_OK;
}

int VegasEngine::load_grid(int job, const double *src, hipMemcpyKind kind, hipStream_t s) {
  const VJob &J = hjobs_[job];
  const long long row = (long long)J.ndim * (J.nbins + 1);
  CCUBA_HIP(hipMemcpyAsync(J.grid, src, row * sizeof(double), kind, s));
  if (kind == hipMemcpyHostToDevice) CCUBA_HIP(hipStreamSynchronize(s));
  return CCUBA_OK;
}

int VegasEngine::collect(double *sums_dev, double *hist_dev, hipStream_t s) {
  CCUBA_HIP(launch_collect(args_, 1, sums_dev, hist_dev, s));
  return CCUBA_OK;
}

int VegasEngine::refine_only(const double *hist, const double *grid_in, double *grid_out,
                             hipStream_t s) {
  const VJob &J = hjobs_[0];
  const long long dN = (long long)J.ndim * J.nbins;
  int rc = load_grid(0, grid_in, hipMemcpyHostToDevice, s);
  if (rc) return rc;
  // a synthetic finished iteration with n = 2, S1 = 1, S2 = 2 (I = 1/2,
  // sigma^2 = 3/4 > 0, so the zero-tolerance job never converges)
  // (the refine kernel reads the group rows: row 0 holds it all)
  const double sums[2] = {1.0, 2.0};
  const long long ng = ngroups_of(J.ntiles);
  CCUBA_HIP(hipMemsetAsync(J.gsums, 0, 2 * ng * sizeof(double), s));
  CCUBA_HIP(hipMemsetAsync(J.ghist, 0, ng * dN * sizeof(double), s));
  CCUBA_HIP(hipMemcpyAsync(J.gsums, sums, sizeof(sums), hipMemcpyHostToDevice, s));
  CCUBA_HIP(hipMemcpyAsync(J.ghist, hist, dN * sizeof(double), hipMemcpyHostToDevice, s));
  CCUBA_HIP(hipStreamSynchronize(s));
  rc = set_iteration(0, 0, s);
  if (rc) return rc;
  // (the refine kernel reads the state through the snapshot the fold takes)
  CCUBA_HIP(hipMemcpyAsync(hjobs_[0].snap, hjobs_[0].state, sizeof(VState),
                           hipMemcpyDeviceToDevice, s));
  CCUBA_HIP(launch_refine(args_, 1, dmax_, s));
  return read_grid(0, grid_out, s);
}

}  // namespace ccuba
