// api.cpp -- the C ABI of libccuba (declared in include/ccuba.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <mutex>
#include <thread>

#include "ccuba.h"
#include "context.h"
#include "cuhre_engine.h"
#include "serve.h"
#include "tune.h"
#include "rtc.h"
#include "vegas_state.h"
#include "suave_engine.h"
#include "divonne_engine.h"
#include "vegas_batched.h"
#include "vegas_engine.h"
#include "noalloc.h"

void ccuba::note_hip_error(hipError_t e, const char *file, int line) {
  static const bool on = std::getenv("CCUBA_DEBUG") != nullptr;
  if (on) std::fprintf(stderr, "ccuba: %s at %s:%d\n", hipGetErrorString(e), file, line);
}

using namespace ccuba;

namespace ccuba {

namespace {

// Size classes: 256 B, then four steps per power of two (at most 25% unused).
size_t size_class(size_t bytes) {
  if (bytes <= 256) return 256;
  size_t p = 256;
  while (p * 2 < bytes) p *= 2;  // p < bytes <= 2p
  const size_t q = p / 4;
  return (bytes + q - 1) / q * q;
}

}  // namespace

int dev_alloc(ccuba_ctx *ctx, void **p, size_t bytes) {
  const size_t cls = size_class(bytes);
  {
    std::lock_guard<std::mutex> g(ctx->pool_lock);
    auto it = ctx->pool.find(cls);
    if (it != ctx->pool.end()) {
      if (ctx->used.load() + cls > ctx->budget) return CCUBA_ENOMEM;
      *p = it->second;
      ctx->pool.erase(it);
      ctx->pooled -= cls;
      ctx->used.fetch_add(cls);
      return CCUBA_OK;
    }
    if (ctx->used.load() + cls > ctx->budget) return CCUBA_ENOMEM;
    // pooled blocks count against the budget too: give them back first
    if (ctx->used.load() + ctx->pooled + cls > ctx->budget) {
      for (auto &kv : ctx->pool) (void)hipFree(kv.second);
      ctx->pool.clear();
      ctx->pooled = 0;
    }
    ctx->used.fetch_add(cls);
  }
  if (hipMalloc(p, cls) != hipSuccess) {
    // a full device: release the pool and try once more
    pool_release(ctx);
    if (hipMalloc(p, cls) != hipSuccess) {
      ctx->used.fetch_sub(cls);
      *p = nullptr;
      return CCUBA_ENOMEM;
    }
  }
  return CCUBA_OK;
}

void dev_free(ccuba_ctx *ctx, void *p, size_t bytes) {
  if (!p) return;
  const size_t cls = size_class(bytes);
  std::lock_guard<std::mutex> g(ctx->pool_lock);
  ctx->pool.emplace(cls, p);
  ctx->pooled += cls;
  ctx->used.fetch_sub(cls);
}

void pool_release(ccuba_ctx *ctx) {
  std::lock_guard<std::mutex> g(ctx->pool_lock);
  for (auto &kv : ctx->pool) (void)hipFree(kv.second);
  ctx->pool.clear();
  ctx->pooled = 0;
}

}  // namespace ccuba

namespace {

long long env_ll(const char *name, long long dflt) {
  const char *v = std::getenv(name);
  if (!v || !*v) return dflt;
  char *end = nullptr;
  const long long r = std::strtoll(v, &end, 10);
  return (end && *end == 0) ? r : dflt;
}

// The three cases of the paper's `spin' argument (Sect. 3.2.3).
struct CtxScope {
  ccuba_ctx *ctx = nullptr;
  bool temporary = false;
  int rc = CCUBA_OK;
  explicit CtxScope(ccuba_ctx **pp) {
    if (!pp) {
      rc = ccuba_init(&ctx, -1, 0);
      temporary = true;
    } else if (!*pp) {
      rc = ccuba_init(pp, -1, 0);
      ctx = *pp;
    } else {
      ctx = *pp;
    }
  }
  ~CtxScope() {
    if (temporary && ctx) ccuba_shutdown(&ctx);
  }
};

}  // namespace

namespace ccuba {
int pinned_block(ccuba_ctx *ctx, double **host, double **dev) {
  if (!ctx->pinned_host) {
    void *h = nullptr, *d = nullptr;
    // host-coherent: the device's system-scope stores to it are seen by a
    // polling host while the kernel runs
    if (hipHostMalloc(&h, ccuba_ctx::kPinnedBytes, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
      return CCUBA_EHIP;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
      (void)hipHostFree(h);
      return CCUBA_EHIP;
    }
    ctx->pinned_host = (double *)h;
    ctx->pinned_dev = (double *)d;
  }
  *host = ctx->pinned_host;
  *dev = ctx->pinned_dev;
  return CCUBA_OK;
}
}  // namespace ccuba

namespace {

void drop_engine_cache(ccuba_ctx *ctx) {
  delete ctx->vcache;
  ctx->vcache = nullptr;
}

// run a set-up single-integral engine to the end and read its results
int vegas_finish(ccuba_ctx *ctx, VegasEngine &eng, long long *neval, int *fail,
                 double integral[], double error[], double prob[], ccuba_vegas_trace *trace);
// The outputs of a finished run of job 0.
int vegas_results(ccuba_ctx *ctx, VegasEngine &eng, long long *neval, int *fail,
                  double integral[], double error[], double prob[], ccuba_vegas_trace *trace);

int fill_spec(VegasSpec &sp, int ndim, int ncomp, const ccuba_integrand *f, double epsrel,
              double epsabs, int flags, unsigned long long seed, long long mineval,
              long long maxeval, long long nstart, long long nincrease, long long nbatch,
              int nbins, unsigned int stream_id) {
  if (!f || ncomp != 1 || nbatch < 1 || ndim < 1 || ndim > kMaxDim || !f->a || !f->u)
    return CCUBA_EINVAL;
  const int prec = flags & CCUBA_PRECISION_MASK;
  if (prec != CCUBA_FP64 && prec != CCUBA_FP32_EVAL) return CCUBA_EINVAL;
  sp.ndim = ndim;
  sp.nbins = nbins;
  sp.family = f->family;
  sp.prec = prec == CCUBA_FP64 ? FP64 : FP32;
  sp.flags = flags & CCUBA_FREEZE_GRID;
  sp.seed = seed;
  sp.sid = stream_id;
  sp.nstart = nstart;
  sp.nincrease = nincrease;
  sp.mineval = mineval;
  sp.maxeval = maxeval;
  sp.epsrel = epsrel;
  sp.epsabs = epsabs;
  for (int j = 0; j < ndim; ++j) {
    sp.a[j] = f->a[j];
    sp.u[j] = f->u[j];
  }
  return validate_vegas(sp);
}

}  // namespace

extern "C" {

const char *ccuba_strerror(int status) {
  switch (status) {
    case CCUBA_OK: return "success";
    case CCUBA_EINVAL: return "invalid argument";
    case CCUBA_EHIP: return "HIP runtime error";
    case CCUBA_ENOMEM: return "device memory budget exceeded";
    case CCUBA_ENOENT: return "unknown ticket or key";
    case CCUBA_ESTATE: return "not allowed in the current state";
  }
  return "unknown status";
}

int ccuba_init(ccuba_ctx **ctx, int device, size_t hbm_budget) {
  if (!ctx) return CCUBA_EINVAL;
  *ctx = nullptr;
  if (device < 0) device = (int)env_ll("CCUBA_DEVICE", 0);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return CCUBA_EHIP;
  if (device >= ndev) return CCUBA_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return CCUBA_EHIP;
  std::unique_ptr<ccuba_ctx> c(new (std::nothrow) ccuba_ctx());
  if (!c) return CCUBA_ENOMEM;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return CCUBA_EHIP;
  c->ncu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  if (hbm_budget == 0) hbm_budget = (size_t)env_ll("CCUBA_HBM_BUDGET", 0);
  if (hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return CCUBA_EHIP;
    hbm_budget = fr / 10 * 9;
  }
  c->budget = hbm_budget;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return CCUBA_EHIP;
  if (hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) != hipSuccess) return CCUBA_EHIP;
  if (set_kernel_limits() != hipSuccess) return CCUBA_EHIP;
  // the allocation-free entry point's scratch: its address on this device
  if (noalloc_init(device) != CCUBA_OK) return CCUBA_EHIP;
  if (suave_set_kernel_limits() != hipSuccess) return CCUBA_EHIP;
  if (cuhre_set_kernel_limits() != hipSuccess) return CCUBA_EHIP;
  for (int p = 0; p < 2; ++p) {
    c->tune[p].block = (int)env_ll("CCUBA_BLOCK", 256);
    c->tune[p].blocks_per_cu = (int)env_ll("CCUBA_BLOCKS_PER_CU", 3);
    c->tune[p].min_tile = env_ll("CCUBA_MIN_TILE", 16384);
    // measured best on gfx950: two points per lane for FP32, one for FP64
    c->tune[p].ilp = (int)env_ll("CCUBA_ILP", p == FP32 ? 2 : 1) == 2 ? 2 : 1;
    c->tune[p].streams = env_ll("CCUBA_BATCH_STREAMS", 2) == 1 ? 1 : 2;
  }
  // LDS histogram: the exact fixed-point one for FP32 evaluation (faster
  // than FP64 LDS adds); FP64 LDS adds for FP64 evaluation, where the exact
  // one (two integer adds per bin, and order-independent, so reruns give the
  // same bits) measured 12% slower per step; CCUBA_HIST64 sets both
  c->tune[FP32].hist64 = (int)env_ll("CCUBA_HIST64", 0);
  c->tune[FP64].hist64 = (int)env_ll("CCUBA_HIST64", 1);
  c->use_graph = (int)env_ll("CCUBA_GRAPH", 1);
  c->autotune = (int)env_ll("CCUBA_AUTOTUNE", 0);
  c->serve_slots = (int)env_ll("CCUBA_SERVE_SLOTS", 256);
  for (int p = 0; p < 2; ++p) {
    const int b = c->tune[p].block;
    if (b != 64 && b != 128 && b != 256) c->tune[p].block = 256;
    c->tune[p].blocks_per_cu = std::min(16, std::max(1, c->tune[p].blocks_per_cu));
  }
  *ctx = c.release();
  return CCUBA_OK;
}

int ccuba_shutdown(ccuba_ctx **ctx) {
  if (!ctx || !*ctx) return CCUBA_OK;
  ccuba_ctx *c = *ctx;
  (void)hipSetDevice(c->device);
  delete c->server;  // stops the serving thread and frees its requests
  c->server = nullptr;
  drop_engine_cache(c);
  rtc_release(c);
  if (c->pinned_host) (void)hipHostFree(c->pinned_host);
  pool_release(c);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  if (c->stream2) (void)hipStreamDestroy(c->stream2);
  delete c;
  *ctx = nullptr;
  return CCUBA_OK;
}

int ccuba_config_get(ccuba_ctx *ctx, const char *key, int precision, long long *value) {
  if (!ctx || !key || !value || (precision != CCUBA_FP64 && precision != CCUBA_FP32_EVAL))
    return CCUBA_EINVAL;
  std::lock_guard<std::mutex> g(ctx->lock);
  const VegasTune &t = ctx->tune[precision == CCUBA_FP64 ? FP64 : FP32];
  const std::string k(key);
  if (k == "block")
    *value = t.block;
  else if (k == "blocks_per_cu")
    *value = t.blocks_per_cu;
  else if (k == "hist64")
    *value = t.hist64;
  else if (k == "ilp")
    *value = t.ilp;
  else if (k == "min_tile")
    *value = t.min_tile;
  else if (k == "autotune")
    *value = ctx->autotune;
  else if (k == "graph")
    *value = ctx->use_graph;
  else if (k == "profile")
    *value = ctx->profile;
  else if (k == "serve_slots")
    *value = ctx->serve_slots;
  else if (k == "engine_cache")
    *value = ctx->engine_cache;
  else if (k == "batch_streams")
    *value = t.streams;
  else
    return CCUBA_ENOENT;
  return CCUBA_OK;
}

int ccuba_config(ccuba_ctx *ctx, const char *key, long long value) {
  if (!ctx || !key) return CCUBA_EINVAL;
  std::lock_guard<std::mutex> g(ctx->lock);
  const std::string k(key);
  if (k == "block") {
    if (value != 64 && value != 128 && value != 256) return CCUBA_EINVAL;
    ctx->tune[0].block = ctx->tune[1].block = (int)value;
  } else if (k == "blocks_per_cu") {
    if (value < 1 || value > 16) return CCUBA_EINVAL;
    ctx->tune[0].blocks_per_cu = ctx->tune[1].blocks_per_cu = (int)value;
  } else if (k == "hist64") {
    if (value != 0 && value != 1) return CCUBA_EINVAL;
    ctx->tune[0].hist64 = ctx->tune[1].hist64 = (int)value;
  } else if (k == "ilp") {
    if (value != 1 && value != 2) return CCUBA_EINVAL;
    ctx->tune[0].ilp = ctx->tune[1].ilp = (int)value;
  } else if (k == "min_tile") {
    if (value < 64) return CCUBA_EINVAL;
    ctx->tune[0].min_tile = ctx->tune[1].min_tile = value;
  } else if (k == "autotune") {
    ctx->autotune = value != 0;
  } else if (k == "graph") {
    ctx->use_graph = value != 0;
  } else if (k == "engine_cache") {
    ctx->engine_cache = value != 0;
    if (!ctx->engine_cache) drop_engine_cache(ctx);
  } else if (k == "profile") {
    ctx->profile = value != 0;
  } else if (k == "serve_slots") {
    if (value < 1 || value > 1 << 20) return CCUBA_EINVAL;
    ctx->serve_slots = (int)value;
  } else if (k == "batch_streams") {
    if (value != 1 && value != 2) return CCUBA_EINVAL;
    ctx->tune[0].streams = ctx->tune[1].streams = (int)value;
  } else {
    return CCUBA_ENOENT;
  }
  return CCUBA_OK;
}

int ccuba_stats_get(ccuba_ctx *ctx, ccuba_stats *out, int reset) {
  if (!ctx || !out) return CCUBA_EINVAL;
  std::lock_guard<std::mutex> g(ctx->lock);
  *out = ctx->stats;
  if (reset) ctx->stats = ccuba_stats{};
  return CCUBA_OK;
}

int ccuba_vegas_stateful(ccuba_ctx **ctxp, int ndim, int ncomp, const ccuba_integrand *f,
                         double epsrel, double epsabs, int flags, unsigned long long seed,
                         long long mineval, long long maxeval, long long nstart,
                         long long nincrease, long long nbatch, int gridno, const char *statefile,
                         int nbins, unsigned int stream_id, long long *neval, int *fail,
                         double integral[], double error[], double prob[],
                         ccuba_vegas_trace *trace) {
  if (!neval || !fail || !integral || !error || !prob) return CCUBA_EINVAL;
  VegasSpec sp;
  int rc = fill_spec(sp, ndim, ncomp, f, epsrel, epsabs, flags, seed, mineval, maxeval, nstart,
                     nincrease, nbatch, nbins, stream_id);
  if (rc) return rc;
  const bool checkpoint = statefile && *statefile;
  CtxScope scope(ctxp);
  if (scope.rc) return scope.rc;
  ccuba_ctx *ctx = scope.ctx;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  if (ctx->autotune) maybe_autotune(ctx, sp.prec);
  hipStream_t s = ctx->stream;
  VegasEngine eng(ctx);
  if ((rc = eng.setup({sp}, true, s))) return rc;
  const size_t row = (size_t)ndim * (nbins + 1);
  bool resumed = false;
  StateFile sf;
  if (checkpoint) {
    rc = state_read(statefile, sp, sf);
    if (rc < 0) return rc;
    if (rc == 0) {
      if (sf.st.T > eng.max_iters()) return CCUBA_EINVAL;  // more than this budget allows
      if (sf.st.done && sf.st.fail == 1 && sf.st.T < eng.max_iters()) {
        // stopped by an earlier, smaller budget: this one allows more
        sf.st.done = 0;
        sf.st.fail = 0;
        sf.st.chi2 = sf.st.prob = 0.0;
      }
      if ((rc = eng.load_checkpoint(sf.st, sf.grid.data(), sf.I.data(), sf.var.data(), s)))
        return rc;
      resumed = true;
    }
  }
  if (!resumed && gridno != 0) {  // an earlier integration's grid, if its shape fits
    auto it = ctx->grid_table.find(gridno > 0 ? gridno : -gridno);
    if (it != ctx->grid_table.end() && it->second.first == std::make_pair(ndim, nbins))
      if ((rc = eng.load_grid(0, it->second.second.data(), hipMemcpyHostToDevice, s))) return rc;
  }
  if (checkpoint) {
    // the history is kept on the host (a resumed file's first) and grows by
    // the one iteration just done
    if (!resumed) {
      sf.I.clear();
      sf.var.clear();
    }
    rc = eng.run_each(s, [&](const VState &st) {
      sf.st = st;
      sf.grid.resize(row);
      sf.I.resize(st.T);
      sf.var.resize(st.T);
      const int t = st.T - 1;
      const int r = eng.read_step(0, t, sf.grid.data(), &sf.I[t], &sf.var[t], s);
      if (r) return r;
      return state_write(statefile, sp, sf);
    });
  } else {
    rc = eng.run(s);
  }
  if (rc) return rc;
  if ((rc = vegas_results(ctx, eng, neval, fail, integral, error, prob, trace))) return rc;
  if (checkpoint && *fail == 0) std::remove(statefile);  // converged: nothing to resume
  if (gridno > 0) {
    std::vector<double> grid(row);
    if ((rc = eng.read_grid(0, grid.data(), s))) return rc;
    ctx->grid_table[gridno] = {{ndim, nbins}, std::move(grid)};
  }
  return CCUBA_OK;
}

int ccuba_vegas_source(ccuba_ctx **ctxp, int ndim, const char *source, const double *a,
                       const double *u, double epsrel, double epsabs, int flags,
                       unsigned long long seed, long long mineval, long long maxeval,
                       long long nstart, long long nincrease, long long nbatch, int nbins,
                       unsigned int stream_id, long long *neval, int *fail, double integral[],
                       double error[], double prob[]) {
  if (!source || !neval || !fail || !integral || !error || !prob || ndim < 1 || ndim > kMaxDim)
    return CCUBA_EINVAL;
  // the parameters a and u (zeros when absent) reach the function as given
  double za[kMaxDim] = {0}, zu[kMaxDim] = {0};
  const ccuba_integrand f{GAUSSIAN, a ? a : za, u ? u : zu};
  VegasSpec sp;
  int rc = fill_spec(sp, ndim, 1, &f, epsrel, epsabs, flags, seed, mineval, maxeval, nstart,
                     nincrease, nbatch, nbins, stream_id);
  if (rc) return rc;
  sp.family = USER;
  CtxScope scope(ctxp);
  if (scope.rc) return scope.rc;
  ccuba_ctx *ctx = scope.ctx;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  if (ctx->autotune) maybe_autotune(ctx, sp.prec);
  const VegasTune &t = ctx->tune[sp.prec];
  const int nb = (ndim + 3) / 4;
  hipFunction_t fn = nullptr;
  // the histogram type the engine's tile group of this class will take
  const int h64 = fixed_hist(sp.prec, t.hist64, (long long)ndim * nbins) ? 0 : 1;
  rc = rtc_dosample(ctx, source, sp.prec, h64, t.ilp, nb, (nbins & (nbins - 1)) == 0,
                    ndim == 4 * nb, &fn);
  if (rc) return rc;
  // an engine of its own: the cached one's graphs hold the built-in kernels
  VegasEngine eng(ctx);
  eng.set_user_kernel(fn);
  if ((rc = eng.setup({sp}, true, ctx->stream))) return rc;
  return vegas_finish(ctx, eng, neval, fail, integral, error, prob, nullptr);
}

int ccuba_rtc_log(ccuba_ctx *ctx, char *buf, size_t size) {
  if (!ctx || !buf || size == 0) return CCUBA_EINVAL;
  std::lock_guard<std::mutex> g(ctx->lock);
  const std::string &log = ctx->rtc ? ctx->rtc->log : std::string();
  const size_t n = std::min(size - 1, log.size());
  std::memcpy(buf, log.data(), n);
  buf[n] = '\0';
  return CCUBA_OK;
}

int ccuba_vegas_batched(ccuba_ctx **ctxp, int ndim, int ncomp, ccuba_batch_integrand integrand,
                        void *userdata, int nvec, int where, double epsrel, double epsabs,
                        int flags, unsigned long long seed, long long mineval,
                        long long maxeval, long long nstart, long long nincrease, int nbins,
                        unsigned int stream_id, long long *neval, int *fail, double integral[],
                        double error[], double prob[]) {
  const int prec = flags & CCUBA_PRECISION_MASK;
  if (!integrand || !neval || !fail || !integral || !error || !prob || ndim < 1 ||
      ndim > kMaxDim || ncomp < 1 || ncomp > kMaxComp || nbins < 2 || nbins > kMaxBins ||
      nvec < 1 || (where != CCUBA_POINTS_HOST && where != CCUBA_POINTS_DEVICE) ||
      (prec != CCUBA_FP64 && prec != CCUBA_FP32_EVAL) || nstart < 2 ||
      nstart >= (1ll << 32) || nincrease < 0 || maxeval < 0 || mineval < 0 ||
      !(epsrel >= 0) || !(epsabs >= 0))
    return CCUBA_EINVAL;
  BatchedSpec sp;
  sp.ndim = ndim;
  sp.ncomp = ncomp;
  sp.nbins = nbins;
  sp.prec = prec == CCUBA_FP32_EVAL ? FP32 : FP64;
  sp.flags = flags;
  sp.nvec = nvec;
  sp.where = where;
  sp.seed = seed;
  sp.sid = stream_id;
  sp.nstart = nstart;
  sp.nincrease = nincrease;
  sp.mineval = mineval;
  sp.maxeval = maxeval;
  sp.epsrel = epsrel;
  sp.epsabs = epsabs;
  CtxScope scope(ctxp);
  if (scope.rc) return scope.rc;
  ccuba_ctx *ctx = scope.ctx;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  return vegas_batched(ctx, sp, integrand, userdata, neval, fail, integral, error, prob);
}

int ccuba_vegas_ex(ccuba_ctx **ctxp, int ndim, int ncomp, const ccuba_integrand *f,
                   double epsrel, double epsabs, int flags, unsigned long long seed,
                   long long mineval, long long maxeval, long long nstart,
                   long long nincrease, long long nbatch, int nbins, unsigned int stream_id,
                   long long *neval, int *fail, double integral[], double error[],
                   double prob[], ccuba_vegas_trace *trace) {
  if (!neval || !fail || !integral || !error || !prob) return CCUBA_EINVAL;
  VegasSpec sp;
  int rc = fill_spec(sp, ndim, ncomp, f, epsrel, epsabs, flags, seed, mineval, maxeval,
                     nstart, nincrease, nbatch, nbins, stream_id);
  if (rc) return rc;
  CtxScope scope(ctxp);
  if (scope.rc) return scope.rc;
  ccuba_ctx *ctx = scope.ctx;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  if (ctx->autotune) maybe_autotune(ctx, sp.prec);
  // the context's cached engine (its buffers and graphs serve the next call
  // of the same shape), or a fresh one when caching is off
  std::unique_ptr<VegasEngine> own;
  VegasEngine *ep;
  if (ctx->engine_cache) {
    if (!ctx->vcache) ctx->vcache = new VegasEngine(ctx);
    ep = ctx->vcache;
  } else {
    own.reset(new VegasEngine(ctx));
    ep = own.get();
  }
  VegasEngine &eng = *ep;
  rc = eng.setup({sp}, true, ctx->stream);
  if (rc == CCUBA_ENOMEM && ctx->vcache) {
    // the cached buffers may be what exceeds the budget: start afresh
    drop_engine_cache(ctx);
    own.reset(new VegasEngine(ctx));
    rc = own->setup({sp}, true, ctx->stream);
    if (rc) return rc;
    return vegas_finish(ctx, *own, neval, fail, integral, error, prob, trace);
  }
  if (rc) {
    drop_engine_cache(ctx);
    return rc;
  }
  rc = vegas_finish(ctx, eng, neval, fail, integral, error, prob, trace);
  if (rc) drop_engine_cache(ctx);
  return rc;
}

namespace {
int vegas_results(ccuba_ctx *ctx, VegasEngine &eng, long long *neval, int *fail,
                  double integral[], double error[], double prob[], ccuba_vegas_trace *trace) {
  int rc;
  std::vector<VState> st;
  if ((rc = eng.read_states(st, ctx->stream))) return rc;
  *neval = st[0].neval;
  *fail = st[0].fail;
  integral[0] = st[0].integral;
  error[0] = st[0].error;
  prob[0] = st[0].prob;
  if (trace) {
    trace->n_iter = st[0].T;
    trace->chi2 = st[0].chi2;
    trace->dof = st[0].dof;
    const int n = std::min(trace->max_iter, st[0].T);
    if (n > 0 && (trace->iter_I || trace->iter_var))
      if ((rc = eng.read_history(0, n, trace->iter_I, trace->iter_var, ctx->stream))) return rc;
    if (trace->grid)
      if ((rc = eng.read_grid(0, trace->grid, ctx->stream))) return rc;
  }
  return CCUBA_OK;
}

int vegas_finish(ccuba_ctx *ctx, VegasEngine &eng, long long *neval, int *fail,
                 double integral[], double error[], double prob[], ccuba_vegas_trace *trace) {
  const int rc = eng.run(ctx->stream);
  if (rc) return rc;
  return vegas_results(ctx, eng, neval, fail, integral, error, prob, trace);
}
}  // namespace

int ccuba_vegas(ccuba_ctx **ctx, int ndim, int ncomp, const ccuba_integrand *f, double epsrel,
                double epsabs, int flags, unsigned long long seed, long long mineval,
                long long maxeval, long long nstart, long long nincrease, long long nbatch,
                int nbins, unsigned int stream_id, long long *neval, int *fail,
                double integral[], double error[], double prob[]) {
  return ccuba_vegas_ex(ctx, ndim, ncomp, f, epsrel, epsabs, flags, seed, mineval, maxeval,
                        nstart, nincrease, nbatch, nbins, stream_id, neval, fail, integral,
                        error, prob, nullptr);
}

int ccuba_vegas_points(ccuba_ctx *ctx, int ndim, int nbins, int flags, unsigned long long seed,
                       unsigned int stream_id, int iteration, const double *grid, long long i0,
                       long long npts, uint32_t *words, double *x, double *w, int *bin) {
  if (!ctx || !grid || ndim < 1 || ndim > kMaxDim || nbins < 2 || nbins > kMaxBins ||
      npts < 0 || i0 < 0 || i0 + npts > (1ll << 32) || iteration < 0 ||
      iteration >= (1 << 24))
    return CCUBA_EINVAL;
  const int prec = flags & CCUBA_PRECISION_MASK;
  if (prec != CCUBA_FP64 && prec != CCUBA_FP32_EVAL) return CCUBA_EINVAL;
  if (npts == 0) return CCUBA_OK;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  const int nblk = (ndim + 3) / 4;
  const size_t row = (size_t)ndim * (nbins + 1);
  DevBuf<double> dgrid, dx, dw;
  DevBuf<uint32_t> dwords;
  DevBuf<int> dbin;
  int rc;
  if ((rc = dgrid.alloc(ctx, row)) || (rc = dx.alloc(ctx, (size_t)npts * ndim)) ||
      (rc = dw.alloc(ctx, npts)) || (rc = dwords.alloc(ctx, (size_t)npts * 4 * nblk)) ||
      (rc = dbin.alloc(ctx, (size_t)npts * ndim)))
    return rc;
  CCUBA_HIP(hipMemcpyAsync(dgrid.p, grid, row * sizeof(double), hipMemcpyHostToDevice,
                           ctx->stream));
  PointsArgs P;
  P.ndim = ndim;
  P.nbins = nbins;
  P.prec = prec == CCUBA_FP64 ? FP64 : FP32;
  P.iteration = iteration;
  P.key0 = (uint32_t)(seed & 0xffffffffull);
  P.key1 = (uint32_t)(seed >> 32);
  P.sid = stream_id;
  P.i0 = i0;
  P.npts = npts;
  P.grid = dgrid.p;
  P.words = dwords.p;
  P.x = dx.p;
  P.w = dw.p;
  P.bin = dbin.p;
  CCUBA_HIP(launch_points(P, ctx->stream));
  if (words)
    CCUBA_HIP(hipMemcpyAsync(words, dwords.p, (size_t)npts * 4 * nblk * 4,
                             hipMemcpyDeviceToHost, ctx->stream));
  if (x)
    CCUBA_HIP(hipMemcpyAsync(x, dx.p, (size_t)npts * ndim * 8, hipMemcpyDeviceToHost,
                             ctx->stream));
  if (w)
    CCUBA_HIP(hipMemcpyAsync(w, dw.p, (size_t)npts * 8, hipMemcpyDeviceToHost, ctx->stream));
  if (bin)
    CCUBA_HIP(hipMemcpyAsync(bin, dbin.p, (size_t)npts * ndim * 4, hipMemcpyDeviceToHost,
                             ctx->stream));
  CCUBA_HIP(hipStreamSynchronize(ctx->stream));
  return CCUBA_OK;
}

int ccuba_vegas_refine(ccuba_ctx *ctx, int ndim, int nbins, const double *hist,
                       const double *grid_in, double *grid_out) {
  if (!ctx || !hist || !grid_in || !grid_out || ndim < 1 || ndim > kMaxDim || nbins < 2 ||
      nbins > kMaxBins)
    return CCUBA_EINVAL;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  VegasSpec sp;
  sp.ndim = ndim;
  sp.nbins = nbins;
  sp.nstart = 2;
  sp.maxeval = 1ll << 40;
  VegasEngine eng(ctx);
  int rc = eng.setup({sp}, true, ctx->stream);
  if (rc) return rc;
  return eng.refine_only(hist, grid_in, grid_out, ctx->stream);
}

int ccuba_vegas_dosample_raw(ccuba_ctx *ctx, int ndim, int nbins, const ccuba_integrand *f,
                             int flags, unsigned long long seed, unsigned int stream_id,
                             int iteration, long long npts, const double *grid_dev,
                             double *sums_dev, double *hist_dev, void *hip_stream) {
  if (!ctx || !grid_dev || !sums_dev || !hist_dev || iteration < 0 || iteration >= (1 << 24) ||
      npts < 2)
    return CCUBA_EINVAL;
  VegasSpec sp;
  int rc = fill_spec(sp, ndim, 1, f, 0.0, 0.0, flags & CCUBA_PRECISION_MASK, seed, 0,
                     1ll << 62, npts, 0, 1, nbins, stream_id);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  VegasEngine eng(ctx);
  if ((rc = eng.setup({sp}, true, s))) return rc;
  if ((rc = eng.set_iteration(0, iteration, s))) return rc;
  if ((rc = eng.load_grid(0, grid_dev, hipMemcpyDeviceToDevice, s))) return rc;
  if ((rc = eng.dosample_only(s, true))) return rc;
  if ((rc = eng.collect(sums_dev, hist_dev, s))) return rc;
  // the engine's buffers are released on return: finish before that
  CCUBA_HIP(hipStreamSynchronize(s));
  return CCUBA_OK;
}

int ccuba_vegas_dosample_raw_noalloc(ccuba_ctx *ctx, int ndim, int nbins,
                                     const ccuba_integrand *f, int flags,
                                     unsigned long long seed, unsigned int stream_id,
                                     int iteration, long long npts, const double *grid_dev,
                                     double *sums_dev, double *hist_dev, void *hip_stream) {
  if (!ctx || !grid_dev || !sums_dev || !hist_dev || iteration < 0 || iteration >= (1 << 24) ||
      npts < 2)
    return CCUBA_EINVAL;
  VegasSpec sp;
  int rc = fill_spec(sp, ndim, 1, f, 0.0, 0.0, flags & CCUBA_PRECISION_MASK, seed, 0,
                     1ll << 62, npts, 0, 1, nbins, stream_id);
  if (rc) return rc;
  if (validate_vegas(sp) != CCUBA_OK) return CCUBA_EINVAL;
  std::lock_guard<std::mutex> g(ctx->lock);
  unsigned char *base = (unsigned char *)noalloc_scratch(ctx->device);
  if (!base) return CCUBA_EHIP;
  CCUBA_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  const int p = sp.prec;
  const VegasTune &t = ctx->tune[p];
  const long long dN = (long long)ndim * nbins, row = (2 + dN) * 8;
  // Layout, 256-byte aligned: descriptor, state, fold ends, parameters, the
  // folded sums, then per tile and per group of 32 tiles a row of sums and
  // histogram.  Tiles as the allocating entry point takes them (one per
  // persistent block); fewer and larger when their rows would not fit.
  auto a256 = [](long long b) { return (b + 255) / 256 * 256; };
  static_assert(sizeof(VJob) <= 256 && sizeof(VState) <= 256 &&
                    2 * kParamRow * sizeof(double) <= 256 && 2 * kParamRow * sizeof(float) <= 256,
                "the scratch header's slots");
  static_assert(sizeof(NoallocSetup) <= 4096, "kernel arguments");
  const long long o_st = 256, o_end = 512, o_p64 = 768, o_p32 = 1024, o_hsum = 1280;
  const long long o_rows = o_hsum + a256(row);
  const long long avail = (long long)kNoallocScratchBytes - o_rows - 1024;
  const long long bs = t.block, B = (long long)ctx->ncu * t.blocks_per_cu;
  auto round_up = [](long long v, long long m) { return (v + m - 1) / m * m; };
  auto bytes_for = [&](long long nt) {
    return a256(nt * 16) + a256(nt * dN * 8) + a256((long long)ngroups_of((int)nt) * row);
  };
  long long P = std::max(round_up((npts + B - 1) / B, bs), bs);
  long long nt = (npts + P - 1) / P;
  for (long long fit = avail / (row + row / kGroupTiles + 64); bytes_for(nt) > avail;
       fit -= std::max(1ll, fit / 64)) {
    if (fit < ctx->ncu) return CCUBA_ENOMEM;  // not even one tile per compute unit
    P = std::max(round_up((npts + fit - 1) / fit, bs), bs);
    nt = (npts + P - 1) / P;
  }
  if (P > 0x7fffffffll) return CCUBA_ENOMEM;
  const int ng = ngroups_of((int)nt);
  const long long o_tsums = o_rows, o_thist = o_tsums + a256(nt * 16);
  const long long o_gsums = o_thist + a256(nt * dN * 8), o_ghist = o_gsums + a256(ng * 16);

  NoallocSetup S{};
  VJob &J = S.job;
  J.ndim = ndim;
  J.nbins = nbins;
  J.family = sp.family;
  J.prec = p;
  J.flags = sp.flags;
  J.key0 = (uint32_t)(sp.seed & 0xffffffffull);
  J.key1 = (uint32_t)(sp.seed >> 32);
  J.sid = sp.sid;
  J.nstart = npts;
  J.maxeval = sp.maxeval;
  J.tile0 = 0;
  J.ntiles = (int)nt;
  J.tile_pts = P;
  J.hist_cap = 1;
  J.state = (VState *)(base + o_st);
  J.grid = const_cast<double *>(grid_dev);  // read only: no refinement here
  J.tsums = (double *)(base + o_tsums);
  J.thist = (double *)(base + o_thist);
  J.gsums = (double *)(base + o_gsums);
  J.ghist = (double *)(base + o_ghist);
  J.hsum = (double *)(base + o_hsum);
  J.p64 = (const double *)(base + o_p64);
  J.p32 = (const float *)(base + o_p32);
  S.st.T = iteration;  // the rest zero: the state before its first iteration
  genz_constants(sp, S.p64, S.p32);
  const long long nch = (dN + 63) / 64;
  S.ends[0] = (long long)ng * nch;
  S.ends[1] = nch;
  S.job_dst = (VJob *)base;
  S.st_dst = J.state;
  S.p64_dst = (double *)(base + o_p64);
  S.p32_dst = (float *)(base + o_p32);
  S.ends_dst = (long long *)(base + o_end);
  CCUBA_HIP(launch_noalloc_setup(S, s));

  VegasArgs A{};
  A.jobs = S.job_dst;
  A.tile_job = nullptr;  // one job: the kernels look no tile up
  A.tile_first = 0;
  A.tile_count = (int)nt;
  A.njobs = 1;
  A.ilp = t.ilp;
  A.hist64 = fixed_hist(p, t.hist64, dN) ? 0 : 1;
  const size_t grid_bytes = (size_t)(dN * (p == FP64 ? 16 : 8) + 15) / 16 * 16;
  const size_t hsz = A.hist64 ? 8 : (p == FP64 ? 24 : 16);
  A.lds_hist_byte_off = (long long)grid_bytes;
  const int nb = (ndim + 3) / 4;
  CCUBA_HIP(launch_dosample(A, p, nb, (nbins & (nbins - 1)) == 0, ndim == 4 * nb,
                            (int)std::min<long long>(B, nt), (int)bs,
                            grid_bytes + (size_t)dN * hsz, s));
  FoldArgs F{S.job_dst, S.ends_dst, 1, S.ends[0], S.ends_dst + 1, S.ends[1]};
  CCUBA_HIP(launch_fold(F, true, s));
  CCUBA_HIP(launch_collect(A, 1, sums_dev, hist_dev, s));
  return CCUBA_OK;
}

int ccuba_cuhre(ccuba_ctx **ctxp, int ndim, int ncomp, const ccuba_integrand *f, double epsrel,
                double epsabs, int flags, long long mineval, long long maxeval, int key,
                long long max_regions_per_batch, int *nregions, long long *neval, int *fail,
                double integral[], double error[], double prob[]) {
  if (!f || !f->a || !f->u || ncomp != 1 || (key != 0 && key != 7) || !nregions || !neval ||
      !fail || !integral || !error || !prob || ndim < 2 || ndim > kMaxDim ||
      (flags & CCUBA_PRECISION_MASK) != CCUBA_FP64)
    return CCUBA_EINVAL;
  CuhreSpec sp;
  sp.ndim = ndim;
  sp.family = f->family;
  for (int j = 0; j < ndim; ++j) {
    sp.a[j] = f->a[j];
    sp.u[j] = f->u[j];
  }
  sp.epsrel = epsrel;
  sp.epsabs = epsabs;
  sp.mineval = mineval;
  sp.maxeval = maxeval;
  sp.batch = max_regions_per_batch;
  if (validate_cuhre(sp)) return CCUBA_EINVAL;
  CtxScope scope(ctxp);
  if (scope.rc) return scope.rc;
  ccuba_ctx *ctx = scope.ctx;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  CuhreRun run(ctx);
  int rc;
  double *ph = nullptr, *pd = nullptr;
  if ((rc = pinned_block(ctx, &ph, &pd))) return rc;
  run.set_mapped_totals(ph, pd);
  if ((rc = run.start(sp, ctx->stream)) || (rc = run.run(ctx->stream))) return rc;
  *nregions = (int)std::min<long long>(run.nregions(), 0x7fffffff);
  *neval = run.neval();
  *fail = run.fail();
  integral[0] = run.integral();
  error[0] = run.error();
  prob[0] = 0.0;
  return CCUBA_OK;
}

int ccuba_suave(ccuba_ctx **ctxp, int ndim, int ncomp, const ccuba_integrand *f, double epsrel,
                double epsabs, int flags, unsigned long long seed, long long mineval,
                long long maxeval, long long nnew, double flatness, int nbins, int nsplit,
                unsigned int stream_id, int *nregions, long long *neval, int *fail,
                double integral[], double error[], double prob[], ccuba_suave_trace *trace) {
  if (!f || !f->a || !f->u || ncomp != 1 || !nregions || !neval || !fail || !integral ||
      !error || !prob || ndim < 1 || ndim > kMaxDim ||
      (flags & CCUBA_PRECISION_MASK) != CCUBA_FP64 || (flags & ~(CCUBA_PRECISION_MASK |
                                                                 CCUBA_FREEZE_GRID)))
    return CCUBA_EINVAL;
  SuaveSpec sp;
  sp.ndim = ndim;
  sp.nbins = nbins;
  sp.family = f->family;
  sp.flags = flags & CCUBA_FREEZE_GRID ? FLAG_FREEZE_GRID : 0;
  for (int j = 0; j < ndim; ++j) {
    sp.a[j] = f->a[j];
    sp.u[j] = f->u[j];
  }
  sp.seed = seed;
  sp.sid = stream_id;
  sp.epsrel = epsrel;
  sp.epsabs = epsabs;
  sp.mineval = mineval;
  sp.maxeval = maxeval;
  sp.nnew = nnew;
  sp.flatness = flatness;
  sp.nsplit = nsplit;
  if (validate_suave(sp)) return CCUBA_EINVAL;
  if (trace && ((trace->max_regions > 0 && (!trace->lo || !trace->hi || !trace->I ||
                                            !trace->var)) ||
                (trace->max_splits > 0 && !trace->cut) || trace->max_regions < 0 ||
                trace->max_splits < 0))
    return CCUBA_EINVAL;
  CtxScope scope(ctxp);
  if (scope.rc) return scope.rc;
  ccuba_ctx *ctx = scope.ctx;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  SuaveResult res;
  SuaveTraceOut to;
  if (trace) {
    to.max_regions = trace->max_regions;
    to.max_splits = trace->max_splits;
    to.lo = trace->lo;
    to.hi = trace->hi;
    to.I = trace->I;
    to.var = trace->var;
    to.grid = trace->grid;
    to.cut = trace->cut;
  }
  int rc = run_suave(ctx, sp, res, trace ? &to : nullptr, ctx->stream);
  if (rc) return rc;
  *nregions = res.nregions;
  *neval = res.neval;
  *fail = res.fail;
  integral[0] = res.integral;
  error[0] = res.error;
  prob[0] = res.prob;
  if (trace) {
    trace->nregions = res.nregions;
    trace->nsplits = (int)res.nsplits;
    trace->chi2 = res.chi2;
    trace->dof = res.dof;
  }
  return CCUBA_OK;
}

int ccuba_divonne_partition(ccuba_ctx **ctxp, int ndim, const ccuba_integrand *f,
                            unsigned long long seed, unsigned int stream_id, int nsearch,
                            int niter, int maxregions, int nsplit, double spread_tol,
                            int *nregions, long long *neval, int *fail, double *total_spread,
                            ccuba_partition_trace *trace) {
  if (!f || !f->a || !f->u || !nregions || !neval || !fail || !total_spread || ndim < 1 ||
      ndim > kMaxDim)
    return CCUBA_EINVAL;
  PartitionSpec sp;
  sp.ndim = ndim;
  sp.family = f->family;
  for (int j = 0; j < ndim; ++j) {
    sp.a[j] = f->a[j];
    sp.u[j] = f->u[j];
  }
  sp.seed = seed;
  sp.sid = stream_id;
  sp.nsearch = nsearch;
  sp.niter = niter;
  sp.maxregions = maxregions;
  sp.nsplit = nsplit;
  sp.spread_tol = spread_tol;
  if (validate_partition(sp)) return CCUBA_EINVAL;
  if (trace && (trace->max_regions < 0 || trace->max_splits < 0 ||
                (trace->max_splits > 0 && !trace->cut)))
    return CCUBA_EINVAL;
  CtxScope scope(ctxp);
  if (scope.rc) return scope.rc;
  ccuba_ctx *ctx = scope.ctx;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  PartitionResult res;
  PartitionTraceOut to;
  if (trace) {
    to.max_regions = trace->max_regions;
    to.max_splits = trace->max_splits;
    to.lo = trace->lo;
    to.hi = trace->hi;
    to.xmin = trace->xmin;
    to.xmax = trace->xmax;
    to.fmin = trace->fmin;
    to.fmax = trace->fmax;
    to.spread = trace->spread;
    to.cut = trace->cut;
  }
  int rc = run_partition(ctx, sp, res, trace ? &to : nullptr, ctx->stream);
  if (rc) return rc;
  *nregions = res.nregions;
  *neval = res.neval;
  *fail = res.fail;
  *total_spread = res.total_spread;
  if (trace) {
    trace->nregions = res.nregions;
    trace->nsplits = (int)res.nsplits;
  }
  return CCUBA_OK;
}

int ccuba_cuhre_rule(ccuba_ctx *ctx, int ndim, const ccuba_integrand *f, long long nreg,
                     const double *c, const double *h, double *I7, double *I5, double *err,
                     int *axis) {
  if (!ctx || !f || !f->a || !f->u || ndim < 2 || ndim > kMaxDim || nreg < 0 || !c || !h)
    return CCUBA_EINVAL;
  if (nreg == 0) return CCUBA_OK;
  CuhreSpec sp;
  sp.ndim = ndim;
  sp.family = f->family;
  for (int j = 0; j < ndim; ++j) {
    sp.a[j] = f->a[j];
    sp.u[j] = f->u[j];
  }
  sp.maxeval = (nreg + 2) * gm_npoints(ndim) * 2;
  sp.batch = 2;
  if (validate_cuhre(sp)) return CCUBA_EINVAL;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  CuhreRun run(ctx);
  int rc = run.start(sp, ctx->stream);
  if (rc) return rc;
  return run.rule_only(nreg, c, h, I7, I5, err, axis, ctx->stream);
}

namespace {

// One engine over a batch's integrals, on the context's stream: the states
// after the last iteration into st.
int run_batch_engine(ccuba_ctx *ctx, const std::vector<VegasSpec> &specs,
                     std::vector<VState> &st) {
  VegasEngine eng(ctx);
  int rc;
  // one integral: the single-integral tile plan (a tile per block)
  if ((rc = eng.setup(specs, specs.size() == 1, ctx->stream))) return rc;
  if ((rc = eng.run(ctx->stream))) return rc;
  return eng.read_states(st, ctx->stream);
}

// A batch's two halves side by side, one on each of the context's streams.
// When every job runs its whole budget both are launched from this thread,
// their graphs captured first and then queued one right after the other, so
// that their first sampling launches start together; otherwise each runs
// from a thread of its own (its chunks wait on host checks of the states).
// With ref (profile mode) the halves' sampling intervals go to iv.
int run_halves(ccuba_ctx *ctx, const std::vector<VegasSpec> &h0,
               const std::vector<VegasSpec> &h1, std::vector<VState> &st0,
               std::vector<VState> &st1, hipEvent_t ref,
               std::vector<std::pair<double, double>> &iv) {
  VegasEngine e0(ctx), e1(ctx);
  int rc;
  if ((rc = e0.setup(h0, h0.size() == 1, ctx->stream))) return rc;
  if ((rc = e1.setup(h1, h1.size() == 1, ctx->stream2))) return rc;
  e0.set_time_reference(ref);
  e1.set_time_reference(ref);
  int r0 = CCUBA_OK, r1 = CCUBA_OK;
  if (e0.fixed() && e1.fixed()) {
    // both halves' graphs are captured before either is launched
    if ((rc = e0.prepare_run(ctx->stream)) || (rc = e1.prepare_run(ctx->stream2))) return rc;
    r0 = e0.launch_run(ctx->stream);
    if (!r0) r1 = e1.launch_run(ctx->stream2);
    // (what was queued is waited for, also after a failed launch)
    const int f0 = e0.finish_run(ctx->stream);
    const int f1 = r0 ? CCUBA_OK : e1.finish_run(ctx->stream2);
    if (!r0) r0 = f0;
    if (!r1) r1 = f1;
  } else {
    std::thread other;
    try {
      other = std::thread([&] {
        r1 = hipSetDevice(ctx->device) == hipSuccess ? e1.run(ctx->stream2) : CCUBA_EHIP;
      });
    } catch (...) {  // no thread: the halves run one after the other
    }
    r0 = e0.run(ctx->stream);
    if (other.joinable())
      other.join();
    else
      r1 = e1.run(ctx->stream2);
  }
  for (const VegasEngine *e : {&e0, &e1})
    iv.insert(iv.end(), e->dosample_intervals().begin(), e->dosample_intervals().end());
  if (r0) return r0;
  if (r1) return r1;
  if ((rc = e0.read_states(st0, ctx->stream))) return rc;
  return e1.read_states(st1, ctx->stream2);
}

// Length of the union of intervals.
double union_length(std::vector<std::pair<double, double>> iv) {
  std::sort(iv.begin(), iv.end());
  double total = 0.0, lo = 0.0, hi = 0.0;
  bool open = false;
  for (const auto &x : iv) {
    if (open && x.first <= hi) {
      hi = std::max(hi, x.second);
      continue;
    }
    if (open) total += hi - lo;
    lo = x.first;
    hi = x.second;
    open = true;
  }
  if (open) total += hi - lo;
  return total;
}

}  // namespace

int ccuba_vegas_batch(ccuba_ctx *ctx, int njobs, const ccuba_job jobs[], ccuba_result out[]) {
  if (!ctx || njobs < 0 || (njobs > 0 && (!jobs || !out))) return CCUBA_EINVAL;
  if (njobs == 0) return CCUBA_OK;
  std::lock_guard<std::mutex> g(ctx->lock);
  CCUBA_HIP(hipSetDevice(ctx->device));
  std::vector<VegasSpec> specs;
  std::vector<int> index(njobs, -1);
  const double t_submit = ctx->now();
  for (int q = 0; q < njobs; ++q) {
    const ccuba_job &jb = jobs[q];
    out[q] = ccuba_result{};
    out[q].t_submit = t_submit;
    VegasSpec sp;
    int rc = CCUBA_EINVAL;
    if (jb.method == 0)
      rc = fill_spec(sp, jb.ndim, 1, &jb.f, jb.epsrel, jb.epsabs, jb.flags, jb.seed,
                     jb.mineval, jb.maxeval, jb.nstart, jb.nincrease, 1,
                     jb.nbins > 0 ? jb.nbins : 128, jb.stream_id);
    out[q].status = rc;
    if (rc == CCUBA_OK) {
      index[q] = (int)specs.size();
      specs.push_back(sp);
    }
  }
  if (specs.empty()) return CCUBA_OK;
  // Two halves on two streams (Sect. 2.1 makes each integral's iterations a
  // sequence, and separate integrals independent): every iteration of a half
  // ends in its fold and refine launches, a few workgroups that wait on
  // memory, and the other half's sampling launch has the compute units
  // meanwhile.  The split balances the halves' evaluations; it is taken when
  // the setting of every precision in the batch asks for it (the autotuner
  // measures both ways).
  if (ctx->autotune) autotune_batch(ctx, specs);
  bool split = specs.size() >= 2;
  for (const auto &sp : specs) split = split && ctx->tune[sp.prec].streams > 1;
  const size_t cut = split ? batch_cut(specs) : specs.size();
  const std::vector<VegasSpec> half0(specs.begin(), specs.begin() + cut),
      half1(specs.begin() + cut, specs.end());
  std::vector<VState> st, st1;
  int rc = CCUBA_OK;
  if (!split) {
    rc = run_batch_engine(ctx, half0, st);
  } else {
    // In profile mode the halves' sampling launches are timed against one
    // reference event that both streams start after, and the context's busy
    // time gets the union of their intervals.
    hipEvent_t ref = nullptr;
    std::vector<std::pair<double, double>> iv;
    if (ctx->profile) {
      CCUBA_HIP(hipEventCreate(&ref));
      if (hipEventRecord(ref, ctx->stream) != hipSuccess ||
          hipStreamWaitEvent(ctx->stream2, ref, 0) != hipSuccess) {
        (void)hipEventDestroy(ref);
        return CCUBA_EHIP;
      }
    }
    rc = run_halves(ctx, half0, half1, st, st1, ref, iv);
    if (ref) {
      std::lock_guard<std::mutex> g(ctx->stats_lock);
      ctx->stats.dosample_busy_ms += union_length(iv);
      (void)hipEventDestroy(ref);
    }
  }
  if (rc) return rc;
  st.insert(st.end(), st1.begin(), st1.end());
  const double t_done = ctx->now();
  for (int q = 0; q < njobs; ++q) {
    if (index[q] < 0) continue;
    const VState &s = st[index[q]];
    out[q].neval = s.neval;
    out[q].fail = s.fail;
    out[q].integral = s.integral;
    out[q].error = s.error;
    out[q].prob = s.prob;
    out[q].t_done = t_done;
  }
  return CCUBA_OK;
}

int ccuba_submit(ccuba_ctx *ctx, const ccuba_job *job, unsigned long long *ticket) {
  if (!ctx || !job || !ticket) return CCUBA_EINVAL;
  {
    std::lock_guard<std::mutex> g(ctx->lock);
    if (!ctx->server) ctx->server = new (std::nothrow) Server(ctx);
    if (!ctx->server) return CCUBA_ENOMEM;
  }
  return ctx->server->submit(*job, ticket);
}

int ccuba_poll(ccuba_ctx *ctx, unsigned long long ticket, ccuba_result *out) {
  if (!ctx || !out) return CCUBA_EINVAL;
  if (!ctx->server) return CCUBA_ENOENT;
  return ctx->server->poll(ticket, out);
}

int ccuba_drain(ccuba_ctx *ctx) {
  if (!ctx) return CCUBA_EINVAL;
  if (!ctx->server) return CCUBA_OK;
  return ctx->server->drain();
}

}  // extern "C"
