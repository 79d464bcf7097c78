// tune.cpp -- launch-geometry autotuner of the DoSample kernel.
//
// The sweep times one DoSample pass (no refinement) of a fixed synthetic
// integral -- d = 8, oscillatory, 128 bins, 2^23 points -- for every
// candidate (block size, persistent blocks per CU, points per lane per trip,
// FP32 histogram precision)
// and keeps the fastest.  Results do not depend on the choice beyond
// floating-point summation order.  The cache file holds one line per
// (device name, precision): "name prec block blocks_per_cu hist64 ilp", and
// one per (device name, batch signature, precision) for batches:
// "name:batch:signature prec block blocks_per_cu hist64 ilp min_tile streams",
// where the signature hashes the shapes of the batch's jobs of that
// precision and streams is 2 when the batch runs as two halves.
#include "tune.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "vegas_engine.h"

namespace ccuba {

namespace {

std::string device_key(ccuba_ctx *ctx) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return "unknown";
  std::string s = prop.gcnArchName;
  s += "_cu" + std::to_string(prop.multiProcessorCount);
  for (char &c : s)
    if (c == ' ' || c == ':') c = '_';
  return s;
}

bool load_cache(const char *path, const std::string &key, int prec, VegasTune &t,
                bool with_tile = false) {
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {  // the last matching line wins
    std::istringstream is(line);
    std::string k;
    int p, b, bpc, h, ilp, ns = 2;
    long long mt = 0;
    if (!(is >> k >> p >> b >> bpc >> h >> ilp)) continue;
    if (with_tile && !(is >> mt)) continue;
    if (with_tile && !(is >> ns)) ns = 2;
    if (k == key && p == prec) {
      t.block = b;
      t.blocks_per_cu = bpc;
      t.hist64 = h;
      t.ilp = ilp;
      if (with_tile) {
        t.min_tile = mt;
        t.streams = ns == 1 ? 1 : 2;
      }
      found = true;
    }
  }
  return found;
}

void store_cache(const char *path, const std::string &key, int prec, const VegasTune &t,
                 bool with_tile = false) {
  std::ofstream f(path, std::ios::app);
  f << key << " " << prec << " " << t.block << " " << t.blocks_per_cu << " " << t.hist64 << " "
    << t.ilp;
  if (with_tile) f << " " << t.min_tile << " " << t.streams;
  f << "\n";
}

// FNV-1a over the shapes of a batch's jobs: what the launch settings depend on
std::string batch_signature(const std::vector<VegasSpec> &specs) {
  unsigned long long h = 1469598103934665603ull;
  auto mix = [&](long long v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (unsigned long long)((v >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  for (const VegasSpec &s : specs) {
    mix(s.ndim);
    mix(s.nbins);
    mix(s.family);
    mix(s.nstart);
    mix(s.nincrease);
    mix(s.maxeval);
  }
  char buf[32];
  std::snprintf(buf, sizeof(buf), "%016llx", h);
  return buf;
}

double time_candidate(ccuba_ctx *ctx, int prec, const VegasTune &cand) {
  const VegasTune saved = ctx->tune[prec];
  ctx->tune[prec] = cand;
  VegasSpec sp;
  sp.ndim = 8;
  sp.nbins = 128;
  sp.family = 1;
  sp.prec = prec;
  sp.nstart = 1 << 23;
  sp.maxeval = 1ll << 40;
  for (int j = 0; j < 8; ++j) {
    sp.a[j] = 9.0 / 8.0;
    sp.u[j] = 0.1 * j;
  }
  double best = 1e30;
  {
    VegasEngine eng(ctx);
    if (eng.setup({sp}, true, ctx->stream) == 0) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
        (void)eng.dosample_only(ctx->stream);  // warm-up
        for (int r = 0; r < 3; ++r) {
          (void)hipEventRecord(a, ctx->stream);
          (void)eng.dosample_only(ctx->stream);
          (void)hipEventRecord(b, ctx->stream);
          if (hipEventSynchronize(b) != hipSuccess) break;
          float ms = 0;
          (void)hipEventElapsedTime(&ms, a, b);
          if (ms < best) best = ms;
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    }
  }
  ctx->tune[prec] = saved;
  return best;
}

}  // namespace

void maybe_autotune(ccuba_ctx *ctx, int prec) {
  if (ctx->tuned[prec]) return;
  ctx->tuned[prec] = 1;
  const char *path = std::getenv("CCUBA_TUNE_CACHE");
  const std::string key = device_key(ctx);
  VegasTune t = ctx->tune[prec];
  if (path && *path && load_cache(path, key, prec, t)) {
    ctx->tune[prec] = t;
    return;
  }
  VegasTune best = ctx->tune[prec];
  double best_ms = 1e30;
  const int blocks[] = {128, 256};
  const int bpcs[] = {2, 3, 4, 5, 6, 8};
  for (int b : blocks)
    for (int bpc : bpcs)
      for (int ilp = 1; ilp <= 2; ++ilp)
      for (int h = 0; h < 2; ++h) {
        VegasTune c = ctx->tune[prec];
        c.block = b;
        c.blocks_per_cu = b == 128 ? 2 * bpc : bpc;
        c.ilp = ilp;
        c.hist64 = h;
        const double ms = time_candidate(ctx, prec, c);
        if (ms < best_ms) {
          best_ms = ms;
          best = c;
        }
      }
  ctx->tune[prec] = best;
  if (path && *path) store_cache(path, key, prec, best);
}

namespace {

// Full iterations (sampling, fold, refine) of specs as the batch call runs
// them: as one engine on the context's stream, or with split as two halves
// side by side on its two streams (each half with the single-integral tile
// plan if it holds one integral), replayed from graphs captured before
// either half is launched.  Each job runs its first iterations (6 of its
// budget, fewer down to 2 for batches of more than 3.3e7 points an
// iteration, so that a run samples at most ~2e8 points; no early stopping);
// the best of three such runs, from fresh engines, in ms, or of fewer once
// one takes longer than `cutoff' ms (the candidate is then out of the race
// anyway).
double time_batch(ccuba_ctx *ctx, const std::vector<VegasSpec> &specs, bool split,
                  double cutoff) {
  double per_iter = 0.0;
  for (const VegasSpec &sp : specs) per_iter += (double)sp.nstart;
  const int kIters = (int)std::max(2.0, std::min(6.0, 2e8 / std::max(per_iter, 1.0)));
  std::vector<VegasSpec> cut_specs = specs;
  for (VegasSpec &sp : cut_specs) {
    long long budget = 0;
    for (int t = 0; t < kIters; ++t) budget += sp.nstart + (long long)t * sp.nincrease;
    sp.maxeval = std::min(sp.maxeval, budget);
    sp.mineval = 0;
    sp.epsrel = sp.epsabs = 0.0;
  }
  const size_t cut = split ? batch_cut(cut_specs) : cut_specs.size();
  const std::vector<VegasSpec> h0(cut_specs.begin(), cut_specs.begin() + cut),
      h1(cut_specs.begin() + cut, cut_specs.end());
  hipEvent_t a, b, j;
  double best = 1e30;
  if (hipEventCreate(&a) != hipSuccess) return best;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return best;
  }
  if (hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
  }
  for (int r = 0; r < 3; ++r) {
    VegasEngine e0(ctx), e1(ctx);
    bool ok = e0.setup(h0, h0.size() == 1, ctx->stream) == CCUBA_OK &&
              (h1.empty() || e1.setup(h1, h1.size() == 1, ctx->stream2) == CCUBA_OK) &&
              e0.prepare_run(ctx->stream) == CCUBA_OK &&
              (h1.empty() || e1.prepare_run(ctx->stream2) == CCUBA_OK);
    ok = ok && hipEventRecord(a, ctx->stream) == hipSuccess;
    if (!h1.empty()) ok = ok && hipStreamWaitEvent(ctx->stream2, a, 0) == hipSuccess;
    ok = ok && e0.launch_run(ctx->stream) == CCUBA_OK;
    if (!h1.empty())
      ok = ok && e1.launch_run(ctx->stream2) == CCUBA_OK &&
           hipEventRecord(j, ctx->stream2) == hipSuccess &&
           hipStreamWaitEvent(ctx->stream, j, 0) == hipSuccess;
    ok = ok && hipEventRecord(b, ctx->stream) == hipSuccess;
    const bool done = ok && hipEventSynchronize(b) == hipSuccess;
    (void)e0.finish_run(ctx->stream);
    if (!h1.empty()) (void)e1.finish_run(ctx->stream2);
    if (!done) break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    if (ms < best) best = ms;
    if (ms > cutoff) break;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipEventDestroy(j);
  return best;
}

}  // namespace

void autotune_batch(ccuba_ctx *ctx, const std::vector<VegasSpec> &specs) {
  for (int prec = 0; prec < 2; ++prec) {
    if (ctx->tuned_batch[prec]) continue;
    std::vector<VegasSpec> mine;
    for (const auto &sp : specs)
      if (sp.prec == prec) mine.push_back(sp);
    if (mine.empty()) continue;
    ctx->tuned_batch[prec] = 1;
    const char *path = std::getenv("CCUBA_TUNE_CACHE");
    const std::string key = device_key(ctx) + ":batch:" + batch_signature(mine);
    VegasTune cached = ctx->tune[prec];
    if (path && *path && load_cache(path, key, prec, cached, true)) {
      ctx->tune[prec] = cached;
      continue;
    }
    const VegasTune saved = ctx->tune[prec];
    VegasTune best = saved;
    double best_ms = 1e30;
    const int profile = ctx->profile;  // (the tuning runs are not profiled)
    ctx->profile = 0;
    const int bpcs[] = {2, 3, 4, 6};
    const long long tiles[] = {4096, 16384, 65536};
    // one engine, or two halves (2+ integrals); a tile plan that holds one
    // integral is the single-integral one, which does not use the minimum
    // tile size
    for (int streams = 1; streams <= (mine.size() >= 2 ? 2 : 1); ++streams) {
      const bool split = streams == 2;
      const size_t cut = split ? batch_cut(mine) : mine.size();
      const bool single = split ? (cut == 1 && mine.size() == 2) : mine.size() == 1;
      const int ntiles = single ? 1 : 3;
      for (int bpc : bpcs)
        for (int ilp = 1; ilp <= 2; ++ilp)
          for (int ti = 0; ti < ntiles; ++ti)
            for (int h = 0; h < 2; ++h) {
              VegasTune c = saved;
              c.blocks_per_cu = bpc;
              c.ilp = ilp;
              c.min_tile = single ? saved.min_tile : tiles[ti];
              c.hist64 = h;
              c.streams = streams;
              ctx->tune[prec] = c;
              // (a candidate 25% slower than the best so far stops after one run)
              const double ms = time_batch(ctx, mine, split, 1.25 * best_ms);
              if (ms < best_ms) {
                best_ms = ms;
                best = c;
              }
            }
    }
    ctx->profile = profile;
    ctx->tune[prec] = best;
    if (path && *path) store_cache(path, key, prec, best, true);
  }
}

}  // namespace ccuba
