// context.h -- the library context (the analog of the paper's `spin'
// handle, Sect. 3.2.3) and the device-memory accounting every engine uses.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <utility>

#include "ccuba.h"
#include "engine.h"

namespace ccuba {
class Server;
class VegasEngine;
struct RtcCache;
}

struct ccuba_ctx {
  int device = 0;
  int ncu = 256;
  size_t budget = 0;                // bytes the context may hold on the device
  std::atomic<size_t> used{0};      // bytes currently held
  hipStream_t stream = nullptr;     // the context's own stream (default priority)
  // a second stream (default priority) for the second half of a Vegas batch
  hipStream_t stream2 = nullptr;
  ccuba::VegasTune tune[2];         // per precision: [FP64], [FP32]
  int use_graph = 1;
  int autotune = 0;
  int tuned[2] = {0, 0};
  int tuned_batch[2] = {0, 0};
  int serve_slots = 256;
  int profile = 0;
  ccuba_stats stats{};
  std::mutex stats_lock;            // guards stats (a batch's halves run in two threads)
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  std::mutex lock;                  // serialises engine use with the server thread
  ccuba::Server *server = nullptr;  // the serving loop, started by the first submit
  // the engine of the last single-integral Vegas call, kept (with its device
  // buffers and captured graphs) for the next call of the same shape
  ccuba::VegasEngine *vcache = nullptr;
  int engine_cache = 1;
  // DoSample kernels compiled at run time for callers' device integrands
  ccuba::RtcCache *rtc = nullptr;
  // a small mapped pinned host block (host and device addresses) that the
  // step-wise integrators' totals kernels write into, so that the host reads
  // a step's totals after a stream synchronisation without a copy; calls on
  // one context are serialised by `lock', so one block serves them all
  double *pinned_host = nullptr, *pinned_dev = nullptr;
  static constexpr size_t kPinnedBytes = 256;
  // Vegas grids kept between calls (gridno): slot -> ((ndim, nbins), edges)
  std::map<int, std::pair<std::pair<int, int>, std::vector<double>>> grid_table;
  // freed device blocks kept for reuse, by size class (see dev_alloc)
  std::mutex pool_lock;
  std::multimap<size_t, void *> pool;
  size_t pooled = 0;  // bytes held in the pool (not in `used')
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace ccuba {

// Device allocation charged to a context's budget.  Returns CCUBA_OK,
// CCUBA_ENOMEM (budget) or CCUBA_EHIP.  Blocks come from and return to a
// per-context pool of size classes, so that repeated calls and the serving
// loop do not pay for hipMalloc/hipFree.
int dev_alloc(ccuba_ctx *ctx, void **p, size_t bytes);
void dev_free(ccuba_ctx *ctx, void *p, size_t bytes);
// Return every pooled block to the device.
void pool_release(ccuba_ctx *ctx);
// The context's mapped pinned block (allocated on first use).  Returns
// CCUBA_OK or CCUBA_EHIP.
int pinned_block(ccuba_ctx *ctx, double **host, double **dev);

// A typed device buffer that returns its bytes to the context on release.
template <typename T>
struct DevBuf {
  ccuba_ctx *ctx = nullptr;
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  int alloc(ccuba_ctx *c, size_t count) {
    release();
    ctx = c;
    if (count == 0) count = 1;
    void *q = nullptr;
    const int rc = dev_alloc(c, &q, count * sizeof(T));
    if (rc != 0) return rc;
    p = (T *)q;
    n = count;
    return 0;
  }
  // keep the current buffer if it is this context's and large enough
  int reserve(ccuba_ctx *c, size_t count) {
    if (p && ctx == c && n >= (count ? count : 1)) return 0;
    return alloc(c, count);
  }
  void release() {
    if (p) dev_free(ctx, p, n * sizeof(T));
    p = nullptr;
    n = 0;
  }
  void swap(DevBuf &o) {
    std::swap(ctx, o.ctx);
    std::swap(p, o.p);
    std::swap(n, o.n);
  }
};

}  // namespace ccuba

namespace ccuba {
// With CCUBA_DEBUG set in the environment, a failed HIP call is reported on
// stderr (its error and source line) before CCUBA_EHIP is returned.
void note_hip_error(hipError_t e, const char *file, int line);
}  // namespace ccuba
#define CCUBA_HIP(call)                                 \
  do {                                                  \
    const hipError_t ccuba_e_ = (call);                 \
    if (ccuba_e_ != hipSuccess) {                       \
      ccuba::note_hip_error(ccuba_e_, __FILE__, __LINE__); \
      return CCUBA_EHIP;                                \
    }                                                   \
  } while (0)
