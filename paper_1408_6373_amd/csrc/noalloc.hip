// noalloc.hip -- the device scratch of the allocation-free DoSample entry
// point: a fixed array in device memory that the library's code object
// brings with it, so that a DoSample pass can run without any allocation.
#include "noalloc.h"

#include <mutex>

#include "ccuba.h"

namespace ccuba {

// Every call on a device shares this array (and finds it as the last call
// left it).  In host code its name is only a stand-in: host code uses the
// address noalloc_init records.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_ptr[kMaxDevices];
}  // namespace

int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return CCUBA_EINVAL;
  std::lock_guard<std::mutex> g(g_lock);
  if (g_ptr[device]) return CCUBA_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return CCUBA_EHIP;
  }
  g_ptr[device] = p;
  return CCUBA_OK;
}

void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_lock);
  return g_ptr[device];
}

namespace {

// nbytes (a multiple of 4) from the kernel's arguments to device memory
__device__ void copy_words(void *dst, const void *src, int nbytes, int tid) {
  const uint32_t *s = (const uint32_t *)src;
  uint32_t *d = (uint32_t *)dst;
  for (int w = tid; w < nbytes / 4; w += blockDim.x) d[w] = s[w];
}

__global__ void __launch_bounds__(256) noalloc_setup_kernel(NoallocSetup S) {
  const int tid = threadIdx.x;
  static_assert(sizeof(VJob) % 4 == 0 && sizeof(VState) % 4 == 0, "whole words");
  copy_words(S.job_dst, &S.job, (int)sizeof(VJob), tid);
  copy_words(S.st_dst, &S.st, (int)sizeof(VState), tid);
  copy_words(S.p64_dst, S.p64, (int)sizeof(S.p64), tid);
  copy_words(S.p32_dst, S.p32, (int)sizeof(S.p32), tid);
  if (tid < 2) S.ends_dst[tid] = S.ends[tid];
}

}  // namespace

hipError_t launch_noalloc_setup(const NoallocSetup &S, hipStream_t s) {
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(256), 0, s, S);
  return hipGetLastError();
}

}  // namespace ccuba
