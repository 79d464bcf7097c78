// noalloc.h -- the device scratch of the allocation-free DoSample entry point
// (ccuba_vegas_dosample_raw_noalloc).
#pragma once
#include <hip/hip_runtime.h>

#include "engine.h"

namespace ccuba {

// Size of the scratch array every device holds for the process's lifetime.
constexpr size_t kNoallocScratchBytes = (size_t)16 << 20;

// Records, once per device and with that device current, the device address
// of the scratch array.  Returns CCUBA_OK, CCUBA_EINVAL (device index beyond
// the table) or CCUBA_EHIP (the runtime could not give the address).
int noalloc_init(int device);
// The recorded address of the device's scratch array, or nullptr.
void *noalloc_scratch(int device);

// The descriptors of one DoSample pass, passed by value to a kernel that
// writes them into the scratch (kernel arguments need no host buffer that
// must outlive the call, nor a copy to wait for).
struct NoallocSetup {
  VJob job;
  VState st;
  double p64[2][kParamRow];
  float p32[2][kParamRow];
  long long ends[2];  // the fold tasks of the one job: level 1, level 2
  VJob *job_dst;
  VState *st_dst;
  double *p64_dst;
  float *p32_dst;
  long long *ends_dst;
};
hipError_t launch_noalloc_setup(const NoallocSetup &S, hipStream_t s);

}  // namespace ccuba
