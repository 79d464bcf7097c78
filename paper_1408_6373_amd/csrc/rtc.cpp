// rtc.cpp -- the DoSample kernel for a caller's device integrand, compiled at
// run time with hiprtc.
//
// The paper's integrand is a user function (Sect. 3.2.2).  On the GPU path it
// has to be device code inside DoSample, so the library compiles the DoSample
// kernel again at run time with the caller's function in it: the kernel's own
// headers (their text is in the library) with CCUBA_RTC defined, which keeps
// their host-only parts out and makes the per-point loop collect x and call
// ccuba_user(x, ndim, a, u).  The result is one kernel instance of the class
// the integral needs, launched by the engine like the built-in ones.
#include "rtc.h"

#include <hip/hiprtc.h>

#include <cstdio>
#include <vector>

#include "engine.h"

namespace ccuba {

extern const int kRtcHeaderCount;
extern const char *const kRtcHeaderNames[];
extern const char *const kRtcHeaderTexts[];

namespace {

std::string arch_of(ccuba_ctx *ctx) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return "gfx950";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

}  // namespace

int rtc_dosample(ccuba_ctx *ctx, const char *source, int prec, int hist64, int ilp, int nb,
                 bool pow2, bool full, hipFunction_t *out) {
  if (!ctx->rtc) ctx->rtc = new RtcCache;
  RtcCache &cache = *ctx->rtc;
  const char *T = prec == FP64 ? "double" : "float";
  const char *HT = hist64 ? "double" : "unsigned long long";
  char inst[256];
  std::snprintf(inst, sizeof(inst), "ccuba::vegas_dosample_kernel<%s, %s, %d, %d, %s, %s>", T,
                HT, ilp, nb, pow2 ? "true" : "false", full ? "true" : "false");
  const std::string arch = arch_of(ctx);
  const std::string key = arch + "|" + inst + "|" + source;
  auto it = cache.mods.find(key);
  if (it != cache.mods.end()) {
    *out = it->second.second;
    return CCUBA_OK;
  }
  // the program: integer types hiprtc keeps in its own namespace, the
  // caller's function, the kernel headers, one explicit instance
  std::string src =
      "#define CCUBA_RTC 1\n"
      "typedef __hip_internal::uint32_t uint32_t;\n"
      "typedef __hip_internal::uint64_t uint64_t;\n"
      "typedef __hip_internal::int32_t int32_t;\n"
      "typedef __hip_internal::int64_t int64_t;\n";
  src += source;
  src += "\n#include \"vegas_sample.h\"\ntemplate __global__ void ";
  src += inst;
  src += "(ccuba::VegasArgs);\n";
  hiprtcProgram p;
  if (hiprtcCreateProgram(&p, src.c_str(), "ccuba_user.hip", kRtcHeaderCount, kRtcHeaderTexts,
                          kRtcHeaderNames) != HIPRTC_SUCCESS)
    return CCUBA_EHIP;
  hiprtcAddNameExpression(p, inst);
  const std::string archopt = "--offload-arch=" + arch;
  // the library's own flags: no FP contraction, no packed FP32 instructions
  const char *opts[] = {archopt.c_str(), "-O3", "-std=c++17", "-ffp-contract=off",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult cr = hiprtcCompileProgram(p, 8, opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(p, &ls);
  cache.log.assign(ls, '\0');
  if (ls) hiprtcGetProgramLog(p, &cache.log[0]);
  while (!cache.log.empty() && cache.log.back() == '\0') cache.log.pop_back();
  if (cr != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&p);
    return CCUBA_EINVAL;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(p, &cs);
  std::vector<char> code(cs);
  hiprtcGetCode(p, code.data());
  const char *lowered = nullptr;
  std::string name;
  if (hiprtcGetLoweredName(p, inst, &lowered) == HIPRTC_SUCCESS && lowered) name = lowered;
  hiprtcDestroyProgram(&p);
  if (name.empty()) return CCUBA_EHIP;
  hipModule_t mod;
  hipFunction_t fn;
  CCUBA_HIP(hipModuleLoadData(&mod, code.data()));
  if (hipModuleGetFunction(&fn, mod, name.c_str()) != hipSuccess) {
    (void)hipModuleUnload(mod);
    return CCUBA_EHIP;
  }
  cache.mods[key] = {mod, fn};
  *out = fn;
  return CCUBA_OK;
}

void rtc_release(ccuba_ctx *ctx) {
  if (!ctx->rtc) return;
  for (auto &m : ctx->rtc->mods) (void)hipModuleUnload(m.second.first);
  delete ctx->rtc;
  ctx->rtc = nullptr;
}

}  // namespace ccuba
