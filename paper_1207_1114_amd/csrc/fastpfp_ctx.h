// The handle behind fastpfp_t and the error helpers shared by the host-side
// sources of the library.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "fastpfp.h"

struct fastpfp_ctx;
namespace fpfp {
struct WarmState;                  // learned warm start (warmstart_api.cpp)
void warm_free(WarmState* w);      // releases its device memory
void warm_prepare(fastpfp_ctx* h); // creates its streams (best effort)
}  // namespace fpfp

struct fastpfp_ctx {
  int device = 0;
  int max_n = 0, max_np = 0;
  hipStream_t stream = nullptr;
  std::string err;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int cu_count = 0;
  double wall_khz = 100000.0;  // device wall clock (s_memrealtime) rate
  int occupancy = 0;
  int die_exchange = 1;        // 0: every team exchanges at device scope
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<double> trace;
  fpfp::WarmState* warm = nullptr;
  void* dws = nullptr;        // device greedy discretisation scratch
  size_t dws_bytes = 0;
  void* pws = nullptr;        // streaming projection scratch
  size_t pws_bytes = 0;
};

namespace fpfp {

// Records a formatted message on the handle and returns the status.
inline fastpfp_status fail(fastpfp_t h, fastpfp_status s, const char* fmt,
                           ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h->err = buf;
  }
  return s;
}

}  // namespace fpfp

#define HIPCHK(h, call)                                                     \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return ::fpfp::fail((h), FASTPFP_ERR_HIP, "%s failed: %s", #call,     \
                          hipGetErrorString(e_));                           \
  } while (0)
