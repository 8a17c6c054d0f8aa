// Fixed device scratch for fastpfp_solve_noalloc: a file-scope device array
// that stands in for the handle's workspace, so that a solve allocates
// nothing.  Each GPU the library runs on holds its own copy of the array
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for that device (the array's name is a host-side
// stand-in, not a device address).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "fastpfp.h"
#include "fastpfp_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[FASTPFP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Writes the pair descriptor and clears `words` 32-bit words at `zero` (the
// launch's queue, per-pair results and exchange words, which must start at
// zero).  A kernel rather than hipMemsetAsync, so that the call can also be
// recorded into a graph.
__global__ void noalloc_prepare(fpfp::PairDesc d, fpfp::PairDesc* dst,
                                uint32_t* zero, long long words) {
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) *dst = d;
  for (long long i = i0; i < words; i += (long long)gridDim.x * blockDim.x)
    zero[i] = 0u;
}

}  // namespace

// Device address and size of `device`'s scratch array.  The address is
// looked up once per device, with that device current, and kept.
extern "C" hipError_t fpfp_noalloc_scratch(int device, void** ptr,
                                           size_t* bytes) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  *bytes = (size_t)FASTPFP_NOALLOC_SCRATCH_BYTES;
  return hipSuccess;
}

// Enqueues noalloc_prepare on `stream`: *dst = *d, and `bytes` bytes at
// `zero` (a multiple of 4) set to zero.
extern "C" hipError_t fpfp_noalloc_prepare(const fpfp::PairDesc* d,
                                           void* dst, void* zero, size_t bytes,
                                           hipStream_t stream) {
  const long long words = (long long)(bytes / 4);
  const int threads = 256;
  long long blocks = (words + threads - 1) / threads;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(noalloc_prepare, dim3((unsigned)blocks), dim3(threads), 0,
                     stream, *d, (fpfp::PairDesc*)dst, (uint32_t*)zero, words);
  return hipGetLastError();
}
