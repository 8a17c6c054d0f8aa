// Host side of the device greedy discretisation (Sec. 4.5): validation,
// batch layout, scratch and launch.  The kernels are in
// discretize_device.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "discretize_internal.h"
#include "fastpfp_ctx.h"

extern "C" hipError_t fpfp_greedy_launch(const fpfp::GreedyPair* P_dev,
                                         int batch, long long total_rows,
                                         long long total_cols,
                                         hipStream_t stream);

using fpfp::fail;

extern "C" fastpfp_status fastpfp_discretize_greedy_batched(
    fastpfp_t h, int batch, const int* n_host, const int* np_host,
    const float* X, const int64_t* offX_host, int32_t* match,
    const int64_t* offM_host, int* status_host) {
  if (!h) return FASTPFP_ERR_INVALID_ARG;
  if (batch < 1 || !n_host || !np_host || !X || !offX_host || !match ||
      !offM_host)
    return fail(h, FASTPFP_ERR_INVALID_ARG,
                "batch >= 1 and non-NULL sizes, offsets and buffers needed");
  long long rows = 0, cols = 0;
  for (int b = 0; b < batch; ++b) {
    const int n = n_host[b], np = np_host[b];
    if (n < 1 || np < 1 || n > h->max_n || np > h->max_np)
      return fail(h, FASTPFP_ERR_SHAPE,
                  "pair %d: n=%d n'=%d outside [1, %d] x [1, %d]", b, n, np,
                  h->max_n, h->max_np);
    if ((unsigned long long)n * (unsigned long long)np >= 0xFFFFFFFFull)
      return fail(h, FASTPFP_ERR_UNSUPPORTED, "pair %d: n n' too large", b);
    if (offX_host[b] < 0 || offM_host[b] < 0)
      return fail(h, FASTPFP_ERR_INVALID_ARG, "pair %d: negative offset", b);
    rows += n;
    cols += np;
  }
  HIPCHK(h, hipSetDevice(h->device));
  // scratch: descriptors | suitor keys | flags (2 per pair)
  const size_t desc_bytes = sizeof(fpfp::GreedyPair) * batch;
  const size_t off_suitor = (desc_bytes + 255) / 256 * 256;
  const size_t off_flags = off_suitor + sizeof(uint64_t) * cols;
  const size_t need = off_flags + sizeof(unsigned) * 2 * batch;
  if (need > h->dws_bytes) {
    if (h->dws) (void)hipFree(h->dws);
    h->dws = nullptr;
    h->dws_bytes = 0;
    if (hipMalloc(&h->dws, need) != hipSuccess) {
      h->dws = nullptr;
      return fail(h, FASTPFP_ERR_NOMEM, "cannot allocate %zu bytes", need);
    }
    h->dws_bytes = need;
  }
  char* base = (char*)h->dws;
  uint64_t* suitor = (uint64_t*)(base + off_suitor);
  unsigned* flags = (unsigned*)(base + off_flags);
  std::vector<fpfp::GreedyPair> P(batch);
  long long r0 = 0, c0 = 0;
  for (int b = 0; b < batch; ++b) {
    fpfp::GreedyPair& d = P[b];
    d.X = X + offX_host[b];
    d.ldx = np_host[b];
    d.n = n_host[b];
    d.np = np_host[b];
    d.match = match + offM_host[b];
    d.suitor = suitor + c0;
    d.flags = flags + 2 * b;
    d.row_begin = r0;
    d.col_begin = c0;
    r0 += d.n;
    c0 += d.np;
  }
  HIPCHK(h, hipMemcpyAsync(base, P.data(), desc_bytes, hipMemcpyHostToDevice,
                           h->stream));
  HIPCHK(h, fpfp_greedy_launch((const fpfp::GreedyPair*)base, batch, rows, cols,
                               h->stream));
  std::vector<unsigned> fl(2 * batch);
  HIPCHK(h, hipMemcpyAsync(fl.data(), flags, sizeof(unsigned) * 2 * batch,
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  fastpfp_status st = FASTPFP_OK;
  for (int b = 0; b < batch; ++b) {
    int s = FASTPFP_OK;
    if (fl[2 * b + 1]) s = FASTPFP_ERR_TIMEOUT;
    else if (fl[2 * b]) s = FASTPFP_ERR_NUMERIC;
    if (status_host) status_host[b] = s;
    if (s != FASTPFP_OK && st == FASTPFP_OK) {
      st = (fastpfp_status)s;
      fail(h, st, s == FASTPFP_ERR_NUMERIC
                      ? "pair %d: X has a non-finite entry"
                      : "pair %d: proposal cap reached", b);
    }
  }
  return st;
}
