// Host side of the streaming projection (steps 4-7 with Y in HBM): workspace,
// the pass loop and the result.  Kernels: project_stream.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "fastpfp_ctx.h"
#include "project_stream_internal.h"

extern "C" void fpfp_stream_geometry(long long N, int* TR, int* TC, int* nrb);
extern "C" hipError_t fpfp_stream_step(const fpfp::StreamState* st, int mode,
                                       int first, double tol,
                                       hipStream_t stream);

using fpfp::fail;

namespace {
size_t align256(size_t x) { return (x + 255) / 256 * 256; }
}  // namespace

extern "C" fastpfp_status fastpfp_project_stream(fastpfp_t h, int N, float* Y,
                                                 double tol, int max_inner,
                                                 int projection,
                                                 fastpfp_info* info) {
  if (!h) return FASTPFP_ERR_INVALID_ARG;
  if (N < 1 || N > std::max(h->max_n, h->max_np))
    return fail(h, FASTPFP_ERR_SHAPE, "N=%d out of range", N);
  if (!Y) return fail(h, FASTPFP_ERR_INVALID_ARG, "Y is NULL");
  if (!(tol > 0.0) || !std::isfinite(tol) || max_inner < 1)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "bad tolerance or cap");
  if (projection != FASTPFP_PROJ_ALTERNATING &&
      projection != FASTPFP_PROJ_DYKSTRA)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "unknown projection %d",
                projection);
  HIPCHK(h, hipSetDevice(h->device));
  int TR = 0, TC = 0, nrb_i = 0;
  fpfp_stream_geometry(N, &TR, &TC, &nrb_i);
  const size_t nt = (size_t)TR * TC;
  size_t off = 0;
  const size_t o_a = off;  off = align256(off + sizeof(double) * N);
  const size_t o_b = off;  off = align256(off + sizeof(float) * N);
  const size_t o_rp = off; off = align256(off + sizeof(float) * N * (size_t)TC);
  const size_t o_cp = off; off = align256(off + sizeof(float) * N * (size_t)TR);
  const size_t nrb = (size_t)nrb_i;  // reduce blocks
  const size_t o_tm = off; off = align256(off + sizeof(float) * nt);
  const size_t o_sp = off; off = align256(off + sizeof(double) * nrb);
  const size_t o_mp = off; off = align256(off + sizeof(float) * nrb);
  const size_t o_sc = off; off = align256(off + sizeof(double) * 2);
  const size_t o_ct = off; off = align256(off + sizeof(unsigned) * 2);
  const size_t need = off;
  if (need > h->pws_bytes) {
    if (h->pws) (void)hipFree(h->pws);
    h->pws = nullptr;
    h->pws_bytes = 0;
    if (hipMalloc(&h->pws, need) != hipSuccess) {
      h->pws = nullptr;
      return fail(h, FASTPFP_ERR_NOMEM, "cannot allocate %zu bytes", need);
    }
    h->pws_bytes = need;
  }
  char* base = (char*)h->pws;
  fpfp::StreamState st;
  st.Y = Y;
  st.N = N;
  st.a = (double*)(base + o_a);
  st.b = (float*)(base + o_b);
  st.rowpart = (float*)(base + o_rp);
  st.colpart = (float*)(base + o_cp);
  st.tmax = (float*)(base + o_tm);
  st.spart = (double*)(base + o_sp);
  st.mpart = (float*)(base + o_mp);
  st.scal = (double*)(base + o_sc);
  unsigned* cw = (unsigned*)(base + o_ct);
  st.ctl = cw;
  st.counters = cw + 1;
  const bool dyk = projection == FASTPFP_PROJ_DYKSTRA;
  HIPCHK(h, hipMemsetAsync(base + o_sc, 0, sizeof(double) * 2, h->stream));
  HIPCHK(h, hipMemsetAsync(cw, 0, sizeof(unsigned) * 2, h->stream));
  HIPCHK(h, hipEventRecord(h->ev0, h->stream));
  HIPCHK(h, fpfp_stream_step(&st, 0, 0, tol, h->stream));
  // passes go out in chunks; once the stop test holds (or values turn
  // non-finite) the remaining launches of the chunk return at once
  const int chunk = 32;
  unsigned ctl = 0;
  for (int done = 0; done < max_inner;) {
    const int k = std::min(chunk, max_inner - done);
    for (int j = 0; j < k; ++j)
      HIPCHK(h, fpfp_stream_step(&st, dyk ? 2 : 1, done + j == 0 ? 1 : 0, tol,
                                 h->stream));
    done += k;
    HIPCHK(h, hipMemcpyAsync(&ctl, cw, sizeof ctl, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (ctl != 0) break;
  }
  if (dyk) HIPCHK(h, fpfp_stream_step(&st, 3, 0, tol, h->stream));
  HIPCHK(h, hipEventRecord(h->ev1, h->stream));
  unsigned cnt[2] = {0, 0};
  double sc[2] = {0.0, 0.0};
  HIPCHK(h, hipMemcpyAsync(cnt, cw, sizeof cnt, hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipMemcpyAsync(sc, st.scal, sizeof sc, hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  float ms = 0.f;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
  if (info) {
    std::memset(info, 0, sizeof *info);
    info->outer_iters = 0;
    info->inner_iters_total = (int)cnt[1];
    info->inner_iters_max = (int)cnt[1];
    info->inner_capped = (cnt[0] == 0 && (int)cnt[1] >= max_inner) ? 1 : 0;
    info->converged = cnt[0] == 1 ? 1 : 0;
    info->eps2_last = sc[1];
    info->kernel_ms = ms;
    info->proj_ms = ms;
    info->pair_ms = ms;
    info->status = cnt[0] == 2 ? FASTPFP_ERR_NUMERIC : FASTPFP_OK;
  }
  if (cnt[0] == 2)
    return fail(h, FASTPFP_ERR_NUMERIC, "non-finite values in the projection");
  return FASTPFP_OK;
}
