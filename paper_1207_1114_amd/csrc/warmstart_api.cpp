// Host side of the learned warm start: parameter storage, validation, and the
// sequence of kernel launches (warmstart.hip) for the forward pass that
// writes X0 and for the backward pass and Adam step that train it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fastpfp.h"
#include "fastpfp_ctx.h"
#include "warmstart_internal.h"

static_assert(fpws::kNumParams == FASTPFP_WS_NPARAMS,
              "parameter count of the ABI and the kernels differ");

namespace fpfp {

// Activations of one graph of a pair; rows = nodes.
struct Side {
  float* deg;     // [cap]
  double* wdeg;   // [cap]
  double* means;  // [2]
  float *x, *h1, *h2, *e;   // [cap x kDin], [cap x kH] x2, [cap x kDout]
  float *dE, *d2, *d1;      // gradients of e, h2 (pre-activation), h1
};

struct WarmState {
  // params | grad | adam m | adam v, each kNumParams floats
  float* pbuf = nullptr;
  bool loaded = false;
  int adam_t = 0;
  // node buffers of both sides
  void* nbuf = nullptr;
  int node_cap = 0;
  Side side[2];
  // pair buffers: S (then dS), Q, lse, target sums, loss partials, loss, flag
  void* qbuf = nullptr;
  long long pair_cap = 0;
  int axis_cap = 0;
  float *S = nullptr, *Q = nullptr, *lse = nullptr;
  double *tsum = nullptr, *partial = nullptr, *loss = nullptr;
  int* bad = nullptr;
  int* bads = nullptr;  // one flag per pair of a batched call
  int bads_cap = 0;
  // a batched call runs its pairs' forward passes on kLanes streams at once
  // (each pass is a dozen small launches): a stream, an event and the node
  // buffers of both sides per lane
  static constexpr int kLanes = 4;
  hipStream_t lane_s[kLanes] = {};
  hipEvent_t lane_ev[kLanes] = {};
  hipEvent_t start_ev = nullptr;
  void* lbuf = nullptr;
  int lane_cap = 0;
  Side lside[kLanes][2];

  float* params() { return pbuf; }
  float* grad() { return pbuf + fpws::kNumParams; }
  float* adam_m() { return pbuf + 2 * fpws::kNumParams; }
  float* adam_v() { return pbuf + 3 * fpws::kNumParams; }
};

void warm_free(WarmState* w) {
  if (!w) return;
  if (w->pbuf) (void)hipFree(w->pbuf);
  if (w->nbuf) (void)hipFree(w->nbuf);
  if (w->qbuf) (void)hipFree(w->qbuf);
  if (w->bads) (void)hipFree(w->bads);
  if (w->lbuf) (void)hipFree(w->lbuf);
  for (int l = 0; l < WarmState::kLanes; ++l) {
    if (w->lane_s[l]) (void)hipStreamDestroy(w->lane_s[l]);
    if (w->lane_ev[l]) (void)hipEventDestroy(w->lane_ev[l]);
  }
  if (w->start_ev) (void)hipEventDestroy(w->start_ev);
  delete w;
}

void warm_prepare(fastpfp_ctx* h) {
  if (!h->warm) h->warm = new WarmState;
  WarmState* w = h->warm;
  // failures are left for ensure_lanes to report when the lanes are used
  if (!w->start_ev &&
      hipEventCreateWithFlags(&w->start_ev, hipEventDisableTiming) !=
          hipSuccess)
    w->start_ev = nullptr;
  for (int l = 0; l < WarmState::kLanes; ++l) {
    if (!w->lane_s[l] &&
        hipStreamCreateWithFlags(&w->lane_s[l], hipStreamNonBlocking) !=
            hipSuccess)
      w->lane_s[l] = nullptr;
    if (!w->lane_ev[l] &&
        hipEventCreateWithFlags(&w->lane_ev[l], hipEventDisableTiming) !=
            hipSuccess)
      w->lane_ev[l] = nullptr;
  }
}

}  // namespace fpfp

namespace {

using fpfp::fail;
using fpfp::Side;
using fpfp::WarmState;
using fpws::GemmArgs;

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

WarmState* state(fastpfp_t h) {
  if (!h->warm) h->warm = new WarmState;
  return h->warm;
}

// Bytes of one side's node buffers for `c` rows.
size_t side_bytes(size_t c) {
  return up256(c * sizeof(float)) + up256(c * sizeof(double)) + 256 +
         up256(c * sizeof(float) * fpws::kDin) +
         2 * up256(c * sizeof(float) * fpws::kH) +
         up256(c * sizeof(float) * fpws::kDout) +
         up256(c * sizeof(float) * fpws::kDout) +
         2 * up256(c * sizeof(float) * fpws::kH);
}

// Carves one side's buffers for `c` rows out of p.
char* carve_side(char* p, size_t c, Side& d) {
  auto take = [&](size_t bytes) {
    char* r = p;
    p += up256(bytes);
    return r;
  };
  d.deg = (float*)take(c * sizeof(float));
  d.wdeg = (double*)take(c * sizeof(double));
  d.means = (double*)take(2 * sizeof(double));
  d.x = (float*)take(c * sizeof(float) * fpws::kDin);
  d.h1 = (float*)take(c * sizeof(float) * fpws::kH);
  d.h2 = (float*)take(c * sizeof(float) * fpws::kH);
  d.e = (float*)take(c * sizeof(float) * fpws::kDout);
  d.dE = (float*)take(c * sizeof(float) * fpws::kDout);
  d.d2 = (float*)take(c * sizeof(float) * fpws::kH);
  d.d1 = (float*)take(c * sizeof(float) * fpws::kH);
  return p;
}

// Node buffers for both sides, grown to hold `nodes` rows each.
fastpfp_status ensure_nodes(fastpfp_t h, int nodes) {
  WarmState* w = state(h);
  if (nodes <= w->node_cap) return FASTPFP_OK;
  const size_t c = (size_t)nodes, per_side = side_bytes(c);
  if (w->nbuf) (void)hipFree(w->nbuf);
  w->nbuf = nullptr;
  w->node_cap = 0;
  if (hipMalloc(&w->nbuf, 2 * per_side) != hipSuccess) {
    w->nbuf = nullptr;
    return fail(h, FASTPFP_ERR_NOMEM, "cannot allocate %zu bytes",
                2 * per_side);
  }
  char* p = (char*)w->nbuf;
  for (int s = 0; s < 2; ++s) p = carve_side(p, c, w->side[s]);
  w->node_cap = nodes;
  return FASTPFP_OK;
}

// The lanes of a batched forward pass: streams and events (created once, at
// the default priority) and node buffers for `nodes` rows per side.
fastpfp_status ensure_lanes(fastpfp_t h, int nodes) {
  WarmState* w = state(h);
  if (!w->start_ev &&
      hipEventCreateWithFlags(&w->start_ev, hipEventDisableTiming) !=
          hipSuccess) {
    w->start_ev = nullptr;
    return fail(h, FASTPFP_ERR_HIP, "cannot create an event");
  }
  for (int l = 0; l < WarmState::kLanes; ++l) {
    if (!w->lane_s[l] &&
        hipStreamCreateWithFlags(&w->lane_s[l], hipStreamNonBlocking) !=
            hipSuccess) {
      w->lane_s[l] = nullptr;
      return fail(h, FASTPFP_ERR_HIP, "cannot create a stream");
    }
    if (!w->lane_ev[l] &&
        hipEventCreateWithFlags(&w->lane_ev[l], hipEventDisableTiming) !=
            hipSuccess) {
      w->lane_ev[l] = nullptr;
      return fail(h, FASTPFP_ERR_HIP, "cannot create an event");
    }
  }
  if (nodes <= w->lane_cap) return FASTPFP_OK;
  const size_t c = (size_t)nodes, per_side = side_bytes(c);
  const size_t bytes = 2 * WarmState::kLanes * per_side;
  if (w->lbuf) (void)hipFree(w->lbuf);
  w->lbuf = nullptr;
  w->lane_cap = 0;
  if (hipMalloc(&w->lbuf, bytes) != hipSuccess) {
    w->lbuf = nullptr;
    return fail(h, FASTPFP_ERR_NOMEM, "cannot allocate %zu bytes", bytes);
  }
  char* p = (char*)w->lbuf;
  for (int l = 0; l < WarmState::kLanes; ++l)
    for (int s = 0; s < 2; ++s) p = carve_side(p, c, w->lside[l][s]);
  w->lane_cap = nodes;
  return FASTPFP_OK;
}

// Pair buffers: `elems` entries of S and Q (0 when only X0 is formed, which
// is written straight into the caller's buffer), `axis` entries of the
// per-row / per-column vectors.
fastpfp_status ensure_pair(fastpfp_t h, long long elems, int axis) {
  WarmState* w = state(h);
  if (w->qbuf && elems <= w->pair_cap && axis <= w->axis_cap)
    return FASTPFP_OK;
  elems = std::max(elems, w->pair_cap);
  axis = std::max(axis, w->axis_cap);
  const size_t bytes = 2 * up256(sizeof(float) * elems) +
                       up256(sizeof(float) * axis) +
                       up256(sizeof(double) * axis) +
                       up256(sizeof(double) * fpws::kLossBlocks) + 256 + 256;
  if (w->qbuf) (void)hipFree(w->qbuf);
  w->qbuf = nullptr;
  w->pair_cap = 0;
  w->axis_cap = 0;
  if (hipMalloc(&w->qbuf, bytes) != hipSuccess) {
    w->qbuf = nullptr;
    return fail(h, FASTPFP_ERR_NOMEM, "cannot allocate %zu bytes", bytes);
  }
  char* p = (char*)w->qbuf;
  auto take = [&](size_t b) {
    char* r = p;
    p += up256(b);
    return r;
  };
  w->S = (float*)take(sizeof(float) * elems);
  w->Q = (float*)take(sizeof(float) * elems);
  w->lse = (float*)take(sizeof(float) * axis);
  w->tsum = (double*)take(sizeof(double) * axis);
  w->partial = (double*)take(sizeof(double) * fpws::kLossBlocks);
  w->loss = (double*)take(sizeof(double));
  w->bad = (int*)take(sizeof(int));
  w->pair_cap = elems;
  w->axis_cap = axis;
  return FASTPFP_OK;
}

GemmArgs gemm(const float* A, long long sam, long long sak, const float* B,
              long long sbk, long long sbn, float* C, long long ldc, int M,
              int N, int K) {
  GemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.A = A;
  g.sam = sam;
  g.sak = sak;
  g.B = B;
  g.sbk = sbk;
  g.sbn = sbn;
  g.C = C;
  g.ldc = ldc;
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = 1.0f;
  return g;
}

#define WSCHK(call) HIPCHK(h, (call))

// Degrees, their means and the 48 features of one graph into d.x.
fastpfp_status features(fastpfp_t h, const Side& d, int n, const float* A,
                        int lda, const float* F, int ldf, int fdim,
                        hipStream_t s) {
  WSCHK(fpws_degree(A, lda, n, d.deg, d.wdeg, s));
  WSCHK(fpws_means(d.deg, d.wdeg, n, d.means, s));
  WSCHK(fpws_features(A, lda, n, d.deg, d.wdeg, d.means, F, ldf,
                      std::min(fdim, fpws::kAttr), d.x, fpws::kDin, s));
  return FASTPFP_OK;
}

// h1 = relu(x W1^T + b1), h2 = relu(h1 W2^T + b2), e = h2 W3^T + b3.
fastpfp_status mlp_forward(fastpfp_t h, const Side& d, int n,
                           const float* P, bool bf16, hipStream_t s) {
  using namespace fpws;
  GemmArgs g = gemm(d.x, kDin, 1, P + kOffW1, 1, kDin, d.h1, kH, n, kH, kDin);
  g.bias = P + kOffB1;
  g.relu = 1;
  g.round_b = bf16;
  WSCHK(fpws_gemm(&g, s));
  g = gemm(d.h1, kH, 1, P + kOffW2, 1, kH, d.h2, kH, n, kH, kH);
  g.bias = P + kOffB2;
  g.relu = 1;
  g.round_b = bf16;
  WSCHK(fpws_gemm(&g, s));
  g = gemm(d.h2, kH, 1, P + kOffW3, 1, kH, d.e, kDout, n, kDout, kH);
  g.bias = P + kOffB3;
  g.round_b = bf16;
  WSCHK(fpws_gemm(&g, s));
  return FASTPFP_OK;
}

// Backpropagates d.dE (n x kDout) through the MLP, accumulating into G.
fastpfp_status mlp_backward(fastpfp_t h, const Side& d, int n,
                            const float* P, float* G) {
  using namespace fpws;
  hipStream_t s = h->stream;
  // dW3 += dE^T h2 ; db3 += colsum(dE)
  GemmArgs g = gemm(d.dE, 1, kDout, d.h2, kH, 1, G + kOffW3, kH, kDout, kH, n);
  g.accumulate = 1;
  WSCHK(fpws_gemm(&g, s));
  WSCHK(fpws_colsum_acc(d.dE, kDout, n, kDout, G + kOffB3, s));
  // d2 = (dE W3) * (h2 > 0)
  g = gemm(d.dE, kDout, 1, P + kOffW3, kH, 1, d.d2, kH, n, kH, kDout);
  g.mask = d.h2;
  g.ldm = kH;
  WSCHK(fpws_gemm(&g, s));
  // dW2 += d2^T h1 ; db2 += colsum(d2)
  g = gemm(d.d2, 1, kH, d.h1, kH, 1, G + kOffW2, kH, kH, kH, n);
  g.accumulate = 1;
  WSCHK(fpws_gemm(&g, s));
  WSCHK(fpws_colsum_acc(d.d2, kH, n, kH, G + kOffB2, s));
  // d1 = (d2 W2) * (h1 > 0)
  g = gemm(d.d2, kH, 1, P + kOffW2, kH, 1, d.d1, kH, n, kH, kH);
  g.mask = d.h1;
  g.ldm = kH;
  WSCHK(fpws_gemm(&g, s));
  // dW1 += d1^T x ; db1 += colsum(d1)
  g = gemm(d.d1, 1, kH, d.x, kDin, 1, G + kOffW1, kDin, kH, kDin, n);
  g.accumulate = 1;
  WSCHK(fpws_gemm(&g, s));
  WSCHK(fpws_colsum_acc(d.d1, kH, n, kH, G + kOffB1, s));
  return FASTPFP_OK;
}

fastpfp_status check_graph_args(fastpfp_t h, int n, int np, const float* A,
                                int lda, const float* B, int ldb,
                                const float* F, int ldf, const float* G,
                                int ldg, int fdim) {
  if (n < 1 || np < 1 || n > h->max_n || np > h->max_np)
    return fail(h, FASTPFP_ERR_SHAPE, "n=%d n'=%d outside [1, %d] x [1, %d]",
                n, np, h->max_n, h->max_np);
  if (!A || !B) return fail(h, FASTPFP_ERR_INVALID_ARG, "A and B must be set");
  if (lda < n || ldb < np)
    return fail(h, FASTPFP_ERR_SHAPE, "a leading dimension is too small");
  if (fdim < 0)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "fdim must be >= 0");
  if (fdim > 0 && (!F || !G))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "fdim > 0 needs F and G");
  if (fdim > 0 && (ldf < std::min(fdim, fpws::kAttr) ||
                   ldg < std::min(fdim, fpws::kAttr)))
    return fail(h, FASTPFP_ERR_SHAPE, "ldf/ldg smaller than the attributes");
  return FASTPFP_OK;
}

fastpfp_status ready(fastpfp_t h) {
  if (!h) return FASTPFP_ERR_INVALID_ARG;
  if (!h->warm || !h->warm->loaded)
    return fail(h, FASTPFP_ERR_INVALID_ARG,
                "no warm-start parameters loaded (fastpfp_warmstart_load)");
  if (hipSetDevice(h->device) != hipSuccess)
    return fail(h, FASTPFP_ERR_HIP, "hipSetDevice(%d) failed", h->device);
  return FASTPFP_OK;
}

// Waits for the stream and turns the device-side flag into a status.
fastpfp_status finish(fastpfp_t h, const char* what) {
  int bad = 0;
  HIPCHK(h, hipMemcpyAsync(&bad, h->warm->bad, sizeof(int),
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (bad)
    return fail(h, FASTPFP_ERR_NUMERIC, "%s produced non-finite values", what);
  return FASTPFP_OK;
}

// Enqueues the forward pass of one pair: features, MLP of both graphs,
// S = E E'^T exp(-logtau) into X0, softmax in place; *bad_dev is set when an
// output is not finite.
fastpfp_status enqueue_x0(fastpfp_t h, int n, int np, const float* A, int lda,
                          const float* B, int ldb, const float* F, int ldf,
                          const float* G, int ldg, int fdim, bool bf16,
                          float* X0, int ldx, int* bad_dev, const Side& a,
                          const Side& b, hipStream_t s) {
  WarmState* w = h->warm;
  fastpfp_status st;
  if ((st = features(h, a, n, A, lda, F, ldf, fdim, s)) != FASTPFP_OK)
    return st;
  if ((st = features(h, b, np, B, ldb, G, ldg, fdim, s)) != FASTPFP_OK)
    return st;
  if ((st = mlp_forward(h, a, n, w->params(), bf16, s)) != FASTPFP_OK)
    return st;
  if ((st = mlp_forward(h, b, np, w->params(), bf16, s)) != FASTPFP_OK)
    return st;
  GemmArgs g = gemm(a.e, fpws::kDout, 1, b.e, 1, fpws::kDout, X0, ldx, n, np,
                    fpws::kDout);
  g.logtau = w->params() + fpws::kOffTau;
  HIPCHK(h, fpws_gemm(&g, s));
  HIPCHK(h, fpws_softmax(X0, ldx, X0, ldx, nullptr, n, np, n <= np ? 1 : 0,
                         bad_dev, s));
  return FASTPFP_OK;
}

}  // namespace

extern "C" {

fastpfp_status fastpfp_warmstart_load(fastpfp_t h, const void* blob_host,
                                      size_t bytes) {
  if (!h || !blob_host) return FASTPFP_ERR_INVALID_ARG;
  if (bytes != sizeof(float) * (size_t)fpws::kNumParams)
    return fail(h, FASTPFP_ERR_SHAPE, "parameter blob is %zu bytes, want %zu",
                bytes, sizeof(float) * (size_t)fpws::kNumParams);
  const float* src = (const float*)blob_host;
  for (int k = 0; k < fpws::kNumParams; ++k)
    if (!std::isfinite(src[k]))
      return fail(h, FASTPFP_ERR_INVALID_ARG, "parameter %d is not finite",
                  k);
  HIPCHK(h, hipSetDevice(h->device));
  WarmState* w = state(h);
  if (!w->pbuf &&
      hipMalloc((void**)&w->pbuf, 4 * sizeof(float) * fpws::kNumParams) !=
          hipSuccess) {
    w->pbuf = nullptr;
    return fail(h, FASTPFP_ERR_NOMEM, "cannot allocate the parameters");
  }
  HIPCHK(h, fpws_fill(w->grad(), 3LL * fpws::kNumParams, 0.0f, h->stream));
  HIPCHK(h, hipMemcpyAsync(w->params(), src, bytes, hipMemcpyHostToDevice,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  w->adam_t = 0;
  w->loaded = true;
  return FASTPFP_OK;
}

fastpfp_status fastpfp_warmstart_get(fastpfp_t h, float* params_host,
                                     float* grad_host, size_t count) {
  fastpfp_status st = ready(h);
  if (st != FASTPFP_OK) return st;
  if (count != (size_t)fpws::kNumParams)
    return fail(h, FASTPFP_ERR_SHAPE, "count must be %d", fpws::kNumParams);
  WarmState* w = h->warm;
  const size_t bytes = sizeof(float) * count;
  if (params_host)
    HIPCHK(h, hipMemcpyAsync(params_host, w->params(), bytes,
                             hipMemcpyDeviceToHost, h->stream));
  if (grad_host)
    HIPCHK(h, hipMemcpyAsync(grad_host, w->grad(), bytes,
                             hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return FASTPFP_OK;
}

fastpfp_status fastpfp_warmstart_features(fastpfp_t h, int n, const float* A,
                                          int lda, const float* F, int ldf,
                                          int fdim, float* x_out, int ldx) {
  if (!h) return FASTPFP_ERR_INVALID_ARG;
  if (n < 1 || n > std::max(h->max_n, h->max_np))
    return fail(h, FASTPFP_ERR_SHAPE, "n=%d outside [1, %d]", n,
                std::max(h->max_n, h->max_np));
  if (!A || lda < n)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "A must hold n x n");
  if (fdim < 0 || (fdim > 0 && (!F || ldf < std::min(fdim, fpws::kAttr))))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "bad attributes");
  if (!x_out || ldx < fpws::kDin)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "x_out must hold n x %d",
                fpws::kDin);
  fastpfp_status st;
  HIPCHK(h, hipSetDevice(h->device));
  if ((st = ensure_nodes(h, n)) != FASTPFP_OK) return st;
  const Side& d = h->warm->side[0];
  hipStream_t s = h->stream;
  HIPCHK(h, fpws_degree(A, lda, n, d.deg, d.wdeg, s));
  HIPCHK(h, fpws_means(d.deg, d.wdeg, n, d.means, s));
  HIPCHK(h, fpws_features(A, lda, n, d.deg, d.wdeg, d.means, F, ldf,
                          std::min(fdim, fpws::kAttr), x_out, ldx, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return FASTPFP_OK;
}

fastpfp_status fastpfp_warmstart(fastpfp_t h, int n, int np, const float* A,
                                 int lda, const float* B, int ldb,
                                 const float* F, int ldf, const float* G,
                                 int ldg, int fdim, int flags, float* X0,
                                 int ldx) {
  fastpfp_status st = ready(h);
  if (st != FASTPFP_OK) return st;
  if ((st = check_graph_args(h, n, np, A, lda, B, ldb, F, ldf, G, ldg,
                             fdim)) != FASTPFP_OK)
    return st;
  if (!X0 || ldx < np)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "X0 must hold n x n'");
  if (flags & ~FASTPFP_WS_BF16_WEIGHTS)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  if ((st = ensure_nodes(h, std::max(n, np))) != FASTPFP_OK) return st;
  if ((st = ensure_pair(h, 0, 0)) != FASTPFP_OK) return st;
  WarmState* w = h->warm;
  HIPCHK(h, fpws_fill_int(w->bad, 1, 0, h->stream));
  if ((st = enqueue_x0(h, n, np, A, lda, B, ldb, F, ldf, G, ldg, fdim,
                       (flags & FASTPFP_WS_BF16_WEIGHTS) != 0, X0, ldx,
                       w->bad, w->side[0], w->side[1], h->stream)) !=
      FASTPFP_OK)
    return st;
  return finish(h, "the warm start");
}

fastpfp_status fastpfp_warmstart_batched(
    fastpfp_t h, int batch, const int* n_host, const int* np_host,
    const float* A, const int64_t* offA_host, const float* B,
    const int64_t* offB_host, const float* F, const int64_t* offF_host,
    const float* G, const int64_t* offG_host, int fdim, int flags, float* X,
    const int64_t* offX_host, int* status_host) {
  fastpfp_status st = ready(h);
  if (st != FASTPFP_OK) return st;
  if (batch < 1 || !n_host || !np_host || !A || !offA_host || !B ||
      !offB_host || !X || !offX_host)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "NULL batch argument");
  if (fdim < 0 || (fdim > 0 && (!F || !G || !offF_host || !offG_host)))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "bad attributes");
  if (flags & ~FASTPFP_WS_BF16_WEIGHTS)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  int nodes = 1;
  for (int b = 0; b < batch; ++b) {
    const int n = n_host[b], np = np_host[b];
    if (n < 1 || np < 1 || n > h->max_n || np > h->max_np)
      return fail(h, FASTPFP_ERR_SHAPE, "pair %d: n=%d n'=%d out of range", b,
                  n, np);
    if (offA_host[b] < 0 || offB_host[b] < 0 || offX_host[b] < 0 ||
        (fdim > 0 && (offF_host[b] < 0 || offG_host[b] < 0)))
      return fail(h, FASTPFP_ERR_INVALID_ARG, "pair %d: negative offset", b);
    nodes = std::max(nodes, std::max(n, np));
  }
  if ((st = ensure_lanes(h, nodes)) != FASTPFP_OK) return st;
  if ((st = ensure_pair(h, 0, 0)) != FASTPFP_OK) return st;
  WarmState* w = h->warm;
  if (batch > w->bads_cap) {
    if (w->bads) (void)hipFree(w->bads);
    w->bads = nullptr;
    w->bads_cap = 0;
    if (hipMalloc((void**)&w->bads, sizeof(int) * batch) != hipSuccess) {
      w->bads = nullptr;
      return fail(h, FASTPFP_ERR_NOMEM, "cannot allocate %d flags", batch);
    }
    w->bads_cap = batch;
  }
  hipStream_t s = h->stream;
  HIPCHK(h, fpws_fill_int(w->bads, batch, 0, s));
  const bool bf16 = (flags & FASTPFP_WS_BF16_WEIGHTS) != 0;
  // pair b on lane b % kLanes: the lanes start after the caller's stream has
  // cleared the flags (and whatever it ran before), and the caller's stream
  // waits for all of them; each lane has its own node buffers, and every
  // pair writes only its own X0 and flag
  constexpr int L = WarmState::kLanes;
  HIPCHK(h, hipEventRecord(w->start_ev, s));
  for (int l = 0; l < L; ++l)
    HIPCHK(h, hipStreamWaitEvent(w->lane_s[l], w->start_ev, 0));
  for (int b = 0; b < batch; ++b) {
    const int n = n_host[b], np = np_host[b], l = b % L;
    const float* Fb = fdim > 0 ? F + offF_host[b] : nullptr;
    const float* Gb = fdim > 0 ? G + offG_host[b] : nullptr;
    st = enqueue_x0(h, n, np, A + offA_host[b], n, B + offB_host[b], np, Fb,
                    fdim, Gb, fdim, fdim, bf16, X + offX_host[b], np,
                    w->bads + b, w->lside[l][0], w->lside[l][1],
                    w->lane_s[l]);
    if (st != FASTPFP_OK) break;
  }
  // joined even after a failed enqueue, so that no lane is left running
  // work the caller's stream does not wait for
  for (int l = 0; l < L; ++l) {
    HIPCHK(h, hipEventRecord(w->lane_ev[l], w->lane_s[l]));
    HIPCHK(h, hipStreamWaitEvent(s, w->lane_ev[l], 0));
  }
  if (st != FASTPFP_OK) return st;
  std::vector<int> bad(batch);
  HIPCHK(h, hipMemcpyAsync(bad.data(), w->bads, sizeof(int) * batch,
                           hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  st = FASTPFP_OK;
  for (int b = 0; b < batch; ++b) {
    const fastpfp_status sb = bad[b] ? FASTPFP_ERR_NUMERIC : FASTPFP_OK;
    if (status_host) status_host[b] = sb;
    if (sb != FASTPFP_OK && st == FASTPFP_OK) {
      st = sb;
      fail(h, sb, "pair %d: the warm start produced non-finite values", b);
    }
  }
  return st;
}

fastpfp_status fastpfp_warmstart_grad(fastpfp_t h, int n, int np,
                                      const float* A, int lda, const float* B,
                                      int ldb, const float* F, int ldf,
                                      const float* G, int ldg, int fdim,
                                      const float* T, int ldt,
                                      double* loss_host) {
  fastpfp_status st = ready(h);
  if (st != FASTPFP_OK) return st;
  if ((st = check_graph_args(h, n, np, A, lda, B, ldb, F, ldf, G, ldg,
                             fdim)) != FASTPFP_OK)
    return st;
  if (!T || ldt < np)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "T must hold n x n'");
  if ((st = ensure_nodes(h, std::max(n, np))) != FASTPFP_OK) return st;
  const int axis = n <= np ? 1 : 0;  // softmax over each row when n <= n'
  if ((st = ensure_pair(h, (long long)n * np, std::max(n, np))) != FASTPFP_OK)
    return st;
  WarmState* w = h->warm;
  hipStream_t s = h->stream;
  const float* P = w->params();
  float* Gr = w->grad();
  HIPCHK(h, fpws_fill_int(w->bad, 1, 0, s));
  const Side &a = w->side[0], &b = w->side[1];
  if ((st = features(h, a, n, A, lda, F, ldf, fdim, s)) != FASTPFP_OK)
    return st;
  if ((st = features(h, b, np, B, ldb, G, ldg, fdim, s)) != FASTPFP_OK)
    return st;
  if ((st = mlp_forward(h, a, n, P, false, s)) != FASTPFP_OK) return st;
  if ((st = mlp_forward(h, b, np, P, false, s)) != FASTPFP_OK) return st;
  using fpws::kDout;
  GemmArgs g = gemm(a.e, kDout, 1, b.e, 1, kDout, w->S, np, n, np, kDout);
  g.logtau = P + fpws::kOffTau;
  HIPCHK(h, fpws_gemm(&g, s));
  HIPCHK(h, fpws_softmax(w->S, np, w->Q, np, w->lse, n, np, axis, w->bad, s));
  HIPCHK(h, fpws_axis_sums(T, ldt, n, np, axis, w->tsum, s));
  const double inv_ns = 1.0 / (double)std::min(n, np);
  HIPCHK(h, fpws_dsoftmax(w->S, np, w->Q, np, w->lse, T, ldt, w->tsum, n, np,
                          axis, inv_ns, w->partial, w->loss, w->bad, s));
  // dE = dS E' exp(-logtau) ; dE' = dS^T E exp(-logtau)
  g = gemm(w->S, np, 1, b.e, kDout, 1, a.dE, kDout, n, kDout, np);
  g.logtau = P + fpws::kOffTau;
  HIPCHK(h, fpws_gemm(&g, s));
  g = gemm(w->S, 1, np, a.e, kDout, 1, b.dE, kDout, np, kDout, n);
  g.logtau = P + fpws::kOffTau;
  HIPCHK(h, fpws_gemm(&g, s));
  HIPCHK(h, fpws_tau_grad(a.e, a.dE, n * kDout, Gr + fpws::kOffTau, s));
  if ((st = mlp_backward(h, a, n, P, Gr)) != FASTPFP_OK) return st;
  if ((st = mlp_backward(h, b, np, P, Gr)) != FASTPFP_OK) return st;
  if (loss_host)
    HIPCHK(h, hipMemcpyAsync(loss_host, w->loss, sizeof(double),
                             hipMemcpyDeviceToHost, s));
  return finish(h, "the warm-start gradient");
}

fastpfp_status fastpfp_warmstart_zero_grad(fastpfp_t h) {
  fastpfp_status st = ready(h);
  if (st != FASTPFP_OK) return st;
  HIPCHK(h, fpws_fill(h->warm->grad(), fpws::kNumParams, 0.0f, h->stream));
  return FASTPFP_OK;
}

fastpfp_status fastpfp_warmstart_adam(fastpfp_t h, double lr, double beta1,
                                      double beta2, double eps,
                                      double grad_scale) {
  fastpfp_status st = ready(h);
  if (st != FASTPFP_OK) return st;
  if (!(lr > 0.0) || !std::isfinite(lr) || !(beta1 >= 0.0 && beta1 < 1.0) ||
      !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0) ||
      !std::isfinite(grad_scale))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  WarmState* w = h->warm;
  w->adam_t += 1;
  const double bc1 = 1.0 - std::pow(beta1, w->adam_t);
  const double bc2 = 1.0 - std::pow(beta2, w->adam_t);
  HIPCHK(h, fpws_adam(w->params(), w->grad(), w->adam_m(), w->adam_v(),
                      fpws::kNumParams, (float)lr, (float)beta1, (float)beta2,
                      (float)eps, (float)grad_scale, (float)bc1, (float)bc2,
                      h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return FASTPFP_OK;
}

}  // extern "C"
