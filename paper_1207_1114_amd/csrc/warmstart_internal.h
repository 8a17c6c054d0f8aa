// Shapes and launch arguments of the learned warm start, shared by its
// kernels (warmstart.hip) and its host API (warmstart_api.cpp).  Not part of
// the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fpws {

// Node features: 16 degree bins, 16 weighted-degree bins, 16 attributes.
constexpr int kBins = 16;
constexpr int kAttr = 16;
constexpr int kDin = 2 * kBins + kAttr;  // 48
constexpr int kH = 128;                  // both hidden layers
constexpr int kDout = 64;                // embedding width

// Offsets of the flat parameter vector: W1 (kH x kDin), b1, W2 (kH x kH),
// b2, W3 (kDout x kH), b3, logtau.  Weights are row-major (out x in).
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kDin;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kDout * kH;
constexpr int kOffTau = kOffB3 + kDout;
constexpr int kNumParams = kOffTau + 1;  // 31041

constexpr int kLossBlocks = 512;  // fixed grid of the loss reduction

// C[m, j] (op)= alpha * sum_k A(m, k) B(k, j), with A(m, k) =
// A[m*sam + k*sak] and B(k, j) = B[k*sbk + j*sbn], then in order: + bias[j],
// relu, times (mask[m*ldm + j] > 0), and store or accumulate into C.
// When logtau is set, alpha is multiplied by exp(-logtau[0]).
// round_b rounds every B element to bfloat16 (nearest even) before use.
struct GemmArgs {
  const float* A;
  long long sam, sak;
  const float* B;
  long long sbk, sbn;
  float* C;
  long long ldc;
  const float* bias;
  const float* mask;
  long long ldm;
  const float* logtau;
  int M, N, K;
  float alpha;
  int relu, accumulate, round_b;
};

}  // namespace fpws

extern "C" {
hipError_t fpws_degree(const float* A, long long lda, int n, float* deg,
                       double* wdeg, hipStream_t s);
hipError_t fpws_means(const float* deg, const double* wdeg, int n,
                      double* means, hipStream_t s);
hipError_t fpws_features(const float* A, long long lda, int n,
                         const float* deg, const double* wdeg,
                         const double* means, const float* F, long long ldf,
                         int fdim, float* x, long long ldx, hipStream_t s);
hipError_t fpws_gemm(const fpws::GemmArgs* g, hipStream_t s);
// Softmax of S along rows (axis 1) or columns (axis 0) into Q (may alias S);
// lse (nullable) receives max + log(sum exp) per row / column; *bad is set
// to 1 when an output is not finite.
hipError_t fpws_softmax(const float* S, long long lds, float* Q,
                        long long ldq, float* lse, int rows, int cols,
                        int axis, int* bad, hipStream_t s);
hipError_t fpws_axis_sums(const float* T, long long ldt, int rows, int cols,
                          int axis, double* sums, hipStream_t s);
hipError_t fpws_dsoftmax(float* S, long long lds, const float* Q,
                         long long ldq, const float* lse, const float* T,
                         long long ldt, const double* tsum, int rows,
                         int cols, int axis, double inv_ns, double* partial,
                         double* loss, int* bad, hipStream_t s);
hipError_t fpws_colsum_acc(const float* D, long long ldd, int rows, int cols,
                           float* out, hipStream_t s);
hipError_t fpws_tau_grad(const float* E, const float* dE, int count,
                         float* g_logtau, hipStream_t s);
hipError_t fpws_adam(float* p, const float* g, float* m, float* v, int count,
                     float lr, float b1, float b2, float eps, float scale,
                     float bc1, float bc2, hipStream_t s);
hipError_t fpws_fill(float* p, long long count, float value, hipStream_t s);
hipError_t fpws_fill_int(int* p, int count, int value, hipStream_t s);
}
