// Kernels of the learned warm start.  The warm start is not part of FastPFP:
// it replaces Algorithm 1's uniform X0 by a softmax of similarities between
// per-node embeddings (the paper notes the method depends on its
// initialisation, Sec. 4.5).  All of it is small next to one outer step of
// the solver (about 61 kFLOP per node plus 2 n n' 64 for the similarities),
// so the kernels favour plainness and determinism over peak throughput:
// every reduction runs in a fixed order and no floating-point atomics are
// used, so repeated calls give bitwise-identical results.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "warmstart_internal.h"

namespace {

using fpws::GemmArgs;

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Round to the nearest bfloat16, ties to even (finite inputs; NaN stays NaN).
__device__ inline float bf16r(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// Histogram bin of a (weighted) degree v against the graph mean m > 0:
// floor((4 v) / m) in float64, clipped to [0, 15]; NaN lands in bin 0.
__device__ inline int bin_of(double v, double m) {
  double q = floor((4.0 * v) / m);
  q = fmin(fmax(q, 0.0), (double)(fpws::kBins - 1));
  return (int)q;
}

// One wave per row: number of nonzero entries and their sum (float64).
__global__ __launch_bounds__(256) void k_degree(const float* __restrict__ A,
                                                long long lda, int n,
                                                float* __restrict__ deg,
                                                double* __restrict__ wdeg) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;  // whole wave leaves together
  const float* a = A + (long long)row * lda;
  int cnt = 0;
  double s = 0.0;
  for (int k = lane; k < n; k += 64) {
    const float v = a[k];
    cnt += (v != 0.0f);
    s += (double)v;
  }
  cnt = wave_sum(cnt);
  s = wave_sum(s);
  if (lane == 0) {
    deg[row] = (float)cnt;
    wdeg[row] = s;
  }
}

// Single workgroup: means[0] = sum(deg) / n, means[1] = sum(wdeg) / n.
__global__ __launch_bounds__(256) void k_means(const float* __restrict__ deg,
                                               const double* __restrict__ wdeg,
                                               int n,
                                               double* __restrict__ means) {
  __shared__ double sd[256], sw[256];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = t; i < n; i += 256) {
    a += (double)deg[i];
    b += wdeg[i];
  }
  sd[t] = a;
  sw[t] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      sd[t] += sd[t + o];
      sw[t] += sw[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    means[0] = sd[0] / (double)n;
    means[1] = sw[0] / (double)n;
  }
}

// One wave per node i: histograms over i's neighbours k (A[i,k] != 0) of
// their degree and weighted-degree bins, divided by deg(i), then the node's
// attributes zero-padded to kAttr.  Integer counts make the histogram exact.
__global__ __launch_bounds__(256) void k_features(
    const float* __restrict__ A, long long lda, int n,
    const float* __restrict__ deg, const double* __restrict__ wdeg,
    const double* __restrict__ means, const float* __restrict__ F,
    long long ldf, int fdim, float* __restrict__ x, long long ldx) {
  __shared__ int cnt[4][2 * fpws::kBins];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + w;
  if (lane < 2 * fpws::kBins) cnt[w][lane] = 0;
  __syncthreads();
  const double md = means[0], mw = means[1];
  const bool use_d = md > 0.0, use_w = mw > 0.0;
  if (row < n) {
    const float* a = A + (long long)row * lda;
    for (int k = lane; k < n; k += 64) {
      if (a[k] != 0.0f) {
        if (use_d) atomicAdd(&cnt[w][bin_of((double)deg[k], md)], 1);
        if (use_w) atomicAdd(&cnt[w][fpws::kBins + bin_of(wdeg[k], mw)], 1);
      }
    }
  }
  __syncthreads();
  if (row < n && lane < fpws::kDin) {
    float v = 0.0f;
    if (lane < 2 * fpws::kBins) {
      const float d = deg[row];
      if (d > 0.0f) v = (float)((double)cnt[w][lane] / (double)d);
    } else {
      const int c = lane - 2 * fpws::kBins;
      if (F != nullptr && c < fdim) v = F[(long long)row * ldf + c];
    }
    x[(long long)row * ldx + lane] = v;
  }
}

// 64 x 64 output tile per workgroup, 4 x 4 outputs per thread, K in chunks
// of 16 staged through LDS.  Operand loads are bounds-checked (zero fill);
// the load pattern follows whichever stride of the operand is 1 so that
// global reads stay coalesced for both plain and transposed views.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ float As[16][68];
  __shared__ float Bs[16][68];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0f;
  const bool a_kfast = g.sak == 1;
  const bool b_nfast = g.sbn == 1;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int r, ka;
      if (a_kfast) {
        r = e >> 4;
        ka = e & 15;
      } else {
        ka = e >> 6;
        r = e & 63;
      }
      const int m = m0 + r, k = k0 + ka;
      As[ka][r] = (m < g.M && k < g.K)
                      ? g.A[(long long)m * g.sam + (long long)k * g.sak]
                      : 0.0f;
      int c, kb;
      if (b_nfast) {
        kb = e >> 6;
        c = e & 63;
      } else {
        c = e >> 4;
        kb = e & 15;
      }
      const int j = n0 + c, k2 = k0 + kb;
      float bv = (j < g.N && k2 < g.K)
                     ? g.B[(long long)k2 * g.sbk + (long long)j * g.sbn]
                     : 0.0f;
      if (g.round_b) bv = bf16r(bv);
      Bs[kb][c] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
    }
    __syncthreads();
  }
  float alpha = g.alpha;
  if (g.logtau) alpha *= expf(-g.logtau[0]);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = m0 + ty + 16 * r;
    if (m >= g.M) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = n0 + tx + 16 * c;
      if (j >= g.N) continue;
      float v = alpha * acc[r][c];
      if (g.bias) v += g.bias[j];
      if (g.relu && v < 0.0f) v = 0.0f;  // NaN passes through, as in max()
      if (g.mask && !(g.mask[(long long)m * g.ldm + j] > 0.0f)) v = 0.0f;
      float* dst = g.C + (long long)m * g.ldc + j;
      *dst = g.accumulate ? *dst + v : v;
    }
  }
}

// Row softmax, one wave per row.  Three sweeps: max, sum of exponentials,
// write.  Q may alias S (each element is read before it is written by the
// same lane).
__global__ __launch_bounds__(256) void k_softmax_rows(
    const float* S, long long lds, float* Q, long long ldq,
    float* __restrict__ lse, int rows, int cols, int* __restrict__ bad) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const float* s = S + (long long)row * lds;
  float* q = Q + (long long)row * ldq;
  float mx = -INFINITY;
  for (int k = lane; k < cols; k += 64) mx = fmaxf(mx, s[k]);
  mx = wave_max(mx);
  float z = 0.0f;
  for (int k = lane; k < cols; k += 64) z += expf(s[k] - mx);
  z = wave_sum(z);
  const float inv = 1.0f / z;
  int nf = 0;
  for (int k = lane; k < cols; k += 64) {
    const float v = expf(s[k] - mx) * inv;
    nf |= !isfinite(v);
    q[k] = v;
  }
  nf = wave_sum(nf);
  if (lane == 0) {
    if (lse) lse[row] = mx + logf(z);
    if (nf) atomicOr(bad, 1);
  }
}

// Column softmax, one thread per column (reads coalesced across threads).
__global__ __launch_bounds__(256) void k_softmax_cols(
    const float* S, long long lds, float* Q, long long ldq,
    float* __restrict__ lse, int rows, int cols, int* __restrict__ bad) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  float mx = -INFINITY;
  for (int i = 0; i < rows; ++i) mx = fmaxf(mx, S[(long long)i * lds + j]);
  float z = 0.0f;
  for (int i = 0; i < rows; ++i) z += expf(S[(long long)i * lds + j] - mx);
  const float inv = 1.0f / z;
  int nf = 0;
  for (int i = 0; i < rows; ++i) {
    const float v = expf(S[(long long)i * lds + j] - mx) * inv;
    nf |= !isfinite(v);
    Q[(long long)i * ldq + j] = v;
  }
  if (lse) lse[j] = mx + logf(z);
  if (nf) atomicOr(bad, 1);
}

// Float64 sums of T along rows (axis 1, one wave per row) or columns
// (axis 0, one thread per column).
__global__ __launch_bounds__(256) void k_row_sums(const float* __restrict__ T,
                                                  long long ldt, int rows,
                                                  int cols,
                                                  double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  double s = 0.0;
  for (int k = lane; k < cols; k += 64) s += (double)T[(long long)row * ldt + k];
  s = wave_sum(s);
  if (lane == 0) out[row] = s;
}

__global__ __launch_bounds__(256) void k_col_sums(const float* __restrict__ T,
                                                  long long ldt, int rows,
                                                  int cols,
                                                  double* __restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int i = 0; i < rows; ++i) s += (double)T[(long long)i * ldt + j];
  out[j] = s;
}

// Cross-entropy against the normalised target and its gradient with respect
// to S: P = T / (sum of T along the softmax axis), loss = -sum P log Q / ns
// with log Q = S - lse, and dS = (Q - P) / ns, written over S.  Each of the
// kLossBlocks workgroups leaves its partial loss in partial[block].
__global__ __launch_bounds__(256) void k_dsoftmax(
    float* S, long long lds, const float* __restrict__ Q, long long ldq,
    const float* __restrict__ lse, const float* __restrict__ T,
    long long ldt, const double* __restrict__ tsum, int rows, int cols,
    int axis, double inv_ns, double* __restrict__ partial,
    int* __restrict__ bad) {
  __shared__ double red[256];
  const long long total = (long long)rows * cols;
  const long long stride = (long long)gridDim.x * 256;
  double l = 0.0;
  int nf = 0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total;
       e += stride) {
    const int i = (int)(e / cols), j = (int)(e % cols);
    const int a = axis ? i : j;
    const double ts = tsum[a];
    nf |= !(ts > 0.0) || !isfinite(ts);
    const double P = (double)T[(long long)i * ldt + j] / ts;
    const float s = S[(long long)i * lds + j];
    if (P != 0.0) l -= P * ((double)s - (double)lse[a]);
    const double q = (double)Q[(long long)i * ldq + j];
    S[(long long)i * lds + j] = (float)((q - P) * inv_ns);
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] * inv_ns;
  if (nf) atomicOr(bad, 1);
}

// loss[0] = sum of partial[0..count) in index order.
__global__ void k_sum_partials(const double* __restrict__ partial, int count,
                               double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < count; ++b) s += partial[b];
  loss[0] = s;
}

// out[c] += sum_r D[r, c]: 64 columns per workgroup, four row groups whose
// partial sums are combined in group order.
__global__ __launch_bounds__(256) void k_colsum_acc(const float* __restrict__ D,
                                                    long long ldd, int rows,
                                                    int cols,
                                                    float* __restrict__ out) {
  __shared__ float part[4][64];
  const int cl = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  float s = 0.0f;
  if (c < cols)
    for (int r = grp; r < rows; r += 4) s += D[(long long)r * ldd + c];
  part[grp][cl] = s;
  __syncthreads();
  if (grp == 0 && c < cols)
    out[c] += ((part[0][cl] + part[1][cl]) + part[2][cl]) + part[3][cl];
}

// g_logtau[0] -= sum_k E[k] dE[k] (float64 accumulation, one workgroup):
// with S = E E'^T exp(-logtau) and dE = dS E' exp(-logtau), the derivative
// of the loss with respect to logtau is -sum dS * S = -sum_k E[k] dE[k].
__global__ __launch_bounds__(256) void k_tau_grad(const float* __restrict__ E,
                                                  const float* __restrict__ dE,
                                                  int count,
                                                  float* __restrict__ g) {
  __shared__ double red[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < count; k += 256)
    s += (double)E[k] * (double)dE[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[0] -= (float)red[0];
}

// Adam (Kingma & Ba, 2015) with bias correction; gradients are first
// multiplied by `scale` (1 / batch for a mean over pairs).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p,
                                              const float* __restrict__ g,
                                              float* __restrict__ m,
                                              float* __restrict__ v, int count,
                                              float lr, float b1, float b2,
                                              float eps, float scale,
                                              float bc1, float bc2) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= count) return;
  const float gk = g[k] * scale;
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p,
                                              long long count, float value) {
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k < count) p[k] = value;
}

__global__ __launch_bounds__(64) void k_fill_int(int* __restrict__ p,
                                                 int count, int value) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k < count) p[k] = value;
}

inline unsigned blocks_for(long long items, int per_block) {
  return (unsigned)((items + per_block - 1) / per_block);
}

}  // namespace

extern "C" {

hipError_t fpws_degree(const float* A, long long lda, int n, float* deg,
                       double* wdeg, hipStream_t s) {
  hipLaunchKernelGGL(k_degree, dim3(blocks_for(n, 4)), dim3(256), 0, s, A,
                     lda, n, deg, wdeg);
  return hipGetLastError();
}

hipError_t fpws_means(const float* deg, const double* wdeg, int n,
                      double* means, hipStream_t s) {
  hipLaunchKernelGGL(k_means, dim3(1), dim3(256), 0, s, deg, wdeg, n, means);
  return hipGetLastError();
}

hipError_t fpws_features(const float* A, long long lda, int n,
                         const float* deg, const double* wdeg,
                         const double* means, const float* F, long long ldf,
                         int fdim, float* x, long long ldx, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(blocks_for(n, 4)), dim3(256), 0, s, A,
                     lda, n, deg, wdeg, means, F, ldf, fdim, x, ldx);
  return hipGetLastError();
}

hipError_t fpws_gemm(const fpws::GemmArgs* g, hipStream_t s) {
  if (g->M <= 0 || g->N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm, dim3(blocks_for(g->N, 64), blocks_for(g->M, 64)),
                     dim3(256), 0, s, *g);
  return hipGetLastError();
}

hipError_t fpws_softmax(const float* S, long long lds, float* Q,
                        long long ldq, float* lse, int rows, int cols,
                        int axis, int* bad, hipStream_t s) {
  if (axis)
    hipLaunchKernelGGL(k_softmax_rows, dim3(blocks_for(rows, 4)), dim3(256),
                       0, s, S, lds, Q, ldq, lse, rows, cols, bad);
  else
    hipLaunchKernelGGL(k_softmax_cols, dim3(blocks_for(cols, 256)), dim3(256),
                       0, s, S, lds, Q, ldq, lse, rows, cols, bad);
  return hipGetLastError();
}

hipError_t fpws_axis_sums(const float* T, long long ldt, int rows, int cols,
                          int axis, double* sums, hipStream_t s) {
  if (axis)
    hipLaunchKernelGGL(k_row_sums, dim3(blocks_for(rows, 4)), dim3(256), 0, s,
                       T, ldt, rows, cols, sums);
  else
    hipLaunchKernelGGL(k_col_sums, dim3(blocks_for(cols, 256)), dim3(256), 0,
                       s, T, ldt, rows, cols, sums);
  return hipGetLastError();
}

hipError_t fpws_dsoftmax(float* S, long long lds, const float* Q,
                         long long ldq, const float* lse, const float* T,
                         long long ldt, const double* tsum, int rows,
                         int cols, int axis, double inv_ns, double* partial,
                         double* loss, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_dsoftmax, dim3(fpws::kLossBlocks), dim3(256), 0, s, S,
                     lds, Q, ldq, lse, T, ldt, tsum, rows, cols, axis, inv_ns,
                     partial, bad);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, partial,
                     fpws::kLossBlocks, loss);
  return hipGetLastError();
}

hipError_t fpws_colsum_acc(const float* D, long long ldd, int rows, int cols,
                           float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum_acc, dim3(blocks_for(cols, 64)), dim3(256), 0,
                     s, D, ldd, rows, cols, out);
  return hipGetLastError();
}

hipError_t fpws_tau_grad(const float* E, const float* dE, int count,
                         float* g_logtau, hipStream_t s) {
  hipLaunchKernelGGL(k_tau_grad, dim3(1), dim3(256), 0, s, E, dE, count,
                     g_logtau);
  return hipGetLastError();
}

hipError_t fpws_adam(float* p, const float* g, float* m, float* v, int count,
                     float lr, float b1, float b2, float eps, float scale,
                     float bc1, float bc2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(count, 256)), dim3(256), 0, s, p,
                     g, m, v, count, lr, b1, b2, eps, scale, bc1, bc2);
  return hipGetLastError();
}

hipError_t fpws_fill(float* p, long long count, float value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(count, 256)), dim3(256), 0, s, p,
                     count, value);
  return hipGetLastError();
}

hipError_t fpws_fill_int(int* p, int count, int value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(count, 64)), dim3(64), 0, s,
                     p, count, value);
  return hipGetLastError();
}

}  // extern "C"
