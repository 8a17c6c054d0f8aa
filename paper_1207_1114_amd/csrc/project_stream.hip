// Streaming inner projection (Algorithm 1, steps 4-7; eqs. P1, P2) for a
// matrix that does not fit on chip: Y stays in HBM and every pass reads and
// writes it once (8 N^2 bytes), so the pass is bound by HBM bandwidth.
//
// One pass is three launches on the caller's stream (the kernel boundaries
// make each one's results visible to the next without fences):
//   stream_pass   tiles of kSR x kSC entries: D = max(0, Y + a_i + b_j)
//                 written in place, with per-tile row partials, column
//                 partials and the tile's max|D - Y|;
//   stream_reduce r_i and c_j from the partials in a fixed order, giving
//                 (1 - r_i)/N (float64) and b_j = (1 - c_j)/N, and partials
//                 of s;
//   stream_final  s = 1^T D 1 (float64, fixed order), max|dY|, the stop test
//                 (max|dY| < eps2) and the pass count.
// After the stop test holds, later launches of the same call return at once,
// so the host can enqueue passes in chunks and check the flag in between.
// a_i = (1 - r_i)/N + (s - N)/N^2 is formed from the float64 parts as the
// on-chip path forms it.  With kDyk the tile holds Dykstra's signed w
// (projection x = max(w, 0)); a final launch writes x.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "project_stream_internal.h"

namespace fpfp {

constexpr int kSR = 64;            // rows per tile
constexpr int kSG = 4;             // rows whose loads are issued together
constexpr int kSC = 1024;          // columns per tile: 4 waves x 256
constexpr int kSThreads = 256;
constexpr int kRC = 16;            // reduction: columns (and rows) per workgroup
constexpr int kRQ = 16;            // reduction: partial chunks per column

// Wave sum with DPP moves (register to register, no LDS): four steps sum
// each 16-lane row, two row broadcasts carry the row sums up to lane 63.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(
                 0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}
__device__ __forceinline__ float wave_sum_f(float v) {
  v = dpp_add<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum_dd(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// mode: 0 sums of Y only; 1 alternating pass; 2 Dykstra pass; 3 x = max(w, 0).
// kVec: lane owns 4 consecutive columns, read and written as one 16-byte
// access (needs N % 4 == 0 and a 16-byte aligned Y); otherwise 4 columns
// 64 apart, one 4-byte access each.  Either way a wave covers 256 columns.
template <int kMode, bool kVec>
__global__ void __launch_bounds__(kSThreads)
stream_pass(StreamState st, int first) {
  if (__hip_atomic_load(st.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u &&
      kMode != 3)
    return;
  __shared__ float lrow[4][kSR];
  __shared__ float lmax[4];
  const long long N = st.N;
  const int tr = blockIdx.x, tc = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long r0 = (long long)tr * kSR;
  const long long cbase = (long long)tc * kSC + wave * 256 +
                          (kVec ? 4 * lane : lane);
  // column of this thread's k-th entry in a row
  auto col = [&](int k) -> long long {
    return kVec ? cbase + k : cbase + 64 * k;
  };
  float bv[4];
  bool cin[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long c = col(k);
    cin[k] = c < N;
    bv[k] = (kMode == 1 || kMode == 2) && cin[k] ? st.b[c] : 0.f;
  }
  const double invN = 1.0 / (double)N;
  const double sterm = (kMode == 1 || kMode == 2)
                           ? (st.scal[0] - (double)N) * invN * invN
                           : 0.0;
  const float lo = (kMode == 2 && first) ? -INFINITY : 0.f;
  float cs[4] = {0.f, 0.f, 0.f, 0.f};
  float dm = 0.f;
  // software pipeline: the loads of the next kSG rows are issued before the
  // stores of the current ones, so a wait for loads leaves stores in flight
  float y[kSG][4], yn[kSG][4];
  auto load_rows = [&](int i0, float (&dst)[kSG][4]) {
#pragma unroll
    for (int g = 0; g < kSG; ++g) {
      const long long r = r0 + i0 + g;
      const float* row = st.Y + r * N;
      if (kVec) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i0 + g < kSR && r < N && cin[0])
          v = *(const float4*)(row + cbase);
        dst[g][0] = v.x;
        dst[g][1] = v.y;
        dst[g][2] = v.z;
        dst[g][3] = v.w;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          dst[g][k] = (i0 + g < kSR && r < N && cin[k]) ? row[col(k)] : 0.f;
      }
    }
  };
  load_rows(0, y);
  for (int i0 = 0; i0 < kSR; i0 += kSG) {
    load_rows(i0 + kSG, yn);
#pragma unroll
    for (int g = 0; g < kSG; ++g) {
      const long long r = r0 + i0 + g;
      float rs = 0.f;
      if (r < N) {
        float* row = st.Y + r * N;
        const float av = (kMode == 1 || kMode == 2)
                             ? (float)(st.a[r] + sterm)
                             : 0.f;
        float o4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          o4[k] = 0.f;
          if (!cin[k]) continue;
          const float yv = y[g][k];
          float out, x;
          if (kMode == 0) {
            out = yv;
            x = yv;
          } else if (kMode == 1) {
            out = fmaxf((yv + av) + bv[k], 0.f);
            x = out;
            dm = fmaxf(dm, fabsf(out - yv));
          } else if (kMode == 2) {
            out = (yv + av) + bv[k];
            x = fmaxf(out, 0.f);
            dm = fmaxf(dm, fabsf(x - fmaxf(yv, lo)));
          } else {
            out = fmaxf(yv, 0.f);
            x = out;
          }
          o4[k] = out;
          if (kMode != 0 && !kVec) row[col(k)] = out;
          rs += x;
          cs[k] += x;
        }
        if (kMode != 0 && kVec && cin[0])
          *(float4*)(row + cbase) = make_float4(o4[0], o4[1], o4[2], o4[3]);
      }
      // row partial of this wave's 256 columns
      const float wr = wave_sum_f(rs);
      if (lane == 0) lrow[wave][i0 + g] = wr;
    }
#pragma unroll
    for (int g = 0; g < kSG; ++g)
#pragma unroll
      for (int k = 0; k < 4; ++k) y[g][k] = yn[g][k];
  }
  if (kMode == 3) return;
  // column partials of this tile's rows
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (cin[k]) st.colpart[(long long)tr * N + col(k)] = cs[k];
  const float wm = wave_max_f(dm);
  if (lane == 0) lmax[wave] = wm;
  __syncthreads();
  if (threadIdx.x < kSR) {
    const long long r = r0 + threadIdx.x;
    if (r < N)
      st.rowpart[(long long)tc * N + r] =
          ((lrow[0][threadIdx.x] + lrow[1][threadIdx.x]) +
           lrow[2][threadIdx.x]) + lrow[3][threadIdx.x];
  }
  if (threadIdx.x == 0)
    st.tmax[(long long)tr * gridDim.y + tc] =
        fmaxf(fmaxf(lmax[0], lmax[1]), fmaxf(lmax[2], lmax[3]));
}

// Workgroup b reduces columns and rows b*kRC .. b*kRC + kRC - 1: thread t
// sums chunk q = t / kRC of the partials of column / row b*kRC + t % kRC
// (every kRQ-th tile row / column), then the kRQ chunk sums are added in a
// fixed order.  It writes (1 - r_i)/N (float64), b_j = (1 - c_j)/N and a
// float64 partial of s over its rows.
__global__ void __launch_bounds__(kSThreads)
stream_reduce(StreamState st, int TR, int TC) {
  if (__hip_atomic_load(st.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
    return;
  __shared__ float lc[kRQ][kRC], lr[kRQ][kRC];
  const long long N = st.N;
  const int t = threadIdx.x, q = t / kRC, e = t % kRC;
  const int lane = t & 63, wave = t >> 6;
  const long long g = (long long)blockIdx.x * kRC + e;
  float c = 0.f, r = 0.f;
  if (g < N) {
    // unrolled so that the independent loads are in flight together
#pragma unroll 8
    for (int k = q; k < TR; k += kRQ) c += st.colpart[(long long)k * N + g];
#pragma unroll 4
    for (int k = q; k < TC; k += kRQ) r += st.rowpart[(long long)k * N + g];
  }
  lc[q][e] = c;
  lr[q][e] = r;
  __syncthreads();
  double rpart = 0.0;
  if (t < kRC && g < N) {
    float cs = 0.f, rs = 0.f;
#pragma unroll
    for (int k = 0; k < kRQ; ++k) {
      cs += lc[k][t];
      rs += lr[k][t];
    }
    const double invN = 1.0 / (double)N;
    st.a[g] = (1.0 - (double)rs) * invN;
    st.b[g] = (float)((1.0 - (double)cs) * invN);
    rpart = (double)rs;
  }
  // this block's rows: partial of s, in lane order within wave 0
  if (wave == 0) {
    const double w = wave_sum_dd(rpart);
    if (lane == 0) st.spart[blockIdx.x] = w;
  }
}

// One workgroup, after stream_reduce: s from the partials in block order,
// max|dY| over the tiles, the stop test and the pass count.
//   ctl: 0 running, 1 converged, 2 non-finite values.
//   scal[0] = s, scal[1] = last max|dY|; counters[0] = passes done.
__global__ void __launch_bounds__(kSThreads)
stream_final(StreamState st, int nparts, int ntiles, int is_pass,
             double tol) {
  if (__hip_atomic_load(st.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
    return;
  __shared__ double ld[4];
  __shared__ float lm[4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // unrolled so that the independent loads are in flight together
  double sp = 0.0;
#pragma unroll 8
  for (int k = t; k < nparts; k += kSThreads) sp += st.spart[k];
  float m = 0.f;
#pragma unroll 8
  for (int k = t; k < ntiles; k += kSThreads) m = fmaxf(m, st.tmax[k]);
  sp = wave_sum_dd(sp);
  m = wave_max_f(m);
  if (lane == 0) {
    ld[wave] = sp;
    lm[wave] = m;
  }
  __syncthreads();
  if (t == 0) {
    const double S = ((ld[0] + ld[1]) + ld[2]) + ld[3];
    const float M = fmaxf(fmaxf(lm[0], lm[1]), fmaxf(lm[2], lm[3]));
    st.scal[0] = S;
    unsigned ctl = 0u;
    if (!isfinite(S) || !isfinite(M)) {
      ctl = 2u;
    } else if (is_pass) {
      st.scal[1] = (double)M;
      st.counters[0] += 1u;
      if (M < tol) ctl = 1u;
    }
    if (ctl != 0u)
      __hip_atomic_store(st.ctl, ctl, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace fpfp

extern "C" void fpfp_stream_tiles(long long N, int* TR, int* TC) {
  *TR = (int)((N + fpfp::kSR - 1) / fpfp::kSR);
  *TC = (int)((N + fpfp::kSC - 1) / fpfp::kSC);
}

// mode 0: sums of Y; 1: alternating pass; 2: Dykstra pass; 3: final clamp.
// Enqueues the launches of one step on `stream`.
extern "C" hipError_t fpfp_stream_step(const fpfp::StreamState* st, int mode,
                                       int first, double tol,
                                       hipStream_t stream) {
  int TR, TC;
  fpfp_stream_tiles(st->N, &TR, &TC);
  const dim3 grid(TR, TC), block(fpfp::kSThreads);
  const bool vec = st->N % 4 == 0 && ((uintptr_t)st->Y & 15u) == 0;
#define FPFP_PASS(M)                                                       \
  if (vec) fpfp::stream_pass<M, true><<<grid, block, 0, stream>>>(*st, first); \
  else fpfp::stream_pass<M, false><<<grid, block, 0, stream>>>(*st, first);
  switch (mode) {
    case 0: FPFP_PASS(0) break;
    case 1: FPFP_PASS(1) break;
    case 2: FPFP_PASS(2) break;
    default:
      FPFP_PASS(3)
      return hipGetLastError();
  }
#undef FPFP_PASS
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned nrb = (unsigned)((st->N + fpfp::kRC - 1) / fpfp::kRC);
  fpfp::stream_reduce<<<dim3(nrb), block, 0, stream>>>(*st, TR, TC);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  fpfp::stream_final<<<dim3(1), block, 0, stream>>>(*st, (int)nrb, TR * TC,
                                                    mode != 0, tol);
  return hipGetLastError();
}
