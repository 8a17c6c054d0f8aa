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
//                 of s and of max|dY|, one per tile row;
//   stream_final  s = 1^T D 1 (float64, fixed order), max|dY|, the stop test
//                 (max|dY| < eps2) and the pass count.
// After the stop test holds, later launches of the same call return at once,
// so the host can enqueue passes in chunks and check the flag in between.
// a_i = (1 - r_i)/N + (s - N)/N^2 is formed from the float64 parts as the
// on-chip path forms it.  In Dykstra's mode the matrix holds the signed w
// (projection x = max(w, 0)); a final launch writes x.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "project_stream_internal.h"

namespace fpfp {

constexpr int kSR = 64;            // rows per tile
constexpr int kSG = 4;             // rows whose loads are issued together
constexpr int kSC = 1024;          // columns per tile: 256 per wave
constexpr int kSW = kSC / 256;     // waves per tile
constexpr int kSThreads = 64 * kSW;
constexpr int kFThreads = 256;     // the final step's workgroup
constexpr int kRC = 64;            // reduction: columns (and rows) per workgroup
constexpr int kRQ = 16;            // reduction: waves, each over every kRQ-th tile
constexpr int kRThreads = 64 * kRQ;

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

// Y is touched once per pass.  kNT selects how its 16-byte accesses treat
// the caches: 0 plain, 1 non-temporal loads, 2 non-temporal loads and
// stores; stream_nt_policy picks, by matrix size, the one that measured
// fastest (non-temporal loads alone, or stores alone, gave nothing for a
// matrix four times the last-level cache; both together 8%).
typedef float f4v __attribute__((ext_vector_type(4)));
template <int kNT>
__device__ __forceinline__ f4v load_y4(const float* p) {
  if (kNT >= 1) return __builtin_nontemporal_load((const f4v*)p);
  return *(const f4v*)p;
}
template <int kNT>
__device__ __forceinline__ void store_y4(float* p, f4v v) {
  if (kNT >= 2) __builtin_nontemporal_store(v, (f4v*)p);
  else *(f4v*)p = v;
}

// Per-thread state of one workgroup's column slice.
struct ColSlice {
  long long cbase;  // first column of this thread
  bool cin[4];      // which of its 4 columns lie inside the matrix
  float bv[4];      // b_j of those columns
  float cs[4];      // column sums of the rows done so far
  float dm;         // max|dY| so far
};

// mode: 0 sums of Y only; 1 alternating pass; 2 Dykstra pass; 3 x = max(w, 0).
// kVec: lane owns 4 consecutive columns, read and written as one 16-byte
// access (needs N % 4 == 0 and a 16-byte aligned Y); otherwise 4 columns
// 64 apart, one 4-byte access each.  Either way a wave covers 256 columns.
// kFull: the kSR rows from r0 lie wholly inside the matrix in this
// workgroup's columns, so no access needs a bounds check.  Its loads and
// stores are then unconditional, which lets the compiler count them exactly
// and keep later rows' loads in flight while the current rows are stored (a
// conditional access makes it wait for all of them).
// Rows r0 .. r0 + kSR - 1: the update in place, column sums into cs, row
// partials of each wave's 256 columns into lrow[wave][i].
template <int kMode, bool kVec, bool kFull, int kNT>
__device__ __forceinline__ void pass_rows(const StreamState& st, long long r0,
                                          double sterm, float lo, ColSlice& c,
                                          float (&lrow)[kSW][kSR]) {
  const long long N = st.N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto col = [&](int k) -> long long {
    return kVec ? c.cbase + k : c.cbase + 64 * k;
  };
  // a_i of these rows, lane i holding row r0 + i; the row loop reads it back
  // with readlane, so that loop issues no loads besides those of Y
  static_assert(kSR == 64, "one row term per lane of a wave");
  float a_lane = 0.f;
  if (kMode == 1 || kMode == 2) {
    const long long r = r0 + lane;
    if (kFull || r < N) a_lane = (float)(st.a[r] + sterm);
  }
  // software pipeline: the loads of later rows are issued before the stores
  // of the current ones, so a wait for loads leaves stores in flight
  float ya[kSG][4], yb[kSG][4];
  auto load_rows = [&](int i0, float (&dst)[kSG][4]) {
#pragma unroll
    for (int g = 0; g < kSG; ++g) {
      const long long r = r0 + i0 + g;
      const float* row = st.Y + r * N;
      if (kVec) {
        f4v v = {0.f, 0.f, 0.f, 0.f};
        if (kFull || (r < N && c.cin[0])) v = load_y4<kNT>(row + c.cbase);
        dst[g][0] = v.x;
        dst[g][1] = v.y;
        dst[g][2] = v.z;
        dst[g][3] = v.w;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          dst[g][k] = (kFull || (r < N && c.cin[k])) ? row[col(k)] : 0.f;
      }
    }
  };
  // rows i0 .. i0 + kSG - 1, whose values are in yg
  auto do_rows = [&](int i0, const float (&yg)[kSG][4]) {
#pragma unroll
    for (int g = 0; g < kSG; ++g) {
      const long long r = r0 + i0 + g;
      float rs = 0.f;
      if (kFull || r < N) {
        float* row = st.Y + r * N;
        const float av = __int_as_float(
            __builtin_amdgcn_readlane(__float_as_int(a_lane), i0 + g));
        float o4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          o4[k] = 0.f;
          if (!c.cin[k]) continue;
          const float yv = yg[g][k];
          float out, x;
          if (kMode == 0) {
            out = yv;
            x = yv;
          } else if (kMode == 1) {
            out = fmaxf((yv + av) + c.bv[k], 0.f);
            x = out;
            c.dm = fmaxf(c.dm, fabsf(out - yv));
          } else if (kMode == 2) {
            out = (yv + av) + c.bv[k];
            x = fmaxf(out, 0.f);
            c.dm = fmaxf(c.dm, fabsf(x - fmaxf(yv, lo)));
          } else {
            out = fmaxf(yv, 0.f);
            x = out;
          }
          o4[k] = out;
          if (kMode != 0 && !kVec) row[col(k)] = out;
          rs += x;
          c.cs[k] += x;
        }
        if (kMode != 0 && kVec && c.cin[0]) {
          const f4v o = {o4[0], o4[1], o4[2], o4[3]};
          store_y4<kNT>(row + c.cbase, o);
        }
      }
      if (kMode != 3) {
        // row partial of this wave's 256 columns
        const float wr = wave_sum_f(rs);
        if (lane == 0) lrow[wave][i0 + g] = wr;
      }
    }
  };
  // two groups in flight, in two buffers used in turn: a group's loads are
  // issued as soon as its buffer is free, one group ahead of their use;
  // every load inside the loop is unconditional when kFull
  static_assert(kSR % (2 * kSG) == 0, "whole pairs of groups");
  load_rows(0, ya);
  load_rows(kSG, yb);
  for (int i0 = 0; i0 < kSR - 2 * kSG; i0 += 2 * kSG) {
    do_rows(i0, ya);
    load_rows(i0 + 2 * kSG, ya);
    do_rows(i0 + kSG, yb);
    load_rows(i0 + 3 * kSG, yb);
  }
  do_rows(kSR - 2 * kSG, ya);
  do_rows(kSR - kSG, yb);
}

// Workgroup (tr, tc): the row tile of kSR rows from tr * kSR in the kSC
// columns of tile column tc.  (Short workgroups dispatched in order stream
// HBM better than long ones that each walk several row tiles.)
template <int kMode, bool kVec, int kNT>
__global__ void __launch_bounds__(kSThreads)
stream_pass(StreamState st, int first) {
  if (__hip_atomic_load(st.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u &&
      kMode != 3)
    return;
  __shared__ float lrow[kSW][kSR];
  __shared__ float lmax[kSW];
  const long long N = st.N;
  const int tr = blockIdx.x, tc = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long r0 = (long long)tr * kSR;
  ColSlice c;
  c.cbase = (long long)tc * kSC + wave * 256 + (kVec ? 4 * lane : lane);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long j = kVec ? c.cbase + k : c.cbase + 64 * k;
    // with 16-byte access N % 4 == 0, so a lane's 4 columns are all inside
    // or all outside the matrix
    c.cin[k] = kVec ? c.cbase < N : j < N;
    c.bv[k] = (kMode == 1 || kMode == 2) && c.cin[k] ? st.b[j] : 0.f;
    c.cs[k] = 0.f;
  }
  c.dm = 0.f;
  const double invN = 1.0 / (double)N;
  const double sterm = (kMode == 1 || kMode == 2)
                           ? (st.scal[0] - (double)N) * invN * invN
                           : 0.0;
  const float lo = (kMode == 2 && first) ? -INFINITY : 0.f;
  if ((long long)(tc + 1) * kSC <= N && r0 + kSR <= N)
    pass_rows<kMode, kVec, true, kNT>(st, r0, sterm, lo, c, lrow);
  else
    pass_rows<kMode, kVec, false, kNT>(st, r0, sterm, lo, c, lrow);
  if (kMode == 3) return;
  // column partials of this tile's rows
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (c.cin[k])
      st.colpart[(long long)tr * N + (kVec ? c.cbase + k : c.cbase + 64 * k)] =
          c.cs[k];
  const float wm = wave_max_f(c.dm);
  if (lane == 0) lmax[wave] = wm;
  __syncthreads();
  if (threadIdx.x < kSR && r0 + threadIdx.x < N) {
    float v = lrow[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kSW; ++w) v += lrow[w][threadIdx.x];
    st.rowpart[(long long)tc * N + r0 + threadIdx.x] = v;
  }
  if (threadIdx.x == 0) {
    float m = lmax[0];
#pragma unroll
    for (int w = 1; w < kSW; ++w) m = fmaxf(m, lmax[w]);
    st.tmax[(long long)tr * gridDim.y + tc] = m;
  }
}

// Workgroup b reduces columns and rows b*kRC .. b*kRC + kRC - 1, one per
// lane: wave q sums the partials of tile rows (tile columns) q, q + kRQ,
// ..., so each load of a wave reads kRC consecutive floats; the kRQ wave
// sums are then added in wave order.  It writes (1 - r_i)/N (float64),
// b_j = (1 - c_j)/N and a float64 partial of s over its rows.  Since
// kRC = kSR, workgroup b also takes the max|dY| of tile row b.
__global__ void __launch_bounds__(kRThreads)
stream_reduce(StreamState st, int TR, int TC) {
  if (__hip_atomic_load(st.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
    return;
  static_assert(kRC == 64 && kRQ * 64 == kRThreads, "a lane per column");
  static_assert(kRC == kSR, "one reduce workgroup per tile row");
  __shared__ float lc[kRQ][kRC], lr[kRQ][kRC], lm[kRQ];
  const long long N = st.N;
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const long long g = (long long)blockIdx.x * kRC + lane;
  float c = 0.f, r = 0.f, m = 0.f;
  for (int k = threadIdx.x; k < TC; k += kRThreads)
    m = fmaxf(m, st.tmax[(long long)blockIdx.x * TC + k]);
  if (g < N) {
    // unrolled so that the independent loads are in flight together
#pragma unroll 8
    for (int k = q; k < TR; k += kRQ) c += st.colpart[(long long)k * N + g];
#pragma unroll 4
    for (int k = q; k < TC; k += kRQ) r += st.rowpart[(long long)k * N + g];
  }
  lc[q][lane] = c;
  lr[q][lane] = r;
  m = wave_max_f(m);
  if (lane == 0) lm[q] = m;
  __syncthreads();
  if (q != 0) return;
  if (lane == 0) {
    float mm = lm[0];
#pragma unroll
    for (int k = 1; k < kRQ; ++k) mm = fmaxf(mm, lm[k]);
    st.mpart[blockIdx.x] = mm;
  }
  double rpart = 0.0;
  if (g < N) {
    float cs = lc[0][lane], rs = lr[0][lane];
#pragma unroll
    for (int k = 1; k < kRQ; ++k) {
      cs += lc[k][lane];
      rs += lr[k][lane];
    }
    const double invN = 1.0 / (double)N;
    st.a[g] = (1.0 - (double)rs) * invN;
    st.b[g] = (float)((1.0 - (double)cs) * invN);
    rpart = (double)rs;
  }
  // this block's rows: partial of s, in lane order
  const double w = wave_sum_dd(rpart);
  if (lane == 0) st.spart[blockIdx.x] = w;
}

// One workgroup, after stream_reduce: s from the partials in block order,
// max|dY| from the tile-row maxima, the stop test and the pass count.
//   ctl: 0 running, 1 converged, 2 non-finite values.
//   scal[0] = s, scal[1] = last max|dY|; counters[0] = passes done.
__global__ void __launch_bounds__(kFThreads)
stream_final(StreamState st, int nparts, int is_pass, double tol) {
  if (__hip_atomic_load(st.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
    return;
  __shared__ double ld[4];
  __shared__ float lm[4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // unrolled so that the independent loads are in flight together
  double sp = 0.0;
#pragma unroll 8
  for (int k = t; k < nparts; k += kFThreads) sp += st.spart[k];
  float m = 0.f;
#pragma unroll 8
  for (int k = t; k < nparts; k += kFThreads) m = fmaxf(m, st.mpart[k]);
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

// Geometry of a pass over an N x N matrix: TR x TC tiles of kSR x kSC
// entries; nrb reduce workgroups.
extern "C" void fpfp_stream_geometry(long long N, int* TR, int* TC, int* nrb) {
  *TR = (int)((N + fpfp::kSR - 1) / fpfp::kSR);
  *TC = (int)((N + fpfp::kSC - 1) / fpfp::kSC);
  *nrb = (int)((N + fpfp::kRC - 1) / fpfp::kRC);
}

// How the pass treats the caches for Y (see load_y4): plain while the matrix
// fits in half of the 256 MiB last-level cache, non-temporal loads while it
// fits in the whole, non-temporal loads and stores beyond.
static int stream_nt_policy(long long N) {
  const long long bytes = 4 * N * N;
  return bytes > (256ll << 20) ? 2 : bytes > (128ll << 20) ? 1 : 0;
}

// mode 0: sums of Y; 1: alternating pass; 2: Dykstra pass; 3: final clamp.
// Enqueues the launches of one step on `stream`.
extern "C" hipError_t fpfp_stream_step(const fpfp::StreamState* st, int mode,
                                       int first, double tol,
                                       hipStream_t stream) {
  int TR, TC, nrb;
  fpfp_stream_geometry(st->N, &TR, &TC, &nrb);
  const dim3 grid(TR, TC), block(fpfp::kSThreads);
  const bool vec = st->N % 4 == 0 && ((uintptr_t)st->Y & 15u) == 0;
  const int nt = vec ? stream_nt_policy(st->N) : 0;
#define FPFP_PASS(M)                                                        \
  if (!vec)                                                                 \
    fpfp::stream_pass<M, false, 0><<<grid, block, 0, stream>>>(*st, first); \
  else if (nt == 0)                                                         \
    fpfp::stream_pass<M, true, 0><<<grid, block, 0, stream>>>(*st, first);  \
  else if (nt == 1)                                                         \
    fpfp::stream_pass<M, true, 1><<<grid, block, 0, stream>>>(*st, first);  \
  else                                                                      \
    fpfp::stream_pass<M, true, 2><<<grid, block, 0, stream>>>(*st, first);
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
  fpfp::stream_reduce<<<dim3(nrb), dim3(fpfp::kRThreads), 0, stream>>>(
      *st, TR, TC);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  fpfp::stream_final<<<dim3(1), dim3(fpfp::kFThreads), 0, stream>>>(
      *st, nrb, mode != 0, tol);
  return hipGetLastError();
}
