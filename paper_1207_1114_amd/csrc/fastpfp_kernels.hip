// Device code of the MI355X FastPFP library.
//
// One persistent launch solves a list of graph pairs.  Its workgroups form
// teams of W; a team pulls one pair at a time from a queue and runs the whole
// of Algorithm 1 on it (Lu, Huang & Liu, arXiv 1207.1114, Sec. 4):
//
//   step 3    T^T = X^T A and Y[0:n,0:n'] = T B + lambda K   (two MFMA GEMMs)
//   steps 4-7 repeat Y <- max(0, Y + a 1^T + 1 b^T)           (eqs. P1, P2)
//             with a_i = (1 - r_i)/N + (s - N)/N^2, b_j = (1 - c_j)/N,
//             r = Y 1, c = Y^T 1, s = 1^T Y 1, until max|dY| < eps2 or I1
//   step 8    X <- (1 - alpha) X + alpha Y[0:n,0:n']           (eq. fastPFP)
//   step 9    X <- X / max(X)
//   until max|dX| < eps1 or I0 steps (Sec. 5, convergence criteria).
//
// P1 written as "Y + a_i + b_j" is the same matrix as the paper's
// Y + (1/N + s/N^2 - r/N) 1^T - 1 (c/N)^T, evaluated without forming the
// large cancelling terms r_i/N and s/N^2 separately.
//
// The team owns the slacked N x N matrix Y as a TR x TC grid of tiles, one per
// workgroup, held in registers for the whole inner loop.  Each inner pass is
// one team-wide exchange of tile row sums, column sums, tile totals and
// max|dY|: every word carries the exchange's sequence number in its high
// half, so the data itself is the signal and no separate barrier or fence is
// needed.  Bulk data (T, Y, X) crosses workgroups through global memory with
// agent-scope release/acquire fences around an exchange.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fastpfp_internal.h"

namespace fpfp {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------ exchange words
__device__ __forceinline__ uint64_t pack(unsigned seq, float v) {
  return ((uint64_t)seq << 32) | (uint64_t)__float_as_uint(v);
}
__device__ __forceinline__ float unpack(uint64_t w) {
  return __uint_as_float((unsigned)(w & 0xffffffffu));
}
__device__ __forceinline__ unsigned tag_of(uint64_t w) {
  return (unsigned)(w >> 32);
}
__device__ __forceinline__ void put_word(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t get_word(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-workgroup view of its team and of the launch.
struct Team {
  int team, rank, W, TR, TC, tr, tc;
  uint64_t* xb;        // this team's exchange words (both parities)
  long long par_words; // words per parity
  unsigned seq;        // sequence number of the last exchange
  unsigned* abort_flag;
  long long timeout;   // wall clock ticks one wait may last
};

struct Shared {
  // GEMM staging
  float lp[32][64];
  float lq[32][64];
  // projection reductions
  float rowred[kTileRows];
  float colred[4][kTileCols];
  float a_l[kTileRows];
  float b_l[kTileCols];
  float scal[512][kScal];
  float wred[4];
  double dred[4];
  int bad;
};

// Value the compiler cannot see through: recomputed wherever it is used, so
// per-element addresses and bounds masks derived from it are not hoisted out
// of the solver's long-lived loops (which would pin hundreds of registers).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Waits until the `n` (<= M) words base[k * stride] all carry tag `seq` and
// returns their payloads in out[].  Returns false when the launch is aborted
// or the wait outlives the timeout.
template <int M>
__device__ __forceinline__ bool gather(const uint64_t* base, long long stride,
                                       int n, unsigned seq, float (&out)[M],
                                       const Team& tm) {
  uint64_t v[M];
#pragma unroll
  for (int k = 0; k < M; ++k) v[k] = (k < n) ? get_word(base + k * stride) : 0;
  int spins = 0;
  long long t0 = 0;
  for (;;) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < M; ++k) ok &= (k >= n) || (tag_of(v[k]) == seq);
    if (ok) break;
    if ((++spins & 63) == 0) {
      if (__hip_atomic_load(tm.abort_flag, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT) != 0u)
        return false;
      const long long now = (long long)wall_clock64();
      if (t0 == 0) t0 = now;
      if (now - t0 > tm.timeout) {
        __hip_atomic_store(tm.abort_flag, 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int k = 0; k < M; ++k)
      if (k < n && tag_of(v[k]) != seq) v[k] = get_word(base + k * stride);
  }
#pragma unroll
  for (int k = 0; k < M; ++k) out[k] = unpack(v[k]);
  return true;
}

// Workgroup-uniform failure flag: true if any thread failed.
__device__ __forceinline__ bool wg_any(Shared& sh, bool fail) {
  return __syncthreads_or(fail) != 0;
}

// Scalar exchange: every workgroup posts kScal floats; afterwards sh.scal[w]
// holds workgroup w's values for this sequence number.
__device__ bool xchg_scalars(Team& tm, Shared& sh, const float (&mine)[kScal]) {
  unsigned seq = ++tm.seq;
  uint64_t* base = tm.xb + (seq & 1u) * tm.par_words +
                   (tm.par_words - (long long)tm.W * kScal);
  __syncthreads();
  if (threadIdx.x < kScal)
    put_word(base + tm.rank * kScal + threadIdx.x,
             pack(seq, mine[threadIdx.x]));
  bool fail = false;
  for (int w = threadIdx.x; w < tm.W; w += kThreads) {
    float v[kScal];
    if (!gather<kScal>(base + w * kScal, 1, kScal, seq, v, tm)) {
      fail = true;
      break;
    }
#pragma unroll
    for (int k = 0; k < kScal; ++k) sh.scal[w][k] = v[k];
  }
  return !wg_any(sh, fail);
}

// Team barrier for bulk data written with ordinary stores: release fence,
// scalar exchange, acquire fence.
__device__ bool team_sync_bulk(Team& tm, Shared& sh) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  float z[kScal] = {0.f, 0.f, 0.f, 0.f};
  bool ok = xchg_scalars(tm, sh, z);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok;
}

// ------------------------------------------------------------------- GEMM
// C[m][c] = sum_k P[k*ldp + m] * Q[k*ldq + c] for m < M, c < Nc, k < Kd,
// in 64 x 64 output tiles dealt round-robin over the team.  Each wave owns a
// 32 x 32 block computed with v_mfma_f32_32x32x2_f32; operands are staged
// through LDS 32 k-rows at a time.  epi(m, c, value) stores one result.
template <class Epi>
__device__ void team_gemm_f32(const float* __restrict__ P, int ldp,
                              const float* __restrict__ Q, int ldq, int M,
                              int Nc, int Kd, const Team& tm, Shared& sh,
                              Epi epi) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int tiles_m = (M + 63) / 64, tiles_n = (Nc + 63) / 64;
  const int ntiles = tiles_m * tiles_n;
  for (int q = tm.rank; q < ntiles; q += tm.W) {
    const int m0 = (q / tiles_n) * 64, n0 = (q % tiles_n) * 64;
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    for (int k0 = 0; k0 < Kd; k0 += 32) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int idx = tid + kThreads * e;
        const int kk = idx >> 6, mm = idx & 63;
        const int kg = k0 + kk;
        sh.lp[kk][mm] = (kg < Kd && m0 + mm < M) ? P[(long long)kg * ldp + m0 + mm] : 0.f;
        sh.lq[kk][mm] = (kg < Kd && n0 + mm < Nc) ? Q[(long long)kg * ldq + n0 + mm] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 32; kk += 2) {
        const float a = sh.lp[kk + (lane >> 5)][wr * 32 + (lane & 31)];
        const float b = sh.lq[kk + (lane >> 5)][wc * 32 + (lane & 31)];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
      }
    }
    // 32x32 accumulator layout: lane holds column (lane & 31) and rows
    // 8*(v/4) + 4*(lane/32) + (v%4).
    const int cc = n0 + wc * 32 + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int mm = m0 + wr * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      if (mm < M && cc < Nc) epi(mm, cc, acc[v]);
    }
  }
}

// ------------------------------------------------------- projection tiles
// Thread (pr, pc) of the 16 x 16 thread grid holds rows pr + 16a (a < kRA)
// and columns pc + 16b (b < kCB) of its workgroup's tile.
struct TileGeom {
  int N, h, w, r0, c0, hv, wv;  // hv, wv: rows / cols of the tile inside N
};

__device__ __forceinline__ TileGeom tile_geom(const Team& tm, int N) {
  TileGeom g;
  g.N = N;
  g.h = (N + tm.TR - 1) / tm.TR;
  g.w = (N + tm.TC - 1) / tm.TC;
  g.r0 = tm.tr * g.h;
  g.c0 = tm.tc * g.w;
  g.hv = max(0, min(g.h, N - g.r0));
  g.wv = max(0, min(g.w, N - g.c0));
  return g;
}

// Reduces per-thread row partials rs[kRA] over the 16 lanes that share a row
// phase (xor 8, 4, 2, 1), halving the live values at each step.  Afterwards
// lanes pc and pc^1 hold the full tile-row partial of row index a = pc >> 1.
__device__ __forceinline__ float reduce_rows16(float (&rs)[kRA], int pc) {
  const bool h3 = pc & 8, h2 = pc & 4, h1 = pc & 2;
  float t[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float send = h3 ? rs[k] : rs[k + 4];
    const float keep = h3 ? rs[k + 4] : rs[k];
    t[k] = keep + __shfl_xor(send, 8);
  }
  float u[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float send = h2 ? t[k] : t[k + 2];
    const float keep = h2 ? t[k + 2] : t[k];
    u[k] = keep + __shfl_xor(send, 4);
  }
  const float send = h1 ? u[0] : u[1];
  const float keep = h1 ? u[1] : u[0];
  float v = keep + __shfl_xor(send, 2);
  v += __shfl_xor(v, 1);
  return v;
}

// Reduces per-thread column partials cs[kCB] over the 4 row phases of a wave
// (lanes xor 32, 16).  Afterwards the lane holds 4 partials for columns
// b = k + 4*bit4(lane) + 8*bit5(lane), k < 4.
__device__ __forceinline__ void reduce_cols4(float (&cs)[kCB], int lane,
                                             float (&out)[4]) {
  const bool h5 = lane & 32, h4 = lane & 16;
  float t[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float send = h5 ? cs[k] : cs[k + 8];
    const float keep = h5 ? cs[k + 8] : cs[k];
    t[k] = keep + __shfl_xor(send, 32);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float send = h4 ? t[k] : t[k + 4];
    const float keep = h4 ? t[k + 4] : t[k];
    out[k] = keep + __shfl_xor(send, 16);
  }
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Polls three strided runs of exchange words -- up to kMaxRun words at
// base_r + k*str_r, up to kMaxRun at base_c + k*str_c and up to kScal at
// base_s + k -- until all carry tag `seq`, keeping every load in flight at
// once.  Returns false on abort or timeout.
constexpr int kMaxRun = 8;
__device__ __forceinline__ bool gather3(const uint64_t* base_r, long long str_r,
                                        int nr, const uint64_t* base_c,
                                        long long str_c, int nc,
                                        const uint64_t* base_s, int ns,
                                        unsigned seq, float* rsum, float* csum,
                                        float (&sv)[kScal], const Team& tm) {
  uint64_t vr[kMaxRun], vc[kMaxRun], vs[kScal];
#pragma unroll
  for (int k = 0; k < kMaxRun; ++k) {
    vr[k] = (k < nr) ? get_word(base_r + k * str_r) : ((uint64_t)seq << 32);
    vc[k] = (k < nc) ? get_word(base_c + k * str_c) : ((uint64_t)seq << 32);
  }
#pragma unroll
  for (int k = 0; k < kScal; ++k)
    vs[k] = (k < ns) ? get_word(base_s + k) : ((uint64_t)seq << 32);
  int spins = 0;
  long long t0 = 0;
  for (;;) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < kMaxRun; ++k)
      ok &= (tag_of(vr[k]) == seq) & (tag_of(vc[k]) == seq);
#pragma unroll
    for (int k = 0; k < kScal; ++k) ok &= (tag_of(vs[k]) == seq);
    if (ok) break;
    if ((++spins & 63) == 0) {
      if (__hip_atomic_load(tm.abort_flag, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT) != 0u)
        return false;
      const long long now = (long long)wall_clock64();
      if (t0 == 0) t0 = now;
      if (now - t0 > tm.timeout) {
        __hip_atomic_store(tm.abort_flag, 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int k = 0; k < kMaxRun; ++k) {
      if (tag_of(vr[k]) != seq) vr[k] = get_word(base_r + k * str_r);
      if (tag_of(vc[k]) != seq) vc[k] = get_word(base_c + k * str_c);
    }
#pragma unroll
    for (int k = 0; k < kScal; ++k)
      if (tag_of(vs[k]) != seq) vs[k] = get_word(base_s + k);
  }
  float r = 0.f, c = 0.f;
#pragma unroll
  for (int k = 0; k < kMaxRun; ++k) {
    if (k < nr) r += unpack(vr[k]);
    if (k < nc) c += unpack(vc[k]);
  }
  *rsum = r;
  *csum = c;
#pragma unroll
  for (int k = 0; k < kScal; ++k) sv[k] = unpack(vs[k]);
  return true;
}

// Sums of the register tile (row partials, column partials, tile total,
// max|dY| in dm) posted to the team; then reads back the full row sums of
// this tile's rows, full column sums of its columns, s = 1^T Y 1 and the
// team's max|dY|, and forms a (rows) and b (cols) in sh.a_l / sh.b_l.
// Returns false on abort; *s_out = s, *dmax_out = max|dY|.
__device__ bool exchange_sums(Team& tm, Shared& sh, const TileGeom& g,
                              float (&rs)[kRA], float (&cs)[kCB], float dm,
                              double* s_out, float* dmax_out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pc = lane & 15, pr = wave * 4 + (lane >> 4);
  // --- in-workgroup reductions
  const float rsum = reduce_rows16(rs, pc);
  float c4[4];
  reduce_cols4(cs, lane, c4);
  const float dw = wave_max(dm);
  __syncthreads();
  if ((pc & 1) == 0) sh.rowred[pr + 16 * (pc >> 1)] = rsum;
  {
    const int bb = 4 * ((lane >> 4) & 1) + 8 * ((lane >> 5) & 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) sh.colred[wave][pc + 16 * (bb + k)] = c4[k];
  }
  if (lane == 0) sh.wred[wave] = dw;
  __syncthreads();
  const float rowpart = (tid < kTileRows) ? sh.rowred[tid] : 0.f;
  const float colpart = sh.colred[0][tid] + sh.colred[1][tid] +
                        sh.colred[2][tid] + sh.colred[3][tid];
  const float dmw = fmaxf(fmaxf(sh.wred[0], sh.wred[1]),
                          fmaxf(sh.wred[2], sh.wred[3]));
  // tile total in float64 (fixed order)
  double ttot = 0.0;
  if (wave == 0) {
    ttot = (double)sh.rowred[lane] + (double)sh.rowred[lane + 64];
    ttot = wave_sum_d(ttot);
  }
  double s;
  float dmax, rfull, cfull;
  if (tm.W == 1) {
    // single-workgroup team: the tile is the whole matrix
    rfull = rowpart;
    cfull = colpart;
    if (tid == 0) {
      sh.dred[1] = ttot;
      sh.wred[0] = dmw;
    }
    __syncthreads();
    s = sh.dred[1];
    dmax = sh.wred[0];
  } else {
    // --- post
    const unsigned seq = ++tm.seq;
    uint64_t* buf = tm.xb + (seq & 1u) * tm.par_words;
    const long long NPR = (long long)tm.TR * g.h, NPC = (long long)tm.TC * g.w;
    uint64_t* rowp = buf;                        // [TC][NPR]
    uint64_t* colp = buf + tm.TC * NPR;          // [TR][NPC]
    uint64_t* scal = buf + (tm.par_words - (long long)tm.W * kScal);
    if (tid < g.h) put_word(rowp + tm.tc * NPR + g.r0 + tid, pack(seq, rowpart));
    if (tid < g.w) put_word(colp + tm.tr * NPC + g.c0 + tid, pack(seq, colpart));
    if (tid == 0) {
      const float hi = (float)ttot;
      const float lo = (float)(ttot - (double)hi);
      put_word(scal + tm.rank * kScal + 0, pack(seq, hi));
      put_word(scal + tm.rank * kScal + 1, pack(seq, lo));
      put_word(scal + tm.rank * kScal + 2, pack(seq, dmw));
      put_word(scal + tm.rank * kScal + 3, pack(seq, 0.f));
    }
    // --- gather: this thread's row (TC words), column (TR words) and one
    // workgroup's scalars, up to 8 + 8 + 4 words in flight together
    float sv[kScal];
    bool ok = true;
    rfull = 0.f;
    cfull = 0.f;
    for (int k0 = 0; k0 < kMaxTeamSide && ok; k0 += kMaxRun) {
      if (k0 >= tm.TC && k0 >= tm.TR) break;
      const int nr = tid < g.h ? min(kMaxRun, tm.TC - k0) : 0;
      const int nc = tid < g.w ? min(kMaxRun, tm.TR - k0) : 0;
      float r, c;
      ok = gather3(rowp + k0 * NPR + g.r0 + tid, NPR, nr,
                   colp + k0 * NPC + g.c0 + tid, NPC, nc, scal + tid * kScal,
                   (k0 == 0 && tid < tm.W) ? kScal : 0, seq, &r, &c, sv, tm);
      rfull += r;
      cfull += c;
      if (k0 == 0 && tid < tm.W) {
#pragma unroll
        for (int k = 0; k < kScal; ++k) sh.scal[tid][k] = sv[k];
      }
    }
    if (__syncthreads_or(!ok)) return false;
    // --- team scalars: s in float64 (fixed order), max|dY|
    if (wave == 0) {
      double t = 0.0;
      float m = 0.f;
      for (int w = lane; w < tm.W; w += 64) {
        t += (double)sh.scal[w][0] + (double)sh.scal[w][1];
        m = fmaxf(m, sh.scal[w][2]);
      }
      t = wave_sum_d(t);
      m = wave_max(m);
      if (lane == 0) {
        sh.dred[1] = t;
        sh.wred[0] = m;
      }
    }
    __syncthreads();
    s = sh.dred[1];
    dmax = sh.wred[0];
  }
  const double Nd = (double)g.N, invN = 1.0 / Nd;
  const double sterm = (s - Nd) * invN * invN;
  if (tid < kTileRows)
    sh.a_l[tid] = (tid < g.hv) ? (float)((1.0 - (double)rfull) * invN + sterm)
                               : -INFINITY;
  sh.b_l[tid] = (tid < g.wv) ? (float)((1.0 - (double)cfull) * invN) : -INFINITY;
  *s_out = s;
  *dmax_out = dmax;
  __syncthreads();
  return true;
}

__device__ __forceinline__ void load_ab(const Shared& sh, float (&av)[kRA],
                                        float (&bv)[kCB], int pr, int pc) {
#pragma unroll
  for (int a = 0; a < kRA; ++a) av[a] = sh.a_l[pr + 16 * a];
#pragma unroll
  for (int b = 0; b < kCB; ++b) bv[b] = sh.b_l[pc + 16 * b];
}

// ------------------------------------------------------ register tile I/O
// Y tile <-> global N x N row-major matrix.  Padding entries read as 0.
__device__ __forceinline__ void load_tile(float (&Yr)[kRA][kCB],
                                          const float* Y, int N,
                                          const TileGeom& g, int pr, int pc) {
  const int hv = opaque(g.hv), wv = opaque(g.wv);
#pragma unroll
  for (int a = 0; a < kRA; ++a) {
    const int li = pr + 16 * a;
    const float* rp = Y + (long long)(g.r0 + li) * N + g.c0 + pc;
#pragma unroll
    for (int b = 0; b < kCB; ++b)
      Yr[a][b] = (li < hv && pc + 16 * b < wv) ? rp[16 * b] : 0.f;
  }
}

__device__ __forceinline__ void store_tile(const float (&Yr)[kRA][kCB],
                                           float* Y, int N, const TileGeom& g,
                                           int pr, int pc) {
  const int hv = opaque(g.hv), wv = opaque(g.wv);
#pragma unroll
  for (int a = 0; a < kRA; ++a) {
    const int li = pr + 16 * a;
    float* rp = Y + (long long)(g.r0 + li) * N + g.c0 + pc;
#pragma unroll
    for (int b = 0; b < kCB; ++b)
      if (li < hv && pc + 16 * b < wv) rp[16 * b] = Yr[a][b];
  }
}

// Steps 4-7 on the register tile.  Returns false on abort; sets *numeric
// when a sum or max|dY| is not finite.
__device__ __forceinline__ bool inner_loop(float (&Yr)[kRA][kCB], Team& tm,
                                           Shared& sh, const TileGeom& g,
                                           int max_inner, float tol,
                                           DevInfo& info, bool* numeric,
                                           int pr, int pc) {
  float rs[kRA], cs[kCB];
#pragma unroll
  for (int a = 0; a < kRA; ++a) rs[a] = 0.f;
#pragma unroll
  for (int b = 0; b < kCB; ++b) cs[b] = 0.f;
#pragma unroll
  for (int a = 0; a < kRA; ++a)
#pragma unroll
    for (int b = 0; b < kCB; ++b) {
      rs[a] += Yr[a][b];
      cs[b] += Yr[a][b];
    }
  double s;
  float d = 0.f;
  if (!exchange_sums(tm, sh, g, rs, cs, 0.f, &s, &d)) return false;
  *numeric = !isfinite(s);
  int u = 0;
  d = 0.f;
  if (!*numeric) {
    for (u = 1; u <= max_inner; ++u) {
      float av[kRA], bv[kCB];
      load_ab(sh, av, bv, pr, pc);
      float dm = 0.f;
#pragma unroll
      for (int a = 0; a < kRA; ++a) rs[a] = 0.f;
#pragma unroll
      for (int b = 0; b < kCB; ++b) cs[b] = 0.f;
#pragma unroll
      for (int a = 0; a < kRA; ++a)
#pragma unroll
        for (int b = 0; b < kCB; ++b) {
          const float y = Yr[a][b];
          const float dd = fmaxf((y + av[a]) + bv[b], 0.f);
          dm = fmaxf(dm, fabsf(dd - y));
          rs[a] += dd;
          cs[b] += dd;
          Yr[a][b] = dd;
        }
      if (!exchange_sums(tm, sh, g, rs, cs, dm, &s, &d)) return false;
      if (!isfinite(s) || !isfinite(d)) {
        *numeric = true;
        break;
      }
      if (d < tol) break;
    }
    if (u > max_inner) {
      u = max_inner;
      info.inner_capped++;
    }
  }
  info.inner_total += u;
  info.inner_max = max(info.inner_max, u);
  info.eps2 = d;
  return true;
}

// Maximum over the workgroup of a per-thread value (all threads get it).
__device__ __forceinline__ float wg_max(Shared& sh, float v) {
  const float wm = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh.wred[threadIdx.x >> 6] = wm;
  __syncthreads();
  return fmaxf(fmaxf(sh.wred[0], sh.wred[1]), fmaxf(sh.wred[2], sh.wred[3]));
}

// --------------------------------------------------------------- the kernel
__global__ void __launch_bounds__(kThreads, 1)
fastpfp_persistent(LaunchDesc L) {
  __shared__ Shared sh;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pc = lane & 15, pr = wave * 4 + (lane >> 4);

  // XCD-aware team membership: workgroup b runs on XCD b % 8, so walking the
  // grid XCD by XCD keeps each team of W <= G/8 on one die.
  const int G = gridDim.x, per = G / kXcds;
  const int v = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  Team tm;
  tm.W = L.W;
  tm.team = v / L.W;
  tm.rank = v % L.W;
  if (tm.team >= L.num_teams) return;
  tm.TR = L.TR;
  tm.TC = L.TC;
  tm.tr = tm.rank / L.TC;
  tm.tc = tm.rank % L.TC;
  tm.xb = L.xbuf + (long long)tm.team * L.xbuf_stride;
  tm.par_words = L.xbuf_stride / 2;
  tm.seq = 0;
  tm.abort_flag = L.queue + 1;
  tm.timeout = L.timeout_ticks;
  float* const Tt = L.wsT + (long long)tm.team * L.wsT_stride;
  float* const Yws = L.wsY + (long long)tm.team * L.wsY_stride;

  for (;;) {
    // ---- next pair: the team leader takes it from the queue and posts it
    if (tm.rank == 0 && tid == 0)
      sh.wred[0] = __uint_as_float(atomicAdd(L.queue, 1u));
    __syncthreads();
    {
      float post[kScal] = {sh.wred[0], 0.f, 0.f, 0.f};
      if (!xchg_scalars(tm, sh, post)) return;
    }
    const unsigned pidx =
        __builtin_amdgcn_readfirstlane(__float_as_uint(sh.scal[0][0]));
    if (pidx >= (unsigned)L.num_pairs) return;
    const PairDesc& pd = L.pairs[pidx];
    const int n = pd.n, np = pd.np, N = pd.N;
    float* const Y = pd.Y ? pd.Y : Yws;
    const TileGeom g = tile_geom(tm, N);
    DevInfo info = {0, 0, 0, 0, 0, 0, 0.f, 0.f};
    float Yr[kRA][kCB];

    if (pd.mode == kModeProject) {
      load_tile(Yr, Y, N, g, pr, pc);
      bool numeric = false;
      if (!inner_loop(Yr, tm, sh, g, pd.max_inner, pd.tol_in, info, &numeric,
                      pr, pc))
        return;
      store_tile(Yr, Y, N, g, pr, pc);
      info.status = numeric ? 5 : 0;
    } else {
      float* const X = pd.X;
      const int ldx = pd.ldx;
      // ---- initialisation (Algorithm 1, step 1): X0 and the slack
      {
        const int hv = opaque(g.hv), wv = opaque(g.wv);
        const float c0 = pd.init_c;
        const bool init_x = !pd.init_user, zero_y = !pd.y_user;
#pragma unroll
        for (int a = 0; a < kRA; ++a)
#pragma unroll
          for (int b = 0; b < kCB; ++b) {
            const int li = pr + 16 * a, lj = pc + 16 * b;
            const int i = g.r0 + li, j = g.c0 + lj;
            if (li < hv && lj < wv) {
              if (i < n && j < np) {
                if (init_x) X[(long long)i * ldx + j] = c0;
              } else if (zero_y) {
                Y[(long long)i * N + j] = 0.f;
              }
            }
          }
      }
      if (!team_sync_bulk(tm, sh)) return;
      for (int t = 1; t <= pd.max_outer; ++t) {
        // ---- step 3: T^T = X^T A  (np x n), then Y[:n,:np] = T B + lam K
        {
          float* const Tw = Tt;
          const int nn = n;
          team_gemm_f32(X, ldx, pd.A, pd.lda, np, n, n, tm, sh,
                        [=](int m, int c, float val) {
                          Tw[(long long)m * nn + c] = val;
                        });
        }
        if (!team_sync_bulk(tm, sh)) return;
        {
          const float lam = pd.lam;
          const float* const Kp = pd.K;
          const int ldk = pd.ldk, NN = N;
          float* const Yw = Y;
          team_gemm_f32(Tt, n, pd.B, pd.ldb, n, np, np, tm, sh,
                        [=](int m, int c, float val) {
                          float yv = val;
                          if (Kp) yv += lam * Kp[(long long)m * ldk + c];
                          Yw[(long long)m * NN + c] = yv;
                        });
        }
        if (!team_sync_bulk(tm, sh)) return;
        // ---- steps 4-7
        load_tile(Yr, Y, N, g, pr, pc);
        bool numeric = false;
        if (!inner_loop(Yr, tm, sh, g, pd.max_inner, pd.tol_in, info,
                        &numeric, pr, pc))
          return;
        if (numeric) {
          info.status = 5;
          break;
        }
        store_tile(Yr, Y, N, g, pr, pc);
        // ---- step 8: X_new = (1 - alpha) X + alpha Y[:n,:np]
        const float alpha = pd.alpha, beta = 1.f - pd.alpha;
        float mloc = 0.f;
        {
          const int hv = opaque(g.hv), wv = opaque(g.wv);
          const int nx = opaque(n), npx = opaque(np);
#pragma unroll
          for (int a = 0; a < kRA; ++a)
#pragma unroll
            for (int b = 0; b < kCB; ++b) {
              const int li = pr + 16 * a, lj = pc + 16 * b;
              const int i = g.r0 + li, j = g.c0 + lj;
              if (li < hv && lj < wv && i < nx && j < npx) {
                const float xo = X[(long long)i * ldx + j];
                const float xn = beta * xo + alpha * Yr[a][b];
                Yr[a][b] = xn;
                mloc = fmaxf(mloc, xn);
              }
            }
        }
        // ---- step 9: m = max X_new over the team, X = X_new / m
        {
          float post[kScal] = {wg_max(sh, mloc), 0.f, 0.f, 0.f};
          if (!xchg_scalars(tm, sh, post)) return;
        }
        float m = 0.f;
        for (int w = 0; w < tm.W; ++w) m = fmaxf(m, sh.scal[w][0]);
        if (!(m > 0.f) || !isfinite(m)) {
          info.status = 5;
          break;
        }
        const bool norm = pd.normalize;
        float eloc = 0.f;
        {
          const int hv = opaque(g.hv), wv = opaque(g.wv);
          const int nx = opaque(n), npx = opaque(np);
#pragma unroll
          for (int a = 0; a < kRA; ++a)
#pragma unroll
            for (int b = 0; b < kCB; ++b) {
              const int li = pr + 16 * a, lj = pc + 16 * b;
              const int i = g.r0 + li, j = g.c0 + lj;
              if (li < hv && lj < wv && i < nx && j < npx) {
                float* xp = X + (long long)i * ldx + j;
                const float xo = *xp;
                const float xv = norm ? Yr[a][b] / m : Yr[a][b];
                eloc = fmaxf(eloc, fabsf(xv - xo));
                *xp = xv;
              }
            }
        }
        {
          float post[kScal] = {wg_max(sh, eloc), 0.f, 0.f, 0.f};
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          if (!xchg_scalars(tm, sh, post)) return;
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        float e1 = 0.f;
        for (int w = 0; w < tm.W; ++w) e1 = fmaxf(e1, sh.scal[w][0]);
        info.eps1 = e1;
        info.outer = t;
        if (pd.trace && tm.rank == 0 && tid == 0) pd.trace[t - 1] = e1;
        if (e1 < pd.tol_out) {
          info.converged = 1;
          break;
        }
      }
    }
    if (tm.rank == 0 && tid == 0) *pd.info = info;
  }
}

}  // namespace fpfp

// Launch helper with C linkage for the host translation unit.
extern "C" hipError_t fpfp_launch_persistent(const fpfp::LaunchDesc* L,
                                             int grid, hipStream_t stream) {
  void* args[] = {const_cast<fpfp::LaunchDesc*>(L)};
  return hipLaunchCooperativeKernel((const void*)fpfp::fastpfp_persistent,
                                    dim3(grid), dim3(fpfp::kThreads), args, 0,
                                    stream);
}

extern "C" hipError_t fpfp_occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, (const void*)fpfp::fastpfp_persistent, fpfp::kThreads, 0);
}
