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
//             (or, in fastpfp_persistent<true>, the exact projection of
//             eq. (DSP) by Dykstra's algorithm over the same two sets)
//   step 8    X <- (1 - alpha) X + alpha Y[0:n,0:n']           (eq. fastPFP)
//             (a Projected Gradient pair, eq. pg, writes X + step * gradient
//             in step 3 and takes alpha = 1 here)
//   step 9    X <- X / max(X)
//   until max|dX| < eps1 or I0 steps (Sec. 5, convergence criteria).
//
// P1 written as "Y + a_i + b_j" is the same matrix as the paper's
// Y + (1/N + s/N^2 - r/N) 1^T - 1 (c/N)^T, evaluated without forming the
// large cancelling terms r_i/N and s/N^2 separately.
//
// The team owns the slacked N x N matrix Y as a TR x TC grid of tiles of at
// most 256 x 256, one per workgroup (one workgroup per compute unit).  A tile
// stays on chip for the whole inner loop: half of each thread's 256 entries
// in registers, half in LDS.  Each inner pass is one team-wide exchange of
// tile row sums, column sums, tile totals and max|dY|: every 64-bit word
// carries the exchange's sequence number in its high half, so the data itself
// is the signal and no separate barrier or fence is needed.  Bulk data (T, Y,
// X) crosses workgroups through global memory with agent-scope
// release/acquire fences around an exchange.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fastpfp_internal.h"

namespace fpfp {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kLdsRows = kRA - kRegRows;  // tile rows per thread held in LDS

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
// Global-memory view of a device pointer.  Every matrix the kernel reads or
// writes is in device memory; through generic pointers those accesses become
// flat instructions, which also count against the LDS counter, so a wait for
// an LDS read (e.g. a product's operand tile) would wait for them as well.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gbl(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Per-workgroup view of its team.
struct Team {
  int team, rank, W, TR, TC, tr, tc;
  int die;             // 1: every workgroup of the team runs on one XCD
  uint64_t* xb;        // this team's exchange words (both parities)
  long long par_words; // words per parity
  unsigned seq;        // sequence number of the last exchange
  unsigned* abort_flag;
  long long timeout;   // wall clock ticks one wait may last
};

constexpr int kGT = 128;  // GEMM output tile (kGT x kGT per workgroup)
constexpr int kGK = 16;   // GEMM k-rows staged per step
constexpr int kBK = 32;   // BF16 GEMM k per step
#ifndef FPFP_BF16_STAGES
#define FPFP_BF16_STAGES 4
#endif
constexpr int kBfStages = FPFP_BF16_STAGES;  // BF16 k-steps held in LDS

struct Shared {
  union {
    // LDS-resident part of the projection tile: entry (a, b) of thread t at
    // ly[(a - kRegRows) * kCB + b][t] (consecutive threads, consecutive banks)
    float ly[kLdsRows * kCB][kThreads];
    struct {  // GEMM operand staging (the tile lives in global Y meanwhile)
      float lp[kGK][kGT];
      float lq[kGK][kGT];
    } g;
    struct {  // BF16 GEMM staging: a ring of k-steps, each the operands'
              // kGT x kBK and (up to) 256 x kBK slices as 16-byte chunks
      uint16_t ring[kBfStages][(kGT + 256) * kBK];
    } h;
  } t;
  float lcol[16][kTileCols];  // column partials [thread row pr][tile col]
  float lrow[kTileRows];
  float a_l[kTileRows];
  float b_l[kTileCols];
  float scal[kMaxTeam][kScal];
  float wred[4];
  double dred[3];
  double dtile[4];
};

// The workgroup's one Shared block.  Every function takes it from here, so
// that the out-of-line projection below addresses it as LDS too.
__device__ __forceinline__ Shared& shm() {
  __shared__ Shared sh;
  return sh;
}

// Value the compiler cannot see through: recomputed wherever it is used, so
// per-element addresses and bounds masks derived from it are not hoisted out
// of the solver's long-lived loops (which would pin hundreds of registers).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

__device__ __forceinline__ bool timed_out(const Team& tm, long long& t0) {
  if (__hip_atomic_load(gbl(tm.abort_flag), __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_AGENT) != 0u)
    return true;
  const long long now = (long long)wall_clock64();
  if (t0 == 0) t0 = now;
  if (now - t0 > tm.timeout) {
    __hip_atomic_store(gbl(tm.abort_flag), 1u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    return true;
  }
  return false;
}

// Cache policy of the exchange words (cache bits of the buffer
// instructions that move them).  Loads are always device-scope (sc1): they
// skip the compute unit's L1, which would otherwise keep answering a poll
// with the line it first fetched.  Agent: stores at device scope too, which
// write through to the memory-side cache that every XCD reads.  Die: for a
// team whose workgroups all run on one XCD, a plain store, which ends in that
// XCD's L2, where the team's device-scope loads find it: a post-and-poll
// round trip between two workgroups of one XCD measured 1217 cycles this way
// against 2176 with device-scope stores (a plain store is not seen from
// another XCD, whose L2 is separate).
struct PolAgent {
  static constexpr int ld = 16, st = 16;
};
struct PolDie {
  static constexpr int ld = 16, st = 0;
};

// Exchange words are addressed as word offsets into the team's buffer.
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t xrsrc(const Team& tm) {
  return __builtin_amdgcn_make_buffer_rsrc(
      tm.xb, 0, (int)(2 * tm.par_words * (long long)sizeof(uint64_t)),
      0x00020000);
}
template <class P>
__device__ __forceinline__ uint64_t ld_word(__amdgpu_buffer_rsrc_t r, int w) {
  const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, w * 8, 0, P::ld);
  return ((uint64_t)v.y << 32) | v.x;
}
template <class P>
__device__ __forceinline__ void st_word(__amdgpu_buffer_rsrc_t r, int w,
                                        uint64_t v) {
  u32x2 x;
  x.x = (unsigned)v;
  x.y = (unsigned)(v >> 32);
  __builtin_amdgcn_raw_buffer_store_b64(x, r, w * 8, 0, P::st);
}
// Compiler-only barrier for memory operations: the buffer loads are not
// atomics, so this keeps a post before the loads that wait for the other
// workgroups' posts, and a polling load inside its loop.
__device__ __forceinline__ void mem_order() { asm volatile("" ::: "memory"); }

// Gathers three strided runs of exchange words -- nr (<= 8) words at
// off_r + k*str_r, nc (<= 8) at off_c + k*str_c and ns (<= kScal) at
// off_s + k -- until all carry tag `seq`.  All loads are issued together,
// and while data is missing every missing word is reloaded each round, so
// the run completes one load after its last word becomes visible (polling
// one word and then reloading the rest cost a further round trip: 6.86 ->
// 6.63 us per pass at n = 1000 in teams of 16).  Returns false on abort or
// timeout.
constexpr int kMaxRun = 8;
template <class P>
__device__ __forceinline__ bool gather3(__amdgpu_buffer_rsrc_t rs, int off_r,
                                        int str_r, int nr, int off_c,
                                        int str_c, int nc, int off_s, int ns,
                                        unsigned seq, float* rsum, float* csum,
                                        float (&sv)[kScal], const Team& tm) {
  const uint64_t done = (uint64_t)seq << 32;
  uint64_t vr[kMaxRun], vc[kMaxRun], vs[kScal];
#pragma unroll
  for (int k = 0; k < kMaxRun; ++k) {
    vr[k] = (k < nr) ? ld_word<P>(rs, off_r + k * str_r) : done;
    vc[k] = (k < nc) ? ld_word<P>(rs, off_c + k * str_c) : done;
  }
#pragma unroll
  for (int k = 0; k < kScal; ++k)
    vs[k] = (k < ns) ? ld_word<P>(rs, off_s + k) : done;
  long long t0 = 0;
  int spins = 0;
  for (;;) {
    int wait_on = -1;
#pragma unroll
    for (int k = kScal - 1; k >= 0; --k)
      if (tag_of(vs[k]) != seq) wait_on = off_s + k;
#pragma unroll
    for (int k = kMaxRun - 1; k >= 0; --k) {
      if (tag_of(vc[k]) != seq) wait_on = off_c + k * str_c;
      if (tag_of(vr[k]) != seq) wait_on = off_r + k * str_r;
    }
    if (wait_on < 0) break;
    __builtin_amdgcn_s_sleep(1);
    mem_order();
    if ((++spins & 31) == 0 && timed_out(tm, t0)) return false;
#pragma unroll
    for (int k = 0; k < kMaxRun; ++k) {
      if (tag_of(vr[k]) != seq) vr[k] = ld_word<P>(rs, off_r + k * str_r);
      if (tag_of(vc[k]) != seq) vc[k] = ld_word<P>(rs, off_c + k * str_c);
    }
#pragma unroll
    for (int k = 0; k < kScal; ++k)
      if (tag_of(vs[k]) != seq) vs[k] = ld_word<P>(rs, off_s + k);
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

// Scalar exchange: every workgroup posts kScal floats; afterwards sh.scal[w]
// holds workgroup w's values for this sequence number.
__device__ bool xchg_scalars(Team& tm, Shared& sh, const float (&mine)[kScal]) {
  const unsigned seq = ++tm.seq;
  const __amdgpu_buffer_rsrc_t rs = xrsrc(tm);
  const int base = (int)((seq & 1u) * tm.par_words + tm.par_words) -
                   tm.W * kScal;
  __syncthreads();
  if (threadIdx.x < kScal)
    st_word<PolAgent>(rs, base + tm.rank * kScal + threadIdx.x,
                      pack(seq, mine[threadIdx.x]));
  mem_order();
  const int w = threadIdx.x;
  bool ok = true;
  if (w < tm.W) {
    float sv[kScal], r, c;
    ok = gather3<PolAgent>(rs, 0, 0, 0, 0, 0, 0, base + w * kScal, kScal, seq,
                           &r, &c, sv, tm);
#pragma unroll
    for (int k = 0; k < kScal; ++k) sh.scal[w][k] = sv[k];
  }
  return __syncthreads_or(!ok) == 0;
}

// Team barrier for bulk data written with ordinary stores: release fence,
// scalar exchange, acquire fence.
__device__ bool team_sync_bulk(Team& tm, Shared& sh) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  const float z[kScal] = {0.f, 0.f, 0.f, 0.f};
  const bool ok = xchg_scalars(tm, sh, z);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok;
}

// ------------------------------------------------------------------- GEMM
// Output tile of a team product for work index q (rank + i * W in round i).
// When a team spans whole XCDs, row-major order gives the 32 ranks on one
// XCD a strip of one or two tile rows by every tile column (at n = 4000:
// one by 32), so their L2 holds a slice of every column panel.  When the
// grid divides into blocks of xg = gm x gn tiles, q instead walks the grid
// block by block, and the xg ranks of an XCD take one near-square block in
// each round (4 x 8 tiles for 32 ranks: 12 operand panels instead of 33).
// (With 128 x 256 tiles the block is 8 x 4.)  Teams smaller than an XCD
// keep row-major order (16 ranks cover 10 panels in it, 8 in blocks, and
// measured no faster).  Every tile is still
// computed once, by the same instructions, so results do not depend on the
// order.  The block size assumes 32 compute units per XCD, as on MI355X;
// elsewhere it is only a worse order.
constexpr int kXcdRanks = 32;
__device__ __forceinline__ int xcd_ranks(int W) {
  return W >= kXcdRanks ? kXcdRanks : 1;
}
struct TileMap {
  int tiles_n, gm, gn, bn, blocked;
};
__device__ __forceinline__ TileMap tile_map(int tiles_m, int tiles_n,
                                            int xg, bool wide) {
  TileMap t;
  t.tiles_n = tiles_n;
  int lg = 0;
  while ((2 << lg) <= xg) ++lg;  // xg = 2^lg for the powers of two used
  // tiles twice as wide as tall take the taller block (8 x 4), so that the
  // block stays near square in outputs
  const int small = 1 << (lg / 2);
  t.gm = wide ? xg / small : small;
  t.gn = xg / t.gm;
  t.blocked = xg >= 32 && (xg & (xg - 1)) == 0 && tiles_m % t.gm == 0 &&
              tiles_n % t.gn == 0;
  t.bn = t.blocked ? tiles_n / t.gn : 1;
  return t;
}
__device__ __forceinline__ void tile_of(const TileMap& t, int q, int& tm_,
                                        int& tn_) {
  if (!t.blocked) {
    tm_ = q / t.tiles_n;
    tn_ = q % t.tiles_n;
    return;
  }
  const int g = t.gm * t.gn, B = q / g, w = q % g;
  tm_ = (B / t.bn) * t.gm + w / t.gn;
  tn_ = (B % t.bn) * t.gn + w % t.gn;
}

// C[m][c] = sum_k P[k*ldp + m] * Q[k*ldq + c] for m < M, c < Nc, k < Kd,
// in kGT x kGT output tiles dealt round-robin over the team.  Each wave owns
// a 64 x 64 quarter as 2 x 2 blocks of v_mfma_f32_32x32x2_f32; operands are
// staged through LDS kGK k-rows at a time, the next step's operands being
// loaded into registers while the current one computes.  The epilogue takes
// each 32 x 32 block in three sweeps, so that its loads are in flight
// together and no store waits on a load: pre(m, c) loads what a result needs
// (it is also called at positions outside the result, m >= M or c >= Nc,
// where it must stay inside its operands), fin(value, pre) forms the value to
// store, and put(m, c, v) stores it (inside the result only).
template <class Pre, class Fin, class Put>
__device__ void team_gemm_f32(const float* __restrict__ P, int ldp,
                              const float* __restrict__ Q, int ldq, int M,
                              int Nc, int Kd, const Team& tm, Shared& sh,
                              Pre pre, Fin fin, Put put) {
  constexpr int kPer = kGK * kGT / kThreads;  // operand elements per thread
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int tiles_m = (M + kGT - 1) / kGT, tiles_n = (Nc + kGT - 1) / kGT;
  const int ntiles = tiles_m * tiles_n;
  for (int q = tm.rank; q < ntiles; q += tm.W) {
    const int m0 = (q / tiles_n) * kGT, n0 = (q % tiles_n) * kGT;
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
    // element e of this thread's share: k-row (tid + 256 e) / kGT, col % kGT
    const int mm = tid & (kGT - 1), kb = tid / kGT;
    const bool pm = m0 + mm < M, qm = n0 + mm < Nc;
    // Loads are unconditional, from addresses clamped into the operands, and
    // values outside them are zeroed when staged: one code path, so the
    // prefetch is not waited for where two paths would merge.
    const int pmc = min(m0 + mm, M - 1), qmc = min(n0 + mm, Nc - 1);
    float pa[kPer], qa[kPer];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int kg = min(k0 + kb + e * (kThreads / kGT), Kd - 1);
        pa[e] = gbl(P)[(long long)kg * ldp + pmc];
        qa[e] = gbl(Q)[(long long)kg * ldq + qmc];
      }
    };
    fetch(0);
    for (int k0 = 0; k0 < Kd; k0 += kGK) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const bool kin = k0 + kb + e * (kThreads / kGT) < Kd;
        sh.t.g.lp[kb + e * (kThreads / kGT)][mm] = (kin && pm) ? pa[e] : 0.f;
        sh.t.g.lq[kb + e * (kThreads / kGT)][mm] = (kin && qm) ? qa[e] : 0.f;
      }
      __syncthreads();
      if (k0 + kGK < Kd) fetch(k0 + kGK);
      // all of this step's operands first, so that the MFMAs issue back to
      // back instead of each group waiting on its own LDS reads
      float a0[kGK / 2], a1[kGK / 2], b0[kGK / 2], b1[kGK / 2];
#pragma unroll
      for (int q = 0; q < kGK / 2; ++q) {
        const int kr = 2 * q + (lane >> 5), col = lane & 31;
        a0[q] = sh.t.g.lp[kr][wr * 64 + col];
        a1[q] = sh.t.g.lp[kr][wr * 64 + 32 + col];
        b0[q] = sh.t.g.lq[kr][wc * 64 + col];
        b1[q] = sh.t.g.lq[kr][wc * 64 + 32 + col];
      }
      __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the MFMAs
#pragma unroll
      for (int q = 0; q < kGK / 2; ++q) {
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[q], b0[q], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[q], b1[q], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[q], b0[q], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[q], b1[q], acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();
    // 32x32 accumulator layout: lane holds column (lane & 31) and rows
    // 8*(v/4) + 4*(lane/32) + (v%4).
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int cc = n0 + wc * 64 + 32 * j + (lane & 31);
        float2 ad[16];
#pragma unroll
        for (int v = 0; v < 16; ++v)
          ad[v] = pre(m0 + wr * 64 + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) +
                          (v & 3),
                      cc);
        float yv[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) yv[v] = fin(acc[i][j][v], ad[v]);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int mr = m0 + wr * 64 + 32 * i + 8 * (v >> 2) +
                         4 * (lane >> 5) + (v & 3);
          if (mr < M && cc < Nc) put(mr, cc, yv[v]);
        }
      }
  }
}

// Round-to-nearest-even float -> bfloat16 bits (NaN stays NaN).
__device__ __forceinline__ uint16_t f2bf(float x) {
  const unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// C[m][c] = sum_k P[m*ld + k] * Q[c*ld + k] with bfloat16 operands and
// float32 accumulation (v_mfma_f32_32x32x16_bf16), over the zero-padded
// shadows: Mt a multiple of kGT, Nt of kWN, Kd of kBK; every tile is
// computed and pre / fin / put (as in team_gemm_f32) see all Mt x Nt
// results.  A workgroup's output tile is kGT x kWN (kWN = 128 or 256), each
// wave owning a 64 x kWN/2 part as 2 x kWN/64 blocks of 32 x 32: the wider
// tile does twice the products per operand read and per barrier (measured
// 15% faster on its own, the results bit for bit the same).
//
// Operands go from global memory straight into an LDS ring of kBfStages
// k-steps (global_load_lds_dwordx4: no registers, no LDS store
// instructions), kBfStages - 1 steps ahead of their use, so that many
// steps' loads are in flight against the latency of the last-level cache
// and HBM.  One barrier per k-step: after it, the step's slices are in LDS
// (each wave waited for its own loads) and every wave has finished reading
// the step whose slot the next loads overwrite.  The 16-byte chunk (row, kc)
// of a slice (kc = k / 8 in the step) sits at chunk row * 4 + (kc ^ ((row >>
// 1) & 3)), which keeps the operand reads (32 rows at one kc) free of bank
// conflicts; a direct load writes 64 consecutive chunks, so each lane loads
// the global chunk that belongs at its place.  The products run in the
// same order as a plain k loop (per accumulator: k ascending).
typedef __attribute__((address_space(3))) void lds_void;
template <int kWN, class Pre, class Fin, class Put>
__device__ void team_gemm_bf16(const uint16_t* __restrict__ P,
                               const uint16_t* __restrict__ Q, int ld, int Mt,
                               int Nt, int Kd, const Team& tm, Shared& sh,
                               Pre pre, Fin fin, Put put) {
  static_assert(kWN == 128 || kWN == 256, "tile widths built");
  constexpr int kNB = kWN / 64;       // 32-column blocks per wave
  constexpr int kQL = kWN / 64;       // Q loads per wave per step
  static_assert(kGT * 4 == 2 * 4 * 64, "two P loads of 64 chunks per wave");
  static_assert(kBfStages >= 3, "at least two steps in flight");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  // Arguments of an out-of-line function arrive in vector registers; the
  // sizes and the rank are the same in every lane, and saying so keeps the
  // loop tests scalar.
  ld = __builtin_amdgcn_readfirstlane(ld);
  const int tiles_n = __builtin_amdgcn_readfirstlane(Nt) / kWN;
  const int ntiles = (__builtin_amdgcn_readfirstlane(Mt) / kGT) * tiles_n;
  const int nsteps = __builtin_amdgcn_readfirstlane(Kd) / kBK;
  const int rank = __builtin_amdgcn_readfirstlane(tm.rank);
  const int W = __builtin_amdgcn_readfirstlane(tm.W);
  // the global chunk this lane loads into each of its wave's 64-chunk
  // blocks of a slice: two of P's 512 chunks, kQL of Q's kWN * 4
  int gp[2], gq[kQL];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int c = (wave * 2 + j) * 64 + lane, row = c >> 2;
    gp[j] = row * ld + ((c & 3) ^ ((row >> 1) & 3)) * 8;
  }
#pragma unroll
  for (int j = 0; j < kQL; ++j) {
    const int c = (wave * kQL + j) * 64 + lane, row = c >> 2;
    gq[j] = row * ld + ((c & 3) ^ ((row >> 1) & 3)) * 8;
  }
  // the chunk a lane reads for rows r0 + (lane & 31) at chunk kc
  const int rr = lane & 31, kh = lane >> 5;
  auto chunk = [&](int row, int kc) { return row * 4 + (kc ^ ((row >> 1) & 3)); };
  // wait for this wave's loads of the oldest step in flight (the newer
  // kBfStages - 2 steps, 2 + kQL loads each, may still be outstanding) and
  // for its LDS reads, then meet the other waves; a workgroup fence here
  // would wait for every load
  constexpr int kNW = (2 + kQL) * (kBfStages - 2);
  static_assert(kNW < 64, "vmcnt range");
  constexpr int kWait = (kNW & 15) | ((kNW >> 4) << 14) | (7 << 4) | (0 << 8);
  auto step_barrier = [&]() {
    __builtin_amdgcn_s_waitcnt(kWait);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  const TileMap map =
      tile_map(ntiles / tiles_n, tiles_n, xcd_ranks(W), kWN > kGT);
  for (int q = rank; q < ntiles; q += W) {
    int ti, tj;
    tile_of(map, q, ti, tj);
    const int m0 = ti * kGT, n0 = tj * kWN;
    floatx16 acc[2][kNB];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < kNB; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
    const uint16_t* const pt = P + (long long)m0 * ld;
    const uint16_t* const qt = Q + (long long)n0 * ld;
    // loads of step s into slot s % kBfStages; steps past the last load
    // the last again (into slots no longer read), so that every step issues
    // the same loads and the wait counts above hold
    auto issue = [&](int s) {
      const int slot = s % kBfStages;
      const int k0 = min(s, nsteps - 1) * kBK;
#pragma unroll
      for (int j = 0; j < 2; ++j)
        __builtin_amdgcn_global_load_lds(
            (const void*)(pt + gp[j] + k0),
            (lds_void*)&sh.t.h.ring[slot][(wave * 2 + j) * 64 * 8], 16, 0, 0);
#pragma unroll
      for (int j = 0; j < kQL; ++j)
        __builtin_amdgcn_global_load_lds(
            (const void*)(qt + gq[j] + k0),
            (lds_void*)&sh.t.h.ring[slot][(kGT * 4 + (wave * kQL + j) * 64) * 8],
            16, 0, 0);
    };
    // operands of one 16-k half step: x[0], x[1] rows of P, x[2 + j] rows of Q
    auto readx = [&](int slot, int kc, bf16x8 (&x)[2 + kNB]) {
      const uint16_t* const sp = sh.t.h.ring[slot];
      const uint16_t* const sq = sp + kGT * 4 * 8;
      x[0] = *(const bf16x8*)&sp[chunk(wr * 64 + rr, kc) * 8];
      x[1] = *(const bf16x8*)&sp[chunk(wr * 64 + 32 + rr, kc) * 8];
#pragma unroll
      for (int j = 0; j < kNB; ++j)
        x[2 + j] = *(const bf16x8*)&sq[chunk(wc * (kWN / 2) + 32 * j + rr, kc) * 8];
    };
#pragma unroll
    for (int s = 0; s < kBfStages - 1; ++s) issue(s);
    // k 0..15 of a step in x0, k 16..31 in x1; the reads of x1 run behind
    // the products of x0 after the first, those of the next step's x0
    // behind the products of x1, and the barrier sits between the two
    // halves of a step
    bf16x8 x0[2 + kNB], x1[2 + kNB];
    step_barrier();
    issue(kBfStages - 1);
    readx(0, kh, x0);
    for (int s = 0; s < nsteps; ++s) {
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0[0], x0[2], acc[0][0], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      readx(s % kBfStages, 2 + kh, x1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < kNB; ++j)
          if (i != 0 || j != 0)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                x0[i], x0[2 + j], acc[i][j], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      // also after the last step (its x0 is not used): with no branch here
      // the products below wait for x1's reads alone
      step_barrier();
      issue(s + kBfStages);
      readx((s + 1) % kBfStages, kh, x0);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < kNB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              x1[i], x1[2 + j], acc[i][j], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    // the repeated loads of the last step land in LDS after the loop: wait
    // for them before the ring's slots are filled again or the LDS is
    // given back to the caller
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        const int cc = n0 + wc * (kWN / 2) + 32 * j + (lane & 31);
        float2 ad[16];
#pragma unroll
        for (int v = 0; v < 16; ++v)
          ad[v] = pre(m0 + wr * 64 + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) +
                          (v & 3),
                      cc);
        float yv[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) yv[v] = fin(acc[i][j][v], ad[v]);
#pragma unroll
        for (int v = 0; v < 16; ++v)
          put(m0 + wr * 64 + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3),
              cc, yv[v]);
      }
  }
}

// ------------------------------------------------------- projection tiles
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

// Wave-wide reductions with DPP moves (register-to-register): butterflies
// within each 16-lane row, then row broadcasts; lane 63 ends up with the
// result, which is returned to every lane.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_mov(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}
#define FPFP_ROW_STEPS(STEP) \
  STEP(0xb1, 0xf) /* quad_perm [1,0,3,2] */ \
  STEP(0x4e, 0xf) /* quad_perm [2,3,0,1] */ \
  STEP(0x141, 0xf) /* row_half_mirror */ \
  STEP(0x140, 0xf) /* row_mirror */
#define FPFP_WAVE_STEPS(STEP) \
  FPFP_ROW_STEPS(STEP) \
  STEP(0x142, 0xa) /* row_bcast:15 */ \
  STEP(0x143, 0xc) /* row_bcast:31 */

__device__ __forceinline__ float wave_max(float v) {
  const int ninf = __float_as_int(-INFINITY);
#define STEP(C, R) v = fmaxf(v, __int_as_float(dpp_mov<C, R>(ninf, __float_as_int(v))));
  FPFP_WAVE_STEPS(STEP)
#undef STEP
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double wave_sum_d(double v) {
#define STEP(C, R)                                                       \
  {                                                                      \
    const long long bits = __double_as_longlong(v);                      \
    const int lo = dpp_mov<C, R>(0, (int)(bits & 0xffffffff));           \
    const int hi = dpp_mov<C, R>(0, (int)(bits >> 32));                  \
    v += __longlong_as_double(((long long)hi << 32) | (unsigned)lo);     \
  }
  FPFP_WAVE_STEPS(STEP)
#undef STEP
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffff), 63);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 16 lanes of a DPP row; every lane of the row gets it.
__device__ __forceinline__ float row16_sum(float v) {
#define STEP(C, R) v += __int_as_float(dpp_mov<C, R>(0, __float_as_int(v)));
  FPFP_ROW_STEPS(STEP)
#undef STEP
  return v;
}

// Cycles to sleep (in units of 64 clocks) between posting an exchange and
// the first load of it: about one store-to-visibility latency, so the first
// loads usually find the data instead of polling.  Measured with 16 teams of
// 16 at n = 1000 (in-solve pass time), device-scope posts: 3 -> 8.08 us,
// 8 -> 8.06, 16 -> 7.53, 24 -> 7.71, 32 -> 7.92, 48 -> 8.34 (shorter sleeps
// add polling traffic that slows every team); posts through one XCD's L2:
// 4 -> 6.90, 8 -> 6.89, 16 -> 6.91.
constexpr int kPostSleep = 8;

// One team exchange of a pass.  In: each thread's row partials rs[a] (over
// its kCB columns), column partials cs[b] (over its kRA rows) and its
// max|dY| dm.  Reduces them over the workgroup (rows with DPP within the 16
// lanes that share them, columns through LDS), posts the tile's row /
// column partials, total (float64 as hi + lo floats) and max|dY|, and
// gathers the full row sums of the tile's rows, column sums of its columns,
// s = 1^T Y 1 and the team's max|dY|.  Leaves a (rows) and b (columns) of P1
// in sh.a_l / sh.b_l.  Returns false on abort.
template <class P>
__device__ bool exchange_sums(Team& tm, Shared& sh, const TileGeom& g,
                              const float (&rs)[kRA], const float (&cs)[kCB],
                              float dm, double* s_out, float* dmax_out) {
  const int tid = threadIdx.x, pr = tid >> 4, pc = tid & 15;
  const int lane = tid & 63, wave = tid >> 6;
  {
    // row partials: lane pc of the row group keeps the sum for a = pc
    float mine = 0.f;
#pragma unroll
    for (int a = 0; a < kRA; ++a) {
      const float v = row16_sum(rs[a]);
      mine = (pc == a) ? v : mine;
    }
    sh.lrow[pr + 16 * pc] = mine;
  }
#pragma unroll
  for (int b = 0; b < kCB; ++b) sh.lcol[pr][pc + 16 * b] = cs[b];
  {
    const float wm = wave_max(dm);
    if (lane == 0) sh.wred[wave] = wm;
  }
  __syncthreads();
  // thread t: tile row t and tile column t
  const int t = tid;
  const float rpart = sh.lrow[t];
  float cpart = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) cpart += sh.lcol[k][t];
  const float dmw = fmaxf(fmaxf(sh.wred[0], sh.wred[1]),
                          fmaxf(sh.wred[2], sh.wred[3]));
  // tile total in float64 over the row partials (one partial per wave)
  {
    const double wt = wave_sum_d((double)rpart);
    if (lane == 0) sh.dtile[wave] = wt;
  }

  const double Nd = (double)g.N, invN = 1.0 / Nd;
  double s;
  float dmax, rfull, cfull;
  if (tm.W == 1) {
    // single-workgroup team: the tile is the whole matrix
    __syncthreads();
    rfull = rpart;
    cfull = cpart;
    s = ((sh.dtile[0] + sh.dtile[1]) + sh.dtile[2]) + sh.dtile[3];
    dmax = dmw;
  } else {
    const unsigned seq = ++tm.seq;
    const __amdgpu_buffer_rsrc_t rs = xrsrc(tm);
    const int buf = (int)((seq & 1u) * tm.par_words);
    const int NPR = tm.TR * g.h, NPC = tm.TC * g.w;
    const int rowp = buf;                        // [TC][NPR]
    const int colp = buf + tm.TC * NPR;          // [TR][NPC]
    const int scal = buf + (int)tm.par_words - tm.W * kScal;
    __syncthreads();  // the four waves' tile partials in sh.dtile
    // Every address and word of this thread's posts is formed first and the
    // stores then issue back to back: the memory counter also counts stores,
    // so a spill reload between two posts of a thread would hold the second
    // until the first is acknowledged.
    int ra = rowp + tm.tc * NPR + g.r0 + t;
    int ca = colp + tm.tr * NPC + g.c0 + t;
    // the tile's scalars: lane k < kScal of wave 0 posts word k (one 64-bit
    // word per lane, so no two words share a store)
    int sa = scal + tm.rank * kScal + tid;
    int post_r = t < g.h, post_c = t < g.w, post_s = tid < kScal;
    uint64_t wr = pack(seq, rpart), wc = pack(seq, cpart), ws = 0;
    if (post_s) {
      const double ttot = ((sh.dtile[0] + sh.dtile[1]) + sh.dtile[2]) +
                          sh.dtile[3];
      const float hi = (float)ttot;
      const float lo = (float)(ttot - (double)hi);
      ws = pack(seq, tid == 0 ? hi : tid == 1 ? lo : tid == 2 ? dmw : 0.f);
    }
    asm volatile("" : "+v"(ra), "+v"(ca), "+v"(sa), "+v"(post_r),
                 "+v"(post_c), "+v"(post_s), "+v"(wr), "+v"(wc), "+v"(ws));
    if (post_r) st_word<P>(rs, ra, wr);
    if (post_c) st_word<P>(rs, ca, wc);
    if (post_s) st_word<P>(rs, sa, ws);
    mem_order();
    __builtin_amdgcn_s_sleep(kPostSleep);
    // this thread's runs: TC row partials of row t and TR column partials of
    // column t (in chunks of 8), plus workgroup t's scalars
    const int nr = t < g.h ? tm.TC : 0, nc = t < g.w ? tm.TR : 0;
    bool ok = true;
    rfull = 0.f;
    cfull = 0.f;
    for (int k0 = 0; k0 < max(max(nr, nc), 1) && ok; k0 += kMaxRun) {
      float r, c, sv[kScal];
      const bool first = k0 == 0;
      ok = gather3<P>(rs, rowp + k0 * NPR + g.r0 + t, NPR,
                      min(kMaxRun, nr - k0), colp + k0 * NPC + g.c0 + t, NPC,
                      min(kMaxRun, nc - k0), scal + tid * kScal,
                      (first && tid < tm.W) ? kScal : 0, seq, &r, &c, sv, tm);
      rfull += r;
      cfull += c;
      if (first && tid < tm.W) {
#pragma unroll
        for (int k = 0; k < kScal; ++k) sh.scal[tid][k] = sv[k];
      }
    }
    if (__syncthreads_or(!ok)) return false;
    // team scalars: s in float64 (fixed order), max|dY|; every wave reduces
    // the same words in the same order, so all get the same bits without
    // another barrier
    {
      double tsum = 0.0;
      float m = 0.f;
      for (int w = lane; w < tm.W; w += 64) {
        tsum += (double)sh.scal[w][0] + (double)sh.scal[w][1];
        m = fmaxf(m, sh.scal[w][2]);
      }
      s = wave_sum_d(tsum);
      dmax = wave_max(m);
    }
  }
  sh.a_l[t] = (t < g.hv) ? (float)((1.0 - (double)rfull) * invN +
                                   (s - Nd) * invN * invN)
                         : -INFINITY;
  sh.b_l[t] = (t < g.wv) ? (float)((1.0 - (double)cfull) * invN) : -INFINITY;
  *s_out = s;
  *dmax_out = dmax;
  __syncthreads();
  return true;
}

// ------------------------------------------------------ tile I/O and loops
// Entry (a, b) of this thread's tile share: register Yr[a][b] for
// a < kRegRows, else LDS sh.ly[(a - kRegRows) * kCB + b][tid].
#define FPFP_LY(a, b) sh.t.ly[((a) - kRegRows) * kCB + (b)][threadIdx.x]

// Y tile <-> global N x N row-major matrix.  Padding entries read as 0.
__device__ __forceinline__ void load_tile(float (&Yr)[kRegRows][kCB],
                                          Shared& sh, const float* Y, int N,
                                          const TileGeom& g, int pr, int pc) {
  const int hv = opaque(g.hv), wv = opaque(g.wv);
#pragma unroll
  for (int a = 0; a < kRA; ++a) {
    const int li = pr + 16 * a;
    const auto rp = gbl(Y + (long long)(g.r0 + li) * N + g.c0 + pc);
#pragma unroll
    for (int b = 0; b < kCB; ++b) {
      const float v = (li < hv && pc + 16 * b < wv) ? rp[16 * b] : 0.f;
      if (a < kRegRows) Yr[a][b] = v;
      else FPFP_LY(a, b) = v;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

__device__ __forceinline__ void store_tile(const float (&Yr)[kRegRows][kCB],
                                           Shared& sh, float* Y, int N,
                                           const TileGeom& g, int pr, int pc) {
  const int hv = opaque(g.hv), wv = opaque(g.wv);
#pragma unroll
  for (int a = 0; a < kRA; ++a) {
    const int li = pr + 16 * a;
    const auto rp = gbl(Y + (long long)(g.r0 + li) * N + g.c0 + pc);
#pragma unroll
    for (int b = 0; b < kCB; ++b)
      if (li < hv && pc + 16 * b < wv)
        rp[16 * b] = (a < kRegRows) ? Yr[a][b] : FPFP_LY(a, b);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Steps 4-7 on the on-chip tile.  Returns false on abort; sets *numeric
// when a sum or max|dY| is not finite.
//
// kDyk selects the exact projection of eq. (DSP) by Dykstra's algorithm in
// place of Algorithm 1's plain alternation.  Only the clamp P2 needs
// Dykstra's correction (P1 projects onto an affine set), and the correction
// q = min(w, 0) and the iterate x = max(w, 0) never overlap, so the tile
// holds one signed matrix w = z + q (z the P1 output): a pass is
// w <- w + a 1^T + 1 b^T with a, b from the sums of x, and x = max(w, 0)
// when the loop ends.  The first pass starts from x = Y itself, as the plain
// loop does; max|dx| is the stopping measure.
template <bool kDyk, class P, bool kPart>
__device__ __forceinline__ bool inner_loop(float (&Yr)[kRegRows][kCB],
                                           Team& tm, Shared& sh,
                                           const TileGeom& g, int max_inner,
                                           float tol, DevInfo& info,
                                           bool* numeric, int pr, int pc) {
  float rs[kRA], cs[kCB];
#pragma unroll
  for (int a = 0; a < kRA; ++a) rs[a] = 0.f;
#pragma unroll
  for (int b = 0; b < kCB; ++b) cs[b] = 0.f;
#pragma unroll
  for (int a = 0; a < kRA; ++a)
#pragma unroll
    for (int b = 0; b < kCB; ++b) {
      const float y = (a < kRegRows) ? Yr[a][b] : FPFP_LY(a, b);
      rs[a] += y;
      cs[b] += y;
    }
  double s;
  float d = 0.f;
  if (!exchange_sums<P>(tm, sh, g, rs, cs, 0.f, &s, &d)) return false;
  *numeric = !isfinite(s);
  int u = 0;
  d = 0.f;
  // rows a < amax hold every row of the tile inside N
  const int amax = __builtin_amdgcn_readfirstlane((g.hv + 15) >> 4);
  if (!*numeric) {
    for (u = 1; u <= max_inner; ++u) {
      // LDS reads are issued well ahead of their use (one wave per SIMD has
      // nothing else to cover their latency): b of P1 first, a of P1 one row
      // ahead, the first LDS-resident row while the register rows are
      // updated, and each entry of a further LDS row as soon as the entry
      // above it has been updated
      float bv[kCB], yl[kCB];
#pragma unroll
      for (int b = 0; b < kCB; ++b) bv[b] = sh.b_l[pc + 16 * b];
      float av_next = sh.a_l[pr];
#pragma unroll
      for (int b = 0; b < kCB; ++b) yl[b] = FPFP_LY(kRegRows, b);
      float dm = 0.f;
      // Dykstra: floor of the previous iterate max(w, lo); the first pass
      // compares with the unclamped input
      const float lo = (kDyk && u == 1) ? -INFINITY : 0.f;
#pragma unroll
      for (int b = 0; b < kCB; ++b) cs[b] = 0.f;
      if constexpr (kPart) {
#pragma unroll
        for (int a = 0; a < kRA; ++a) rs[a] = 0.f;
      }
#pragma unroll
      for (int a = 0; a < kRA; ++a) {
        const float av_a = av_next;
        if (a + 1 < kRA) av_next = sh.a_l[pr + 16 * (a + 1)];
        // a partial tile skips its padding rows, whose entries stay exactly
        // 0 (a uniform branch; rs of a skipped row is 0)
        if (kPart && a >= amax) break;
        float r = 0.f;
#pragma unroll
        for (int b = 0; b < kCB; ++b) {
          const float y = (a < kRegRows) ? Yr[a][b] : yl[b];
          float dd;
          if constexpr (kDyk) {
            dd = (y + av_a) + bv[b];
            const float xn = fmaxf(dd, 0.f);
            dm = fmaxf(dm, fabsf(xn - fmaxf(y, lo)));
            r += xn;
            cs[b] += xn;
          } else {
            // max(y + t, 0) = y + max(t, -y) with t = a_i + b_j: the change
            // of the entry comes out directly, and the new entry is exactly
            // 0 where the clamp acts.  max(t, -y) as the median of
            // (t, -y, FLT_MAX): one instruction with -y as a source modifier
            // (an infinite t, from non-finite sums, is caught by the sums)
            const float del = __builtin_amdgcn_fmed3f(av_a + bv[b], -y,
                                                      3.402823466e38f);
            dd = y + del;
            dm = fmaxf(dm, fabsf(del));
            r += dd;
            cs[b] += dd;
          }
          if (a < kRegRows) {
            Yr[a][b] = dd;
          } else {
            FPFP_LY(a, b) = dd;
            // the register just used takes the same column of the next LDS
            // row, which then has the rest of this row to arrive
            if (a + 1 < kRA) yl[b] = FPFP_LY(a + 1, b);
          }
        }
        rs[a] = r;
      }
      if (!exchange_sums<P>(tm, sh, g, rs, cs, dm, &s, &d)) return false;
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
  if constexpr (kDyk) {
    // the projection is x = max(w, 0)
#pragma unroll
    for (int a = 0; a < kRA; ++a)
#pragma unroll
      for (int b = 0; b < kCB; ++b) {
        if (a < kRegRows) Yr[a][b] = fmaxf(Yr[a][b], 0.f);
        else FPFP_LY(a, b) = fmaxf(FPFP_LY(a, b), 0.f);
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

// ------------------------------------------------- out-of-line projection
// Steps 4-7 on the team's N x N matrix Y in global memory: this workgroup's
// tile is loaded, projected on chip and stored back.  A function of its own
// so that the register allocation of the inner loop is not shared with the
// solver's long-lived state (pair descriptor, step-3 and update addresses):
// that state is saved once around the call instead of competing with the
// tile's 128 registers in every pass.  Arguments arrive in vector registers;
// they are uniform and moved to scalar registers first.
struct ProjIn {
  float* Y;
  uint64_t* xb;
  unsigned* abort_flag;
  long long par_words, timeout;
  int N, max_inner, W, TR, TC, tr, tc, rank, store_always;
  unsigned seq;
  float tol;
};
struct ProjOut {
  unsigned seq;
  int ok, numeric, passes, capped;
  float eps2;
};

__device__ __forceinline__ int rfl(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ long long rfl64(long long v) {
  const int lo = rfl((int)(v & 0xffffffffll)), hi = rfl((int)(v >> 32));
  return ((long long)hi << 32) | (unsigned)lo;
}
template <class T>
__device__ __forceinline__ T* rflp(T* p) {
  return (T*)rfl64((long long)p);
}

template <bool kDyk, class P, bool kPart>
__device__ __attribute__((noinline)) ProjOut project_on_chip(ProjIn in) {
  Shared& sh = shm();
  const int tid = threadIdx.x, pr = tid >> 4, pc = tid & 15;
  Team tm;
  tm.team = 0;
  tm.die = 0;  // the policy is the template argument
  tm.W = rfl(in.W);
  tm.TR = rfl(in.TR);
  tm.TC = rfl(in.TC);
  tm.tr = rfl(in.tr);
  tm.tc = rfl(in.tc);
  tm.rank = rfl(in.rank);
  tm.xb = rflp(in.xb);
  tm.par_words = rfl64(in.par_words);
  tm.seq = (unsigned)rfl((int)in.seq);
  tm.abort_flag = rflp(in.abort_flag);
  tm.timeout = rfl64(in.timeout);
  const int N = rfl(in.N);
  float* const Y = rflp(in.Y);
  const TileGeom g = tile_geom(tm, N);
  float Yr[kRegRows][kCB];
  load_tile(Yr, sh, Y, N, g, pr, pc);
  DevInfo info = {0, 0, 0, 0, 0, 0, 0.f, 0.f, 0ull, 0ull, 0ull};
  bool numeric = false;
  ProjOut o;
  o.ok = inner_loop<kDyk, P, kPart>(Yr, tm, sh, g, rfl(in.max_inner),
                          __int_as_float(rfl(__float_as_int(in.tol))), info,
                          &numeric, pr, pc);
  if (o.ok && (!numeric || rfl(in.store_always)))
    store_tile(Yr, sh, Y, N, g, pr, pc);
  o.seq = tm.seq;
  o.numeric = numeric;
  o.passes = info.inner_total;
  o.capped = info.inner_capped;
  o.eps2 = info.eps2;
  return o;
}

// Runs project_on_chip for this workgroup of team tm and folds its counts
// into info.  Returns false on abort; sets *numeric as inner_loop does.
template <bool kDyk>
__device__ __forceinline__ bool project_team(Team& tm, float* Y, int N,
                                             int max_inner, float tol,
                                             bool store_always, DevInfo& info,
                                             bool* numeric) {
  ProjIn in;
  in.Y = Y;
  in.xb = tm.xb;
  in.abort_flag = tm.abort_flag;
  in.par_words = tm.par_words;
  in.timeout = tm.timeout;
  in.N = N;
  in.max_inner = max_inner;
  in.W = tm.W;
  in.TR = tm.TR;
  in.TC = tm.TC;
  in.tr = tm.tr;
  in.tc = tm.tc;
  in.rank = tm.rank;
  in.store_always = store_always;
  in.seq = tm.seq;
  in.tol = tol;
  // tiles with padding rows take the sweep that skips them (skipping
  // padding columns too, in groups, broke the sweep into blocks too short
  // to schedule well and was slower at most sizes).  Dykstra's build keeps
  // the full sweep: its skipping instantiation once came out of the
  // compiler with two tile registers wrong after an unrelated change
  // elsewhere in the function, and that projection is not on the measured
  // path.
  ProjOut o;
  if constexpr (kDyk) {
    o = tm.die ? project_on_chip<kDyk, PolDie, false>(in)
               : project_on_chip<kDyk, PolAgent, false>(in);
  } else {
    const TileGeom g = tile_geom(tm, N);
    const bool part = g.hv <= kTileRows - 16;
    o = tm.die ? (!part ? project_on_chip<kDyk, PolDie, false>(in)
                        : project_on_chip<kDyk, PolDie, true>(in))
               : (!part ? project_on_chip<kDyk, PolAgent, false>(in)
                        : project_on_chip<kDyk, PolAgent, true>(in));
  }
  tm.seq = (unsigned)rfl((int)o.seq);
  *numeric = rfl(o.numeric) != 0;
  const int u = rfl(o.passes);
  info.inner_total += u;
  info.inner_max = max(info.inner_max, u);
  info.inner_capped += rfl(o.capped);
  info.eps2 = __int_as_float(rfl(__float_as_int(o.eps2)));
  return rfl(o.ok) != 0;
}

// --------------------------------------------------------------- the kernel
// kDyk picks the inner projection: false runs Algorithm 1 as printed (plain
// alternation of P1 and P2 in steps 4-7), true the exact projection
// (Dykstra).
template <bool kDyk>
__global__ void __launch_bounds__(kThreads, 1)
fastpfp_persistent(LaunchDesc L) {
  Shared& sh = shm();
  const int tid = threadIdx.x;
  const int pr = tid >> 4, pc = tid & 15;

  // Team membership.  Workgroup b runs on XCD b % 8; numbering the grid XCD
  // by XCD keeps a team of W <= cpx (compute units per XCD) on one die.
  const int cpx = L.cus_per_xcd, b = blockIdx.x;
  const int slot = b / (kXcds * cpx);
  const int v = slot * kXcds * cpx + (b % kXcds) * cpx + (b / kXcds) % cpx;
  int gi = -1;
#pragma unroll
  for (int k = 0; k < kMaxGroups; ++k)
    if (k < L.num_groups && v >= L.group[k].v_begin &&
        v < L.group[k].v_begin + L.group[k].num_teams * L.group[k].W)
      gi = k;
  if (gi < 0) return;
  const TeamGroup grp = L.group[gi];
  Team tm;
  tm.W = grp.W;
  tm.team = grp.team_base + (v - grp.v_begin) / grp.W;
  tm.rank = (v - grp.v_begin) % grp.W;
  tm.TR = grp.TR;
  tm.TC = grp.TC;
  tm.tr = tm.rank / grp.TC;
  tm.tc = tm.rank % grp.TC;
  tm.xb = L.xbuf + (long long)tm.team * L.xbuf_stride;
  tm.par_words = L.xbuf_stride / 2;
  tm.seq = 0;
  tm.die = 0;
  tm.abort_flag = L.queue;
  tm.timeout = L.timeout_ticks;
  float* const Tt = L.wsT + (long long)tm.team * L.wsT_stride;
  float* const Yws = L.wsY + (long long)tm.team * L.wsY_stride;
  uint16_t* const Hws = L.wsH + (long long)tm.team * L.wsH_stride;

  for (;;) {
    // ---- next pair: the team leader takes it from the queue and posts it
    if (tm.rank == 0 && tid == 0)
      sh.wred[0] = __uint_as_float(grp.pair_begin +
                                   atomicAdd(L.queue + 1 + gi, 1u));
    __syncthreads();
    {
      // with it, each workgroup posts the XCD it runs on (hardware register
      // XCC_ID, bits 3:0)
      const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20);
      const float post[kScal] = {sh.wred[0], __uint_as_float(xcc), 0.f, 0.f};
      if (!xchg_scalars(tm, sh, post)) return;
    }
    const unsigned pidx =
        __builtin_amdgcn_readfirstlane(__float_as_uint(sh.scal[0][0]));
    if (pidx >= (unsigned)grp.pair_end) return;
    {
      // a team on one XCD exchanges its pass sums through that XCD's L2
      int same = 1;
      for (int w = 1; w < tm.W; ++w)
        same &= __float_as_uint(sh.scal[w][1]) == __float_as_uint(sh.scal[0][1]);
      tm.die = __builtin_amdgcn_readfirstlane(same && L.die_exchange);
    }
    const PairDesc& pd = L.pairs[pidx];
    const int n = pd.n, np = pd.np, N = pd.N;
    float* const Y = pd.Y ? pd.Y : Yws;
    const TileGeom g = tile_geom(tm, N);
    DevInfo info = {0, 0, 0, 0, 0, 0, 0.f, 0.f, 0ull, 0ull, 0ull};
    const unsigned long long t_pair = wall_clock64();
    float Yr[kRegRows][kCB];

    if (pd.mode == kModeProject) {
      bool numeric = false;
      if (!project_team<kDyk>(tm, Y, N, pd.max_inner, pd.tol_in, true, info,
                              &numeric))
        return;
      info.t_proj = wall_clock64() - t_pair;
      info.status = numeric ? 5 : 0;
    } else {
      float* const X = pd.X;
      const int ldx = pd.ldx;
      // Entries of the tile inside the n x n' block: tile-local rows
      // li < rmax, columns lj < cmax.
      const int rmax_ = min(g.hv, n - g.r0), cmax_ = min(g.wv, np - g.c0);
      // ---- initialisation (Algorithm 1, step 1): X0 and the slack
      {
        const int hv = opaque(g.hv), wv = opaque(g.wv);
        const int rmax = opaque(rmax_), cmax = opaque(cmax_);
        const float c0 = pd.init_c;
        const bool init_x = !pd.init_user, zero_y = !pd.y_user;
#pragma unroll
        for (int a = 0; a < kRA; ++a) {
          const int li = pr + 16 * a;
          if (li < hv) {
            const auto xrow = gbl(X + (long long)(g.r0 + li) * ldx + g.c0 + pc);
            const auto yrow = gbl(Y + (long long)(g.r0 + li) * N + g.c0 + pc);
#pragma unroll
            for (int bb = 0; bb < kCB; ++bb) {
              const int lj = pc + 16 * bb;
              if (lj < wv) {
                if (li < rmax && lj < cmax) {
                  if (init_x) xrow[16 * bb] = c0;
                } else if (zero_y) {
                  yrow[16 * bb] = 0.f;
                }
              }
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      // BF16 products: zero-padded shadows A_h, B_h (converted once per
      // pair) and X^T_h (the transposed iterate), each Np x Np
      const bool bf = pd.precision == 1;
      const int Np = (N + kGT - 1) / kGT * kGT;
      const long long Np2 = (long long)Np * Np;
      uint16_t* const Ah = Hws;
      uint16_t* const Bh = Hws + Np2;
      uint16_t* const Xh = Hws + 2 * Np2;
      uint16_t* const Th = Hws + 3 * Np2;
      if (bf) {
        const float c0 = pd.init_c;
        const bool user = pd.init_user;
        for (long long e = (long long)tm.rank * kThreads + tid; e < Np2;
             e += (long long)tm.W * kThreads) {
          const int r = (int)(e / Np), c = (int)(e % Np);
          gbl(Ah)[e] =
              (r < n && c < n) ? f2bf(gbl(pd.A)[(long long)r * pd.lda + c]) : 0;
          gbl(Bh)[e] =
              (r < np && c < np) ? f2bf(gbl(pd.B)[(long long)r * pd.ldb + c]) : 0;
          gbl(Xh)[e] = (r < np && c < n)
                           ? f2bf(user ? gbl(X)[(long long)c * ldx + r] : c0)
                           : 0;
        }
      }
      if (!team_sync_bulk(tm, sh)) return;
      const int Mt = (n + kGT - 1) / kGT * kGT, Nt = (np + kGT - 1) / kGT * kGT;
      for (int t = 1; t <= pd.max_outer; ++t) {
        // ---- step 3: Y[:n,:np] = A X B + lam K.  FP32: T^T = X^T A (np x n)
        // then T B; BF16: T = A X from the shadows, then T B.
        const unsigned long long t_step = wall_clock64();
        {
          const int NN = N, nn = n, npp = np;
          float* const Yw = Y;
          // Y = (step * (A X B + lam K) + w X): w = 0, step = 1 for FastPFP;
          // w = 1 and the step of eq. (pg) for Projected Gradient.  The
          // epilogue has no branches on these (inside the out-of-line product
          // they are per-lane values, and a branch there made every store
          // wait): without K its loads read X with lam = 0, and a FastPFP
          // pair reads the K source a second time with w = 0.
          const bool pg = pd.pg_step != 0.f;
          const float* const Ks = pd.K ? pd.K : X;
          const int ldks = pd.K ? pd.ldk : ldx;
          const float lam = pd.K ? pd.lam : 0.f;
          const float* const Xs = pg ? X : Ks;
          const int ldxs = pg ? ldx : ldks;
          const float wx = pg ? 1.f : 0.f, step = pg ? pd.pg_step : 1.f;
          // K and X loaded for a whole block before its stores, from
          // positions clamped into the n x n' block (results outside it are
          // not stored), with no arithmetic on them until all are issued
          auto out_pre = [=](int m, int c) {
            const long long mc = min(m, nn - 1), cl = min(c, npp - 1);
            return make_float2(gbl(Ks)[mc * ldks + cl], gbl(Xs)[mc * ldxs + cl]);
          };
          auto out_fin = [=](float val, float2 ad) {
            return wx * ad.y + step * (val + lam * ad.x);
          };
          auto out = [=](int m, int c, float yv) {
            if (m < nn && c < npp) gbl(Yw)[(long long)m * NN + c] = yv;
          };
          auto no_pre = [](int, int) { return make_float2(0.f, 0.f); };
          auto same = [](float val, float2) { return val; };
          if (bf) {
            const int ld = Np;
            auto put_t = [=](int m, int c, float val) {
              gbl(Th)[(long long)m * ld + c] = f2bf(val);
            };
            const int K1 = (n + kBK - 1) / kBK * kBK;
            const int K2 = (np + kBK - 1) / kBK * kBK;
            // T = A X in 128 x 256 output tiles where the columns divide
            // into them.  The second product keeps 128 x 128 tiles: built
            // wide, it came out of the compiler using every register without
            // saving any, so this kernel kept its own values in scratch
            // around the call and the update phase took twice as long; the
            // first product saves what it uses, and with it alone wide the
            // two products together ran 20% faster.
            if (Nt % 256 == 0)
              team_gemm_bf16<256>(Ah, Xh, Np, Mt, Nt, K1, tm, sh, no_pre, same,
                                  put_t);
            else
              team_gemm_bf16<kGT>(Ah, Xh, Np, Mt, Nt, K1, tm, sh, no_pre, same,
                                  put_t);
            if (!team_sync_bulk(tm, sh)) return;
            team_gemm_bf16<kGT>(Th, Bh, Np, Mt, Nt, K2, tm, sh, out_pre,
                                out_fin, out);
          } else {
            float* const Tw = Tt;
            team_gemm_f32(X, ldx, pd.A, pd.lda, np, n, n, tm, sh, no_pre, same,
                          [=](int m, int c, float val) {
                            gbl(Tw)[(long long)m * nn + c] = val;
                          });
            if (!team_sync_bulk(tm, sh)) return;
            team_gemm_f32(Tt, n, pd.B, pd.ldb, n, np, np, tm, sh, out_pre,
                          out_fin, out);
          }
        }
        if (!team_sync_bulk(tm, sh)) return;
        const unsigned long long t_gemm_end = wall_clock64();
        info.t_gemm += t_gemm_end - t_step;
        // ---- steps 4-7, then the projected tile back for steps 8-9
        bool numeric = false;
        if (!project_team<kDyk>(tm, Y, N, pd.max_inner, pd.tol_in, false, info,
                                &numeric))
          return;
        info.t_proj += wall_clock64() - t_gemm_end;
        if (numeric) {
          info.status = 5;
          break;
        }
        load_tile(Yr, sh, Y, N, g, pr, pc);
        // ---- step 8: X_new = (1 - alpha) X + alpha Y[:n,:np], kept in the
        // tile's storage
        const float alpha = pd.alpha, beta = 1.f - pd.alpha;
        float mloc = 0.f;
        // X of tile row a + 1 is loaded while row a is updated, so each
        // row's loads are in flight behind the previous row's arithmetic
        {
          const int rmax = opaque(rmax_), cmax = opaque(cmax_);
          float xa[kCB], xb[kCB];
          auto load_xrow = [&](int a, float (&dst)[kCB]) {
            const int li = pr + 16 * a;
            const auto xrow = gbl(X + (long long)(g.r0 + li) * ldx + g.c0 + pc);
#pragma unroll
            for (int bb = 0; bb < kCB; ++bb)
              dst[bb] = (li < rmax && pc + 16 * bb < cmax) ? xrow[16 * bb]
                                                           : 0.f;
          };
          load_xrow(0, xa);
#pragma unroll
          for (int a = 0; a < kRA; ++a) {
            float(&cur)[kCB] = (a & 1) ? xb : xa;
            float(&nxt)[kCB] = (a & 1) ? xa : xb;
            if (a + 1 < kRA) load_xrow(a + 1, nxt);
            const int li = pr + 16 * a;
            if (li < rmax) {
#pragma unroll
              for (int bb = 0; bb < kCB; ++bb)
                if (pc + 16 * bb < cmax) {
                  const float y = (a < kRegRows) ? Yr[a][bb] : FPFP_LY(a, bb);
                  const float xn = beta * cur[bb] + alpha * y;
                  if (a < kRegRows) Yr[a][bb] = xn;
                  else FPFP_LY(a, bb) = xn;
                  mloc = fmaxf(mloc, xn);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        // ---- step 9: m = max X_new over the team, X = X_new / m
        {
          const float post[kScal] = {wg_max(sh, mloc), 0.f, 0.f, 0.f};
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
        // eps1 = max|X_new / m - X| first, reading the previous X with the
        // same one-row lookahead as step 8; then X = X_new / m is written by
        // a store-only sweep, which has no loads to wait on
        {
          const int rmax = opaque(rmax_), cmax = opaque(cmax_);
          float xa[kCB], xb[kCB];
          auto load_xrow = [&](int a, float (&dst)[kCB]) {
            const int li = pr + 16 * a;
            const auto xrow = gbl(X + (long long)(g.r0 + li) * ldx + g.c0 + pc);
#pragma unroll
            for (int bb = 0; bb < kCB; ++bb)
              dst[bb] = (li < rmax && pc + 16 * bb < cmax) ? xrow[16 * bb]
                                                           : 0.f;
          };
          load_xrow(0, xa);
#pragma unroll
          for (int a = 0; a < kRA; ++a) {
            float(&cur)[kCB] = (a & 1) ? xb : xa;
            float(&nxt)[kCB] = (a & 1) ? xa : xb;
            if (a + 1 < kRA) load_xrow(a + 1, nxt);
            const int li = pr + 16 * a;
            if (li < rmax) {
#pragma unroll
              for (int bb = 0; bb < kCB; ++bb)
                if (pc + 16 * bb < cmax) {
                  const float xn = (a < kRegRows) ? Yr[a][bb] : FPFP_LY(a, bb);
                  const float xv = norm ? xn / m : xn;
                  eloc = fmaxf(eloc, fabsf(xv - cur[bb]));
                }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        {
          const int rmax = opaque(rmax_), cmax = opaque(cmax_);
#pragma unroll
          for (int a = 0; a < kRA; ++a) {
            const int li = pr + 16 * a;
            if (li < rmax) {
              const auto xrow = gbl(X + (long long)(g.r0 + li) * ldx + g.c0 + pc);
#pragma unroll
              for (int bb = 0; bb < kCB; ++bb)
                if (pc + 16 * bb < cmax) {
                  const float xn = (a < kRegRows) ? Yr[a][bb] : FPFP_LY(a, bb);
                  const float xv = norm ? xn / m : xn;
                  xrow[16 * bb] = xv;
                  if (bf)
                    gbl(Xh)[(long long)(g.c0 + pc + 16 * bb) * Np + g.r0 + li] =
                        f2bf(xv);
                }
            }
            // one row of divisions at a time keeps register use bounded
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        {
          const float post[kScal] = {wg_max(sh, eloc), 0.f, 0.f, 0.f};
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
    info.t_all = wall_clock64() - t_pair;
    if (tm.rank == 0 && tid == 0) *pd.info = info;
  }
}

// This source is compiled twice (see the build script): without
// FPFP_DYKSTRA_BUILD it holds the alternating kernel and its launch helpers,
// with it the Dykstra kernel and helpers suffixed _dykstra.
#ifdef FPFP_DYKSTRA_BUILD
constexpr bool kThisDyk = true;
#define FPFP_ENTRY(name) name##_dykstra
#else
constexpr bool kThisDyk = false;
#define FPFP_ENTRY(name) name
#endif

template __global__ void fastpfp_persistent<kThisDyk>(LaunchDesc);

}  // namespace fpfp

// Launch helper with C linkage for the host translation unit.
extern "C" hipError_t FPFP_ENTRY(fpfp_launch_persistent)(
    const fpfp::LaunchDesc* L, int grid, hipStream_t stream) {
  void* args[] = {const_cast<fpfp::LaunchDesc*>(L)};
  return hipLaunchCooperativeKernel(
      (const void*)fpfp::fastpfp_persistent<fpfp::kThisDyk>, dim3(grid),
      dim3(fpfp::kThreads), args, 0, stream);
}

extern "C" hipError_t FPFP_ENTRY(fpfp_occupancy)(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, (const void*)fpfp::fastpfp_persistent<fpfp::kThisDyk>,
      fpfp::kThreads, 0);
}
