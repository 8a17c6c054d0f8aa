// Structures shared by the host API (fastpfp_api.cpp) and the device code
// (fastpfp_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>

namespace fpfp {

// Threads per workgroup and the projection tile: thread (pr, pc) of the
// 16 x 16 thread grid owns tile rows pr + 16a (a < kRA) and columns
// pc + 16b (b < kCB); rows a < kRegRows live in registers, the others in
// LDS.  One workgroup's tile of the slacked matrix is at most
// kTileRows x kTileCols.
constexpr int kThreads = 256;
constexpr int kRA = 16;
constexpr int kCB = 16;
constexpr int kRegRows = 8;
constexpr int kTileRows = 16 * kRA;  // 256
constexpr int kTileCols = 16 * kCB;  // 256
constexpr int kScal = 4;             // scalars each workgroup posts per exchange
constexpr int kXcds = 8;             // MI355X: 8 accelerator complex dies
constexpr int kMaxTeamSide = 16;     // tile rows / columns per team, each
constexpr int kMaxTeam = kMaxTeamSide * kMaxTeamSide;

enum PairMode { kModeSolve = 0, kModeProject = 1 };

// Per-pair result.  t_gemm / t_proj / t_all: the team's wall-clock ticks
// (s_memrealtime, constant rate) spent in step 3 (both products and their
// team barriers), in steps 4-7 (tile load and inner loop), and on the whole
// pair, as seen by the team leader.
struct DevInfo {
  int outer, inner_total, inner_max, inner_capped, converged, status;
  float eps1, eps2;
  unsigned long long t_gemm, t_proj, t_all;
};

// One matching problem as the persistent kernel sees it.
struct PairDesc {
  const float* A;  // n x n, row pitch lda
  const float* B;  // np x np, row pitch ldb
  const float* K;  // n x np, row pitch ldk, or null when lam == 0
  float* X;        // n x np, row pitch ldx: X0 in, final X out
  float* Y;        // N x N state (row pitch N); null -> team workspace
  float* trace;    // eps1 per outer step (max_outer floats) or null
  DevInfo* info;
  int n, np, N, lda, ldb, ldk, ldx;
  int mode, init_user, y_user, normalize, max_outer, max_inner, precision;
  float lam, alpha, tol_out, tol_in, init_c;
  float pg_step;   // Projected Gradient step (eq. pg); 0 for FastPFP
};

// Teams of one size within a launch.  Pairs pairs[pair_begin, pair_end) are
// served by num_teams teams of W workgroups, each team a TR x TC grid of
// projection tiles; the group's workgroups are virtual indices
// [v_begin, v_begin + num_teams * W) and its teams are numbered from
// team_base.
constexpr int kMaxGroups = 5;
struct TeamGroup {
  int W, TR, TC, num_teams, v_begin, team_base, pair_begin, pair_end;
};

// One persistent launch: up to kMaxGroups team groups pulling pairs from
// per-group queues.  Per-team workspaces all have the same strides.
struct LaunchDesc {
  const PairDesc* pairs;
  int num_pairs;
  int num_groups;
  TeamGroup group[kMaxGroups];
  int max_N;                  // largest N in the launch (workspace sizing)
  int cus_per_xcd;            // compute units per XCD (team placement)
  uint64_t* xbuf;             // exchange words, per team
  long long xbuf_stride;      // u64 words per team
  float* wsT;                 // per team: T^T scratch (max np x n)
  long long wsT_stride;
  float* wsY;                 // per team: slacked Y (max N x N)
  long long wsY_stride;
  uint16_t* wsH;              // per team, BF16 products only: A, B, X^T, T
  long long wsH_stride;       // shadows, each Np x Np (Np = N rounded to 128)
  unsigned* queue;            // [0]: abort flag; [1 + g]: group g's next pair
  long long timeout_ticks;    // wall-clock ticks a wait may last
  int die_exchange;           // teams found on one XCD post through its L2
};

// Exchange layout for one team and one parity buffer (u64 words):
//   rowp[TC][NPR], colp[TR][NPC], scal[W][kScal]
__host__ __device__ inline long long xbuf_words_per_parity(int TR, int TC,
                                                          int W, int maxN) {
  long long h = (maxN + TR - 1) / TR, w = (maxN + TC - 1) / TC;
  return (long long)TC * (TR * h) + (long long)TR * (TC * w) +
         (long long)W * kScal;
}

}  // namespace fpfp
