// Host side of the FastPFP C ABI: validation, team planning, workspace, and
// the launch of the persistent kernel (fastpfp_kernels.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <queue>
#include <vector>

#include "fastpfp.h"
#include "fastpfp_ctx.h"
#include "fastpfp_internal.h"

// The solver kernel in two builds: the alternating inner projection of
// Algorithm 1 and the exact (Dykstra) one.
extern "C" hipError_t fpfp_launch_persistent(const fpfp::LaunchDesc* L,
                                             int grid, hipStream_t stream);
extern "C" hipError_t fpfp_occupancy(int* blocks_per_cu);
extern "C" hipError_t fpfp_launch_persistent_dykstra(const fpfp::LaunchDesc* L,
                                                     int grid,
                                                     hipStream_t stream);
extern "C" hipError_t fpfp_occupancy_dykstra(int* blocks_per_cu);
// The fixed scratch of fastpfp_solve_noalloc (noalloc.hip).
extern "C" hipError_t fpfp_noalloc_scratch(int device, void** ptr,
                                           size_t* bytes);
extern "C" hipError_t fpfp_noalloc_prepare(const fpfp::PairDesc* d, void* dst,
                                           void* zero, size_t bytes,
                                           hipStream_t stream);

namespace {

using fpfp::fail;

struct Plan {
  int W, TR, TC;
};

// The tile grid of a team depends on its size W (a power of two) only:
// TR = 2^ceil(log2(W)/2) tile rows by TC = W / TR tile columns, so a pair is
// cut into the same tiles -- and computed with the same rounding -- whether it
// is solved alone or in a batch with the same W.  The grid fits N when every
// tile fits the register tile (kTileRows x kTileCols).
void grid_for(int W, Plan* pl) {
  int lg = 0;
  while ((1 << lg) < W) ++lg;
  pl->W = W;
  pl->TR = 1 << ((lg + 1) / 2);
  pl->TC = W / pl->TR;
}

bool grid_fits(const Plan& pl, int N) {
  return pl.TR <= fpfp::kMaxTeamSide && pl.TC <= fpfp::kMaxTeamSide &&
         (N + pl.TR - 1) / pl.TR <= fpfp::kTileRows &&
         (N + pl.TC - 1) / pl.TC <= fpfp::kTileCols;
}

// want > 0: that team size (must be a power of two that fits N);
// want == 0: the smallest power of two that fits N.
bool plan_team(int N, int want, Plan* pl) {
  if (want > 0) {
    if ((want & (want - 1)) != 0) return false;
    grid_for(want, pl);
    return grid_fits(*pl, N);
  }
  for (int W = 1; W <= fpfp::kMaxTeamSide * fpfp::kMaxTeamSide; W *= 2) {
    grid_for(W, pl);
    if (grid_fits(*pl, N)) return true;
  }
  return false;
}

fastpfp_status check_params(fastpfp_t h, const fastpfp_params* p) {
  if (!p) return fail(h, FASTPFP_ERR_INVALID_ARG, "params is NULL");
  if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "lambda must be finite and >= 0");
  if (p->method != FASTPFP_METHOD_FASTPFP && p->method != FASTPFP_METHOD_PG)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "unknown method %d", p->method);
  if (p->method == FASTPFP_METHOD_FASTPFP && !(p->alpha > 0.0 && p->alpha <= 1.0))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "alpha must lie in (0, 1]");
  if (p->method == FASTPFP_METHOD_PG &&
      !(p->alpha > 0.0 && std::isfinite(p->alpha)))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "the PG step must be finite and > 0");
  if (!(p->tol_outer > 0.0) || !std::isfinite(p->tol_outer) ||
      !(p->tol_inner > 0.0) || !std::isfinite(p->tol_inner))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "tolerances must be finite and > 0");
  if (p->max_outer < 1 || p->max_inner < 1)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "iteration caps must be >= 1");
  if (p->precision != FASTPFP_FP32 && p->precision != FASTPFP_BF16)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "unknown precision %d", p->precision);
  if (p->init != FASTPFP_INIT_UNIFORM && p->init != FASTPFP_INIT_USER)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "unknown init %d", p->init);
  if (!(p->init_scale >= 0.0) || !std::isfinite(p->init_scale))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "init_scale must be finite and >= 0");
  if (p->team_size < 0)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "team_size must be >= 0");
  if (p->projection != FASTPFP_PROJ_ALTERNATING &&
      p->projection != FASTPFP_PROJ_DYKSTRA)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "unknown projection %d",
                p->projection);
  return FASTPFP_OK;
}

// Workspace layout of one launch, in bytes from the workspace base.
struct Layout {
  size_t pairs, infos, queue, trace, xbuf, wsT, wsY, wsH, total;
  long long xbuf_stride, wsT_stride, wsY_stride, wsH_stride;
};

Layout layout_for(int num_pairs, int num_teams, long long xwords, int maxN,
                  int max_nnp, int max_outer, bool need_y, bool need_trace,
                  bool need_bf16, int num_groups) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  Layout L{};
  size_t o = 0;
  L.pairs = o;
  o = up(o + sizeof(fpfp::PairDesc) * num_pairs);
  L.infos = o;
  o = up(o + sizeof(fpfp::DevInfo) * num_pairs);
  L.queue = o;
  o = up(o + sizeof(unsigned) * (1 + num_groups));
  L.trace = o;
  o = up(o + (need_trace ? sizeof(float) * max_outer : 0));
  L.xbuf_stride = 2 * xwords;
  L.xbuf = o;
  o = up(o + sizeof(uint64_t) * L.xbuf_stride * num_teams);
  L.wsT_stride = ((long long)max_nnp + 63) & ~63LL;
  L.wsT = o;
  o = up(o + sizeof(float) * L.wsT_stride * num_teams);
  L.wsY_stride = need_y ? (((long long)maxN * maxN + 63) & ~63LL) : 0;
  L.wsY = o;
  o = up(o + sizeof(float) * L.wsY_stride * num_teams);
  // BF16 shadows: 4 matrices of Np x Np, Np = maxN rounded up to 128
  const long long Np = (maxN + 127) / 128 * 128;
  L.wsH_stride = need_bf16 ? 4 * Np * Np : 0;
  L.wsH = o;
  o = up(o + sizeof(uint16_t) * L.wsH_stride * num_teams);
  L.total = o;
  return L;
}

fastpfp_status ensure_ws(fastpfp_t h, size_t bytes) {
  if (bytes <= h->ws_bytes) return FASTPFP_OK;
  if (h->ws) {
    (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t want = std::max(bytes, size_t(1) << 20);
  if (hipMalloc(&h->ws, want) != hipSuccess) {
    h->ws = nullptr;
    return fail(h, FASTPFP_ERR_NOMEM, "cannot allocate %zu bytes of workspace",
                want);
  }
  h->ws_bytes = want;
  return FASTPFP_OK;
}

struct PairIn {
  int n, np;
  const float *A, *B, *K;
  float* X;
  float* Y;
  int lda, ldb, ldk, ldx;
};

// The device descriptor of one pair.
void fill_pair(fpfp::PairDesc* dp, const PairIn& q, const fastpfp_params* p,
               int mode, int max_inner, double tol_in, float* trace,
               fpfp::DevInfo* info) {
  fpfp::PairDesc& d = *dp;
  std::memset(&d, 0, sizeof d);
  d.A = q.A;
  d.B = q.B;
  d.K = (p && p->lambda > 0.0) ? q.K : nullptr;
  d.X = q.X;
  d.Y = q.Y;
  d.trace = trace;
  d.info = info;
  d.n = q.n;
  d.np = q.np;
  d.N = std::max(q.n, q.np);
  d.lda = q.lda;
  d.ldb = q.ldb;
  d.ldk = q.ldk;
  d.ldx = q.ldx;
  d.mode = mode;
  d.max_inner = max_inner;
  d.tol_in = (float)tol_in;
  if (mode == fpfp::kModeSolve) {
    d.init_user = p->init == FASTPFP_INIT_USER;
    d.y_user = q.Y != nullptr;
    d.normalize = p->normalize_max != 0;
    d.max_outer = p->max_outer;
    d.precision = p->precision;
    d.lam = (float)p->lambda;
    // Projected Gradient: step 3 forms X + alpha * gradient and step 8
    // takes the projection undamped
    const bool pg = p->method == FASTPFP_METHOD_PG;
    d.alpha = pg ? 1.0f : (float)p->alpha;
    d.pg_step = pg ? (float)p->alpha : 0.0f;
    d.tol_out = (float)p->tol_outer;
    d.init_c = (float)(p->init_scale > 0.0 ? p->init_scale
                                           : 1.0 / (double)d.N);
  } else {
    d.y_user = 1;
  }
}

// Modelled time (microseconds) of one inner pass of a team of W workgroups
// (TR tile rows) on an N x N matrix: a fixed part -- the workgroup's
// reductions, and for W > 1 the team exchange -- plus the sweep over the
// tile rows that hold entries (the sweep skips padding rows).  Fitted to
// passes measured on MI355X at W = 1, 4 and 16 and N = 16 ... 1000; used only
// to divide a mixed batch's workgroups between its team sizes.
double pass_cost(int W, int TR, int N) {
  const int h = (N + TR - 1) / TR;
  const int rows = (std::min(h, fpfp::kTileRows) + 15) / 16;
  return (W == 1 ? 1.6 : 4.2) + 3.0 * rows / 16.0;
}

// Time until the last of `costs` (sorted largest first) is done when
// `teams` teams take them from one queue in that order.
double lpt_makespan(const std::vector<double>& costs, int teams) {
  std::priority_queue<double, std::vector<double>, std::greater<double>> q;
  for (int k = 0; k < teams; ++k) q.push(0.0);
  double end = 0.0;
  for (double c : costs) {
    const double t = q.top() + c;
    q.pop();
    q.push(t);
    end = std::max(end, t);
  }
  return end;
}

// The launch descriptor over a workspace at `base` laid out as `lay`.
void fill_launch(fpfp::LaunchDesc* Lp, fastpfp_t h, char* base,
                 const Layout& lay, int P, int NG, const fpfp::TeamGroup* grp,
                 int maxN) {
  fpfp::LaunchDesc& L = *Lp;
  std::memset(&L, 0, sizeof L);
  L.pairs = (const fpfp::PairDesc*)(base + lay.pairs);
  L.num_pairs = P;
  L.num_groups = NG;
  for (int g = 0; g < NG; ++g) L.group[g] = grp[g];
  L.max_N = maxN;
  L.cus_per_xcd = std::max(1, h->cu_count / fpfp::kXcds);
  L.xbuf = (uint64_t*)(base + lay.xbuf);
  L.xbuf_stride = lay.xbuf_stride;
  L.wsT = (float*)(base + lay.wsT);
  L.wsT_stride = lay.wsT_stride;
  L.wsY = (float*)(base + lay.wsY);
  L.wsY_stride = lay.wsY_stride;
  L.wsH = (uint16_t*)(base + lay.wsH);
  L.wsH_stride = lay.wsH_stride;
  L.queue = (unsigned*)(base + lay.queue);
  L.timeout_ticks = 100000000LL * 20;  // 20 s of the 100 MHz wall clock
  L.die_exchange = h->die_exchange;
}

// Copies one pair's device result into the public info struct.
void copy_info(fastpfp_info* o, const fpfp::DevInfo& d, float ms,
               double wall_khz) {
  o->outer_iters = d.outer;
  o->inner_iters_total = d.inner_total;
  o->inner_iters_max = d.inner_max;
  o->inner_capped = d.inner_capped;
  o->converged = d.converged;
  o->status = d.status;
  o->eps1_last = d.eps1;
  o->eps2_last = d.eps2;
  o->kernel_ms = ms;
  o->gemm_ms = (double)d.t_gemm / wall_khz;
  o->proj_ms = (double)d.t_proj / wall_khz;
  o->pair_ms = (double)d.t_all / wall_khz;
}

// Usable workgroups of one cooperative launch (a multiple of the XCD count).
int launch_grid(fastpfp_t h) {
  int G = std::min(512, h->occupancy * h->cu_count);
  return G - G % fpfp::kXcds;
}

// Plans, launches and waits for one persistent launch over `pairs`.
fastpfp_status run(fastpfp_t h, const std::vector<PairIn>& pairs,
                   const fastpfp_params* p, int mode, int max_inner,
                   double tol_in, int projection, int team_req, bool want_trace,
                   fastpfp_info* infos) {
  HIPCHK(h, hipSetDevice(h->device));
  // ---- team groups: each pair gets the smallest team whose tiles fit it
  // (or the requested team size); one group per distinct size, largest first
  const int P = (int)pairs.size();
  std::vector<Plan> pplan(P);
  for (int b = 0; b < P; ++b) {
    const int Nb = std::max(pairs[b].n, pairs[b].np);
    if (!plan_team(Nb, team_req, &pplan[b])) {
      if (team_req == 0)
        return fail(h, FASTPFP_ERR_UNSUPPORTED,
                    "N = %d exceeds the largest team's tiles (%d x %d)", Nb,
                    fpfp::kMaxTeamSide * fpfp::kTileRows,
                    fpfp::kMaxTeamSide * fpfp::kTileCols);
      return fail(h, FASTPFP_ERR_INVALID_ARG,
                  "team_size %d is not a power of two whose tiles fit N = %d",
                  team_req, Nb);
    }
  }
  const int G = launch_grid(h);
  std::vector<int> sizes;
  for (auto& q : pplan)
    if (std::find(sizes.begin(), sizes.end(), q.W) == sizes.end())
      sizes.push_back(q.W);
  std::sort(sizes.rbegin(), sizes.rend());
  if ((int)sizes.size() > fpfp::kMaxGroups)
    return fail(h, FASTPFP_ERR_UNSUPPORTED, "too many team sizes in a batch");
  const int NG = (int)sizes.size();
  std::vector<std::vector<int>> members(NG);
  std::vector<std::vector<double>> cost(NG);
  for (int b = 0; b < P; ++b) {
    const int g = (int)(std::find(sizes.begin(), sizes.end(), pplan[b].W) -
                        sizes.begin());
    members[g].push_back(b);
    cost[g].push_back(pass_cost(pplan[b].W, pplan[b].TR,
                                std::max(pairs[b].n, pairs[b].np)));
  }
  for (auto& c : cost) std::sort(c.rbegin(), c.rend());
  int need = 0;
  for (int g = 0; g < NG; ++g) need += sizes[g];
  if (need > G)
    return fail(h, FASTPFP_ERR_UNSUPPORTED,
                "a batch needs %d co-resident workgroups; %d fit", need, G);
  // One team per group to start with; then, while workgroups are free, one
  // more team for the group whose pairs (modelled pass costs, taken from its
  // queue largest first) would finish last, as long as it has a pair for the
  // team.  A group that cannot grow any more ends the search, since the
  // batch cannot finish before it.
  std::vector<int> teams(NG, 1);
  std::vector<double> span(NG);
  int used = need;
  for (int g = 0; g < NG; ++g) span[g] = lpt_makespan(cost[g], 1);
  for (;;) {
    int worst = 0;
    for (int g = 1; g < NG; ++g)
      if (span[g] > span[worst]) worst = g;
    if (used + sizes[worst] > G || teams[worst] >= (int)members[worst].size())
      break;
    teams[worst]++;
    used += sizes[worst];
    span[worst] = lpt_makespan(cost[worst], teams[worst]);
  }
  for (bool grew = true; grew;) {  // hand out what is left
    grew = false;
    for (int g = 0; g < NG; ++g)
      if (used + sizes[g] <= G && teams[g] < (int)members[g].size()) {
        teams[g]++;
        used += sizes[g];
        grew = true;
      }
  }
  // pairs in group order, largest first within a group
  std::vector<int> order;
  std::vector<fpfp::TeamGroup> grp(NG);
  int v = 0, tb = 0;
  long long xwords = 0;
  int maxN = 1, max_nnp = 1;
  for (int g = 0; g < NG; ++g) {
    auto& mem = members[g];
    std::stable_sort(mem.begin(), mem.end(), [&](int x, int y) {
      return std::max(pairs[x].n, pairs[x].np) > std::max(pairs[y].n, pairs[y].np);
    });
    Plan pl;
    grid_for(sizes[g], &pl);
    grp[g].W = pl.W;
    grp[g].TR = pl.TR;
    grp[g].TC = pl.TC;
    grp[g].num_teams = teams[g];
    grp[g].v_begin = v;
    grp[g].team_base = tb;
    grp[g].pair_begin = (int)order.size();
    int gmaxN = 1;
    for (int b : mem) {
      order.push_back(b);
      gmaxN = std::max(gmaxN, std::max(pairs[b].n, pairs[b].np));
      max_nnp = std::max(max_nnp, pairs[b].n * pairs[b].np);
    }
    grp[g].pair_end = (int)order.size();
    maxN = std::max(maxN, gmaxN);
    xwords = std::max(xwords, fpfp::xbuf_words_per_parity(pl.TR, pl.TC, pl.W, gmaxN));
    v += teams[g] * pl.W;
    tb += teams[g];
  }
  const int num_teams = tb;
  bool need_y = false;
  for (auto& q : pairs) need_y |= (q.Y == nullptr);
  const int max_outer = mode == fpfp::kModeSolve ? p->max_outer : 1;
  const bool need_bf16 = mode == fpfp::kModeSolve &&
                         p->precision == FASTPFP_BF16;
  Layout lay = layout_for(P, num_teams, xwords, maxN, max_nnp, max_outer,
                          need_y, want_trace, need_bf16, NG);
  fastpfp_status st = ensure_ws(h, lay.total);
  if (st != FASTPFP_OK) return st;
  char* base = (char*)h->ws;

  std::vector<fpfp::PairDesc> pd(P);
  for (int k = 0; k < P; ++k) {
    const int b = order[k];
    fill_pair(&pd[k], pairs[b], p, mode, max_inner, tol_in,
              (want_trace && b == 0) ? (float*)(base + lay.trace) : nullptr,
              (fpfp::DevInfo*)(base + lay.infos) + b);
  }
  fpfp::LaunchDesc L;
  fill_launch(&L, h, base, lay, P, NG, grp.data(), maxN);

  HIPCHK(h, hipMemcpyAsync(base + lay.pairs, pd.data(),
                           sizeof(fpfp::PairDesc) * pd.size(),
                           hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemsetAsync(base + lay.queue, 0,
                           sizeof(unsigned) * (1 + NG), h->stream));
  HIPCHK(h, hipMemsetAsync(base + lay.infos, 0,
                           sizeof(fpfp::DevInfo) * pd.size(), h->stream));
  HIPCHK(h, hipMemsetAsync(base + lay.xbuf, 0,
                           sizeof(uint64_t) * lay.xbuf_stride * num_teams,
                           h->stream));
  HIPCHK(h, hipEventRecord(h->ev0, h->stream));
  HIPCHK(h, projection == FASTPFP_PROJ_DYKSTRA
                ? fpfp_launch_persistent_dykstra(&L, G, h->stream)
                : fpfp_launch_persistent(&L, G, h->stream));
  HIPCHK(h, hipEventRecord(h->ev1, h->stream));
  std::vector<fpfp::DevInfo> di(pd.size());
  unsigned abort_flag = 0;
  std::vector<float> tr(want_trace ? max_outer : 0);
  HIPCHK(h, hipMemcpyAsync(di.data(), base + lay.infos,
                           sizeof(fpfp::DevInfo) * di.size(),
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(&abort_flag, base + lay.queue, sizeof abort_flag,
                           hipMemcpyDeviceToHost, h->stream));
  if (want_trace)
    HIPCHK(h, hipMemcpyAsync(tr.data(), base + lay.trace,
                             sizeof(float) * tr.size(), hipMemcpyDeviceToHost,
                             h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  float ms = 0.f;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
  if (abort_flag != 0)
    return fail(h, FASTPFP_ERR_TIMEOUT,
                "a device-side wait exceeded its limit; results are invalid");
  fastpfp_status first = FASTPFP_OK;
  for (size_t b = 0; b < di.size(); ++b) {
    copy_info(&infos[b], di[b], ms, h->wall_khz);
    if (infos[b].status != 0 && first == FASTPFP_OK)
      first = (fastpfp_status)infos[b].status;
  }
  if (want_trace) {
    h->trace.assign(tr.begin(), tr.begin() + std::min<int>(di[0].outer, max_outer));
  }
  if (first != FASTPFP_OK)
    return fail(h, first, "non-finite values met during the solve");
  return FASTPFP_OK;
}

// One pair, one team, with the workspace in the device's fixed scratch
// array instead of the handle's: the same plan, descriptors and kernel as
// run() gives a single pair, and no allocation.  The descriptor is written
// and the counters cleared by a kernel.
fastpfp_status run_noalloc(fastpfp_t h, const PairIn& q,
                           const fastpfp_params* p, fastpfp_info* info) {
  HIPCHK(h, hipSetDevice(h->device));
  void* scratch = nullptr;
  size_t cap = 0;
  HIPCHK(h, fpfp_noalloc_scratch(h->device, &scratch, &cap));
  const int N = std::max(q.n, q.np);
  Plan pl;
  if (!plan_team(N, p->team_size, &pl)) {
    if (p->team_size == 0)
      return fail(h, FASTPFP_ERR_UNSUPPORTED,
                  "N = %d exceeds the largest team's tiles", N);
    return fail(h, FASTPFP_ERR_INVALID_ARG,
                "team_size %d is not a power of two whose tiles fit N = %d",
                p->team_size, N);
  }
  const int G = launch_grid(h);
  if (pl.W > G)
    return fail(h, FASTPFP_ERR_UNSUPPORTED,
                "a team of %d workgroups does not fit the %d co-resident ones",
                pl.W, G);
  fpfp::TeamGroup grp;
  grp.W = pl.W;
  grp.TR = pl.TR;
  grp.TC = pl.TC;
  grp.num_teams = 1;
  grp.v_begin = 0;
  grp.team_base = 0;
  grp.pair_begin = 0;
  grp.pair_end = 1;
  const long long xwords = fpfp::xbuf_words_per_parity(pl.TR, pl.TC, pl.W, N);
  const Layout lay = layout_for(1, 1, xwords, N, q.n * q.np, p->max_outer,
                                q.Y == nullptr, false,
                                p->precision == FASTPFP_BF16, 1);
  if (lay.total > cap)
    return fail(h, FASTPFP_ERR_SHAPE,
                "the solve needs %zu bytes of scratch; the fixed array has %zu",
                lay.total, cap);
  char* base = (char*)scratch;
  fpfp::PairDesc d;
  fill_pair(&d, q, p, fpfp::kModeSolve, p->max_inner, p->tol_inner, nullptr,
            (fpfp::DevInfo*)(base + lay.infos));
  fpfp::LaunchDesc L;
  fill_launch(&L, h, base, lay, 1, 1, &grp, N);
  // per-pair results, queue, (empty) trace and exchange words are
  // contiguous in the layout and all start at zero
  HIPCHK(h, fpfp_noalloc_prepare(&d, base + lay.pairs, base + lay.infos,
                                 lay.wsT - lay.infos, h->stream));
  HIPCHK(h, hipEventRecord(h->ev0, h->stream));
  HIPCHK(h, p->projection == FASTPFP_PROJ_DYKSTRA
                ? fpfp_launch_persistent_dykstra(&L, G, h->stream)
                : fpfp_launch_persistent(&L, G, h->stream));
  HIPCHK(h, hipEventRecord(h->ev1, h->stream));
  fpfp::DevInfo di;
  unsigned abort_flag = 0;
  HIPCHK(h, hipMemcpyAsync(&di, base + lay.infos, sizeof di,
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(&abort_flag, base + lay.queue, sizeof abort_flag,
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  float ms = 0.f;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
  if (abort_flag != 0)
    return fail(h, FASTPFP_ERR_TIMEOUT,
                "a device-side wait exceeded its limit; results are invalid");
  copy_info(info, di, ms, h->wall_khz);
  if (di.status != 0)
    return fail(h, (fastpfp_status)di.status,
                "non-finite values met during the solve");
  return FASTPFP_OK;
}

bool bad_ld(int ld, int cols) { return ld < cols; }

}  // namespace

extern "C" {

int fastpfp_abi_version(void) { return FASTPFP_ABI_VERSION; }

const char* fastpfp_status_string(fastpfp_status s) {
  switch (s) {
    case FASTPFP_OK: return "ok";
    case FASTPFP_ERR_INVALID_ARG: return "invalid argument";
    case FASTPFP_ERR_SHAPE: return "shape out of range";
    case FASTPFP_ERR_HIP: return "HIP runtime error";
    case FASTPFP_ERR_NOMEM: return "out of device memory";
    case FASTPFP_ERR_NUMERIC: return "non-finite values";
    case FASTPFP_ERR_TIMEOUT: return "device wait timed out";
    case FASTPFP_ERR_UNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

const char* fastpfp_last_error(fastpfp_t h) {
  return h ? h->err.c_str() : "NULL handle";
}

fastpfp_status fastpfp_params_default(fastpfp_params* p) {
  if (!p) return FASTPFP_ERR_INVALID_ARG;
  std::memset(p, 0, sizeof *p);
  p->lambda = 0.0;
  p->alpha = 0.5;
  p->tol_outer = 1e-6;
  p->tol_inner = 1e-8;
  p->max_outer = 1000;
  p->max_inner = 1000;
  p->precision = FASTPFP_FP32;
  p->init = FASTPFP_INIT_UNIFORM;
  p->init_scale = 0.0;
  p->normalize_max = 1;
  p->team_size = 0;
  p->projection = FASTPFP_PROJ_ALTERNATING;
  p->method = FASTPFP_METHOD_FASTPFP;
  return FASTPFP_OK;
}

fastpfp_status fastpfp_create(fastpfp_t* out, int device, int max_n,
                              int max_np, void* hip_stream) {
  if (!out) return FASTPFP_ERR_INVALID_ARG;
  *out = nullptr;
  if (max_n < 1 || max_np < 1) return FASTPFP_ERR_SHAPE;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return FASTPFP_ERR_HIP;
  fastpfp_ctx* h = new fastpfp_ctx;
  int occ_dyk = 0;
  h->device = device;
  h->max_n = max_n;
  h->max_np = max_np;
  h->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess ||
      hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount,
                            device) != hipSuccess ||
      fpfp_occupancy(&h->occupancy) != hipSuccess ||
      fpfp_occupancy_dykstra(&occ_dyk) != hipSuccess ||
      hipEventCreate(&h->ev0) != hipSuccess ||
      hipEventCreate(&h->ev1) != hipSuccess) {
    delete h;
    return FASTPFP_ERR_HIP;
  }
  // launches size their grids for the kernel that fits fewer workgroups
  h->occupancy = std::min(h->occupancy, occ_dyk);
  int wall_khz = 0;
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate,
                            device) == hipSuccess && wall_khz > 0)
    h->wall_khz = wall_khz;
  // FASTPFP_EXCHANGE=agent keeps every team's pass exchange at device scope
  const char* xe = std::getenv("FASTPFP_EXCHANGE");
  h->die_exchange = !(xe && std::strcmp(xe, "agent") == 0);
  // the device address of this device's fixed scratch array (looked up once
  // per device, with the device current)
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  if (fpfp_noalloc_scratch(device, &scratch, &scratch_bytes) != hipSuccess) {
    (void)hipEventDestroy(h->ev0);
    (void)hipEventDestroy(h->ev1);
    delete h;
    return FASTPFP_ERR_HIP;
  }
  // the warm start's streams are made with the handle: made later, after
  // the process's first solver launch, they were measured to run one after
  // another instead of side by side
  fpfp::warm_prepare(h);
  *out = h;
  return FASTPFP_OK;
}

fastpfp_status fastpfp_destroy(fastpfp_t h) {
  if (!h) return FASTPFP_ERR_INVALID_ARG;
  (void)hipSetDevice(h->device);
  if (h->ws) (void)hipFree(h->ws);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  if (h->warm) fpfp::warm_free(h->warm);
  if (h->dws) (void)hipFree(h->dws);
  if (h->pws) (void)hipFree(h->pws);
  delete h;
  return FASTPFP_OK;
}

fastpfp_status fastpfp_solve(fastpfp_t h, int n, int np, const float* A,
                             int lda, const float* B, int ldb, const float* K,
                             int ldk, const fastpfp_params* p, float* X,
                             int ldx, float* Y_state, fastpfp_info* info) {
  if (!h) return FASTPFP_ERR_INVALID_ARG;
  fastpfp_status st = check_params(h, p);
  if (st != FASTPFP_OK) return st;
  if (n < 1 || np < 1 || n > h->max_n || np > h->max_np)
    return fail(h, FASTPFP_ERR_SHAPE, "n=%d n'=%d outside [1, %d] x [1, %d]",
                n, np, h->max_n, h->max_np);
  if (!A || !B || !X)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "A, B and X must be non-NULL");
  if (p->lambda > 0.0 && !K)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "K is NULL but lambda > 0");
  if (bad_ld(lda, n) || bad_ld(ldb, np) || bad_ld(ldx, np) ||
      (p->lambda > 0.0 && bad_ld(ldk, np)))
    return fail(h, FASTPFP_ERR_SHAPE, "a leading dimension is too small");
  std::vector<PairIn> pairs(1);
  pairs[0] = PairIn{n, np, A, B, K, X, Y_state, lda, ldb, ldk, ldx};
  fastpfp_info tmp;
  std::memset(&tmp, 0, sizeof tmp);
  st = run(h, pairs, p, fpfp::kModeSolve, p->max_inner, p->tol_inner,
           p->projection,
           p->team_size, true, &tmp);
  if (info) *info = tmp;
  return st;
}

fastpfp_status fastpfp_solve_noalloc(fastpfp_t h, int n, int np,
                                     const float* A, int lda, const float* B,
                                     int ldb, const float* K, int ldk,
                                     const fastpfp_params* p, float* X,
                                     int ldx, float* Y_state,
                                     fastpfp_info* info) {
  if (!h) return FASTPFP_ERR_INVALID_ARG;
  fastpfp_status st = check_params(h, p);
  if (st != FASTPFP_OK) return st;
  if (n < 1 || np < 1 || n > h->max_n || np > h->max_np)
    return fail(h, FASTPFP_ERR_SHAPE, "n=%d n'=%d outside [1, %d] x [1, %d]",
                n, np, h->max_n, h->max_np);
  if (std::max(n, np) > FASTPFP_NOALLOC_MAX_N)
    return fail(h, FASTPFP_ERR_SHAPE,
                "max(n, n') = %d exceeds the allocation-free limit %d",
                std::max(n, np), FASTPFP_NOALLOC_MAX_N);
  if (!A || !B || !X)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "A, B and X must be non-NULL");
  if (p->lambda > 0.0 && !K)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "K is NULL but lambda > 0");
  if (bad_ld(lda, n) || bad_ld(ldb, np) || bad_ld(ldx, np) ||
      (p->lambda > 0.0 && bad_ld(ldk, np)))
    return fail(h, FASTPFP_ERR_SHAPE, "a leading dimension is too small");
  const PairIn q{n, np, A, B, K, X, Y_state, lda, ldb, ldk, ldx};
  fastpfp_info tmp;
  std::memset(&tmp, 0, sizeof tmp);
  st = run_noalloc(h, q, p, &tmp);
  if (info) *info = tmp;
  return st;
}

fastpfp_status fastpfp_solve_batched(fastpfp_t h, int batch, const int* n_host,
                                     const int* np_host, const float* A,
                                     const int64_t* offA_host, const float* B,
                                     const int64_t* offB_host, const float* K,
                                     const int64_t* offK_host,
                                     const fastpfp_params* p, float* X,
                                     const int64_t* offX_host,
                                     fastpfp_info* infos_host) {
  if (!h) return FASTPFP_ERR_INVALID_ARG;
  fastpfp_status st = check_params(h, p);
  if (st != FASTPFP_OK) return st;
  if (batch < 1 || !n_host || !np_host || !A || !offA_host || !B ||
      !offB_host || !X || !offX_host)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "NULL batch argument");
  if (p->lambda > 0.0 && (!K || !offK_host))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "K is NULL but lambda > 0");
  std::vector<PairIn> pairs(batch);
  for (int b = 0; b < batch; ++b) {
    const int n = n_host[b], np = np_host[b];
    if (n < 1 || np < 1 || n > h->max_n || np > h->max_np)
      return fail(h, FASTPFP_ERR_SHAPE, "pair %d: n=%d n'=%d out of range", b,
                  n, np);
    if (offA_host[b] < 0 || offB_host[b] < 0 || offX_host[b] < 0 ||
        (p->lambda > 0.0 && offK_host[b] < 0))
      return fail(h, FASTPFP_ERR_INVALID_ARG, "pair %d: negative offset", b);
    pairs[b] = PairIn{n,
                      np,
                      A + offA_host[b],
                      B + offB_host[b],
                      (p->lambda > 0.0) ? K + offK_host[b] : nullptr,
                      X + offX_host[b],
                      nullptr,
                      n,
                      np,
                      np,
                      np};
  }
  std::vector<fastpfp_info> tmp(batch);
  st = run(h, pairs, p, fpfp::kModeSolve, p->max_inner, p->tol_inner,
           p->projection,
           p->team_size, false, tmp.data());
  if (infos_host) std::memcpy(infos_host, tmp.data(), sizeof(fastpfp_info) * batch);
  return st;
}

fastpfp_status fastpfp_project(fastpfp_t h, int N, float* Y, double tol,
                               int max_inner, int team_size, int projection,
                               fastpfp_info* info) {
  if (!h) return FASTPFP_ERR_INVALID_ARG;
  if (N < 1 || N > std::max(h->max_n, h->max_np))
    return fail(h, FASTPFP_ERR_SHAPE, "N=%d out of range", N);
  if (!Y) return fail(h, FASTPFP_ERR_INVALID_ARG, "Y is NULL");
  if (!(tol > 0.0) || !std::isfinite(tol) || max_inner < 1 || team_size < 0)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "bad tolerance, cap or team size");
  if (projection != FASTPFP_PROJ_ALTERNATING &&
      projection != FASTPFP_PROJ_DYKSTRA)
    return fail(h, FASTPFP_ERR_INVALID_ARG, "unknown projection %d",
                projection);
  // a matrix no team can hold on chip is projected with Y in HBM
  Plan pl;
  if (team_size == 0 && !plan_team(N, 0, &pl))
    return fastpfp_project_stream(h, N, Y, tol, max_inner, projection, info);
  std::vector<PairIn> pairs(1);
  pairs[0] = PairIn{N, N, nullptr, nullptr, nullptr, nullptr, Y, N, N, N, N};
  fastpfp_info tmp;
  std::memset(&tmp, 0, sizeof tmp);
  fastpfp_status st = run(h, pairs, nullptr, fpfp::kModeProject, max_inner,
                          tol, projection, team_size, false, &tmp);
  if (info) *info = tmp;
  return st;
}

fastpfp_status fastpfp_autotune(fastpfp_t h, int N, int batch, int passes,
                                int* team_size_out, int* W_host,
                                double* rate_host, int cap, int* count) {
  if (!h || !team_size_out) return FASTPFP_ERR_INVALID_ARG;
  if (N < 1 || N > std::max(h->max_n, h->max_np))
    return fail(h, FASTPFP_ERR_SHAPE, "N=%d out of range", N);
  if (batch < 1 || passes < 1 || passes > 100000 || cap < 0 ||
      (cap > 0 && (!W_host || !rate_host)))
    return fail(h, FASTPFP_ERR_INVALID_ARG, "bad batch, passes or outputs");
  HIPCHK(h, hipSetDevice(h->device));
  Plan pl;
  if (!plan_team(N, 0, &pl))
    return fail(h, FASTPFP_ERR_UNSUPPORTED, "N=%d fits no team", N);
  const int G = launch_grid(h);
  std::vector<int> cand;
  for (int W = pl.W; W <= std::min(G, fpfp::kMaxTeam); W *= 2) cand.push_back(W);
  if (cand.empty())
    return fail(h, FASTPFP_ERR_UNSUPPORTED, "N=%d needs more workgroups", N);
  // Concurrent projections of a fixed matrix that keeps changing for many
  // passes (entries of both signs), one copy per concurrent pair.
  const int conc_max = std::min(batch, G / cand[0]);
  const size_t NN = (size_t)N * N;
  std::vector<float> pattern(NN);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      pattern[(size_t)i * N + j] =
          (float)((i * 131 + j * 71) % 97) / 97.0f - 0.3f;
  float* Ybuf = nullptr;
  if (hipMalloc((void**)&Ybuf, sizeof(float) * NN * conc_max) != hipSuccess)
    return fail(h, FASTPFP_ERR_NOMEM, "cannot allocate %zu bytes",
                sizeof(float) * NN * conc_max);
  fastpfp_status st = FASTPFP_OK;
  int best = cand[0];
  double best_rate = -1.0;
  int k = 0;
  for (size_t ci = 0; ci < cand.size() && st == FASTPFP_OK; ++ci) {
    const int W = cand[ci], conc = std::min(batch, G / W);
    std::vector<PairIn> pairs(conc);
    std::vector<fastpfp_info> infos(conc);
    double ms = 0.0;
    for (int rep = 0; rep < 2 && st == FASTPFP_OK; ++rep) {  // warm, timed
      for (int b = 0; b < conc; ++b) {
        float* Yb = Ybuf + NN * b;
        if (hipMemcpyAsync(Yb, pattern.data(), sizeof(float) * NN,
                           hipMemcpyHostToDevice, h->stream) != hipSuccess) {
          st = fail(h, FASTPFP_ERR_HIP, "copy of the tuning matrix failed");
          break;
        }
        pairs[b] = PairIn{N, N, nullptr, nullptr, nullptr, nullptr, Yb,
                          N, N, N, N};
      }
      if (st == FASTPFP_OK)
        st = run(h, pairs, nullptr, fpfp::kModeProject,
                 rep == 0 ? std::min(passes, 8) : passes, 1e-30,
                 FASTPFP_PROJ_ALTERNATING, W, false,
                 infos.data());
      ms = infos[0].kernel_ms;
    }
    if (st != FASTPFP_OK) break;
    double done = 0.0;  // passes actually run (a pass count below `passes`
    for (const auto& inf : infos) done += inf.inner_iters_total;  // = early fixed point)
    const double rate = done / (ms * 1e-3);
    if (k < cap) {
      W_host[k] = W;
      rate_host[k] = rate;
    }
    ++k;
    if (rate > best_rate) {
      best_rate = rate;
      best = W;
    }
  }
  (void)hipFree(Ybuf);
  if (st != FASTPFP_OK) return st;
  *team_size_out = best;
  if (count) *count = std::min(k, cap);
  return FASTPFP_OK;
}

fastpfp_status fastpfp_get_trace(fastpfp_t h, double* out_host, int cap,
                                 int* count) {
  if (!h || !count || (cap > 0 && !out_host)) return FASTPFP_ERR_INVALID_ARG;
  const int m = std::min<int>(cap, (int)h->trace.size());
  for (int i = 0; i < m; ++i) out_host[i] = h->trace[i];
  *count = m;
  return FASTPFP_OK;
}

}  // extern "C"
