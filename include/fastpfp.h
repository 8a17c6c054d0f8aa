/*
 * fastpfp.h -- C ABI of the MI355X FastPFP library (libfastpfp.so).
 *
 * FastPFP (Lu, Huang & Liu, "A Fast Projected Fixed-Point Algorithm for
 * Large Graph Matching", arXiv 1207.1114) relaxes the graph-matching QAP of
 * Sec. 3, eqs. (3)-(4),
 *     max_X  1/2 tr(X^T A X A') + lambda tr(X^T K)
 *     s.t.   X 1 <= 1, X^T 1 = 1, X >= 0                (Sec. 4, relaxed set)
 * and iterates Algorithm 1:
 *     Y[0:n,0:n'] = A X A' + lambda K                        (step 3)
 *     repeat Y = P2(P1(Y)) until max|dY| < tol_inner         (steps 4-7,
 *                                                              eqs. P1, P2)
 *     X = (1 - alpha) X + alpha Y[0:n,0:n']                   (step 8, eq. fastPFP)
 *     X = X / max(X)                                          (step 9)
 * until max|dX| < tol_outer (Sec. 5, convergence criteria).
 * In this ABI the paper's A' is called B.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are row-major float32.  Pointers are DEVICE pointers unless the
 *   argument name ends in _host.  ld* is the row pitch in elements
 *   (ld >= number of columns).
 * - A (n x n) and B (n' x n') must be symmetric (undirected graphs, Sec. 3);
 *   symmetry is assumed, not checked.
 * - Either orientation is accepted: with N = max(n, n'), the smaller side gets
 *   unit sums and the larger side sums <= 1 (the paper writes the n >= n'
 *   case; the other one is its transpose).
 * - The caller owns every buffer it passes; the library never frees one.  A
 *   handle owns its device workspace, grown on demand by solve calls.
 * - All device work is enqueued on the handle's stream; solve/project calls
 *   return after synchronising that stream, when *info is valid.
 * - One handle per host thread.  No C++ exception crosses this ABI; every
 *   function returns a status, and fastpfp_last_error() describes the last
 *   failure on a handle.
 * - Non-convergence is not an error: it returns FASTPFP_OK with
 *   info.converged = 0.
 */
#ifndef FASTPFP_H
#define FASTPFP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FASTPFP_ABI_VERSION 6

typedef struct fastpfp_ctx* fastpfp_t;

typedef enum {
  FASTPFP_OK = 0,
  FASTPFP_ERR_INVALID_ARG = 1, /* bad pointer, NaN/negative parameter, ... */
  FASTPFP_ERR_SHAPE = 2,       /* size or leading dimension out of range   */
  FASTPFP_ERR_HIP = 3,         /* a HIP runtime call failed                */
  FASTPFP_ERR_NOMEM = 4,       /* device workspace allocation failed       */
  FASTPFP_ERR_NUMERIC = 5,     /* NaN/Inf met, or max(X) <= 0 in step 9    */
  FASTPFP_ERR_TIMEOUT = 6,     /* a device-side wait hit its time limit    */
  FASTPFP_ERR_UNSUPPORTED = 7  /* valid request this build cannot run      */
} fastpfp_status;

/* Precision of the two products A X B (step 3).  The projection, the update
 * and all reductions always run in float32, with the global sum 1^T Y 1 in
 * float64. */
enum { FASTPFP_FP32 = 0, FASTPFP_BF16 = 1 };

/* Starting point X0 (Algorithm 1, step 1; initialisation paragraph after it) */
enum { FASTPFP_INIT_UNIFORM = 0, /* X0 = c 1 1^T                     */
       FASTPFP_INIT_USER = 1 };  /* X0 read from the X buffer        */

/* Inner projection of steps 4-7 (Sec. 4.3).  ALTERNATING is Algorithm 1 as
 * printed: repeat Y <- P2(P1(Y)).  DYKSTRA computes the projection P_D of
 * eq. (DSP) that the section defines, by Dykstra's algorithm over the same two
 * sets (a correction term on the clamp P2; same cost per pass, same
 * stopping rule on max|dY|).  The plain alternation converges to a feasible
 * point that is in general not the nearest one; with the paper's start,
 * subgraph-isomorphism pairs of the synthetic benchmark (Sec. 5.1, node
 * deletion) that it misses are recovered exactly with DYKSTRA. */
enum { FASTPFP_PROJ_ALTERNATING = 0, FASTPFP_PROJ_DYKSTRA = 1 };

/* Iteration of the outer loop.  FASTPFP is Algorithm 1 (eq. fastPFP):
 * X <- (1 - alpha) X + alpha P_d(grad f(X)).  PG is the Projected Gradient
 * iteration the paper compares it with (eq. pg, Sec. 4.2):
 * X <- P_d(X + alpha grad f(X)), alpha the step size (any finite value > 0),
 * with the same gradient, projection, stopping rule and step 9 flag (eq. pg
 * has no step 9: pass normalize_max = 0 for it as printed). */
enum { FASTPFP_METHOD_FASTPFP = 0, FASTPFP_METHOD_PG = 1 };

/* Discretisation (Sec. 4.5) */
enum { FASTPFP_HUNGARIAN = 0, /* maximum-weight assignment of X         */
       FASTPFP_GREEDY = 1 };  /* the paper's greedy rule (from SM)      */

typedef struct {
  double lambda;     /* >= 0, weight of K in eq. (3); K may be NULL iff 0    */
  double alpha;      /* step size of eq. fastPFP, in (0, 1]; paper uses 0.5;
                        PG: the step of eq. pg, any finite value > 0        */
  double tol_outer;  /* eps1 > 0: stop when max|X_{t+1} - X_t| < eps1        */
  double tol_inner;  /* eps2 > 0: inner stop when max|Y_{u+1} - Y_u| < eps2  */
  int max_outer;     /* I0 >= 1: cap on outer steps                          */
  int max_inner;     /* I1 >= 1: cap on inner passes per outer step          */
  int precision;     /* FASTPFP_FP32 or FASTPFP_BF16                         */
  int init;          /* FASTPFP_INIT_UNIFORM or FASTPFP_INIT_USER            */
  double init_scale; /* UNIFORM: c; 0 selects c = 1/max(n, n')               */
  int normalize_max; /* 1: step 9 (X /= max X) as in Algorithm 1; 0: skip   */
  int team_size;     /* workgroups per pair; 0 lets the library choose       */
  int projection;    /* FASTPFP_PROJ_ALTERNATING (default) or _DYKSTRA       */
  int method;        /* FASTPFP_METHOD_FASTPFP (default) or _PG              */
} fastpfp_params;

typedef struct {
  int outer_iters;       /* outer steps taken                                */
  int inner_iters_total; /* inner passes summed over outer steps             */
  int inner_iters_max;   /* largest inner pass count of one outer step      */
  int inner_capped;      /* outer steps whose inner loop stopped at I1       */
  int converged;         /* 1 iff the last outer step met eps1               */
  int status;            /* fastpfp_status of this pair                      */
  double eps1_last;      /* max|X_{t+1} - X_t| of the last outer step        */
  double eps2_last;      /* max|Y_{u+1} - Y_u| of the last inner pass        */
  double kernel_ms;      /* device time of the launch that solved the pair   */
  /* The pair's own team time by phase, from device wall-clock stamps taken
   * by the team leader (s_memrealtime): step 3, both products with their
   * team barriers; steps 4-7, tile load and inner loop; and everything
   * (also the set-up and steps 8-9).  A batch runs several teams at once,
   * so these add up per pair, not to kernel_ms. */
  double gemm_ms;
  double proj_ms;
  double pair_ms;
} fastpfp_info;

/* Fills *p with the defaults: lambda 0, alpha 0.5, eps1 1e-6, eps2 1e-8,
 * I0 = I1 = 1000, FP32, uniform start with c = 1/max(n,n'), step 9 on,
 * the alternating projection, the FastPFP iteration. */
fastpfp_status fastpfp_params_default(fastpfp_params* p);

/* Creates a handle bound to HIP device `device` and to `hip_stream` (a
 * hipStream_t; NULL = the null stream).  max_n / max_np bound the sizes
 * later calls may pass (>= 1).  No device memory is allocated here; the
 * first handle on a device looks up that device's fixed scratch array of
 * fastpfp_solve_noalloc.  The environment variable FASTPFP_EXCHANGE=agent,
 * read here, makes the handle's solves exchange every inner pass's sums at
 * device scope even for teams whose workgroups share one XCD (by default
 * those teams post through that XCD's L2); results are the same either way. */
fastpfp_status fastpfp_create(fastpfp_t* h, int device, int max_n, int max_np,
                              void* hip_stream);
fastpfp_status fastpfp_destroy(fastpfp_t h);

/* Solves one pair with Algorithm 1.
 *   A: n x n (lda), B: n' x n' (ldb), K: n x n' (ldk; NULL iff lambda == 0).
 *   X: n x n' (ldx).  In: X0 when p->init == FASTPFP_INIT_USER (ignored
 *      otherwise).  Out: the final iterate X.
 *   Y_state: NULL, or an N x N buffer (row pitch N), N = max(n, n'), holding
 *      the slacked matrix Y of Sec. 4.3.  In: its slack part (the entries
 *      outside the leading n x n' block) seeds the slack; Out: Y after the
 *      last inner loop.  NULL starts the slack at zero (the paper's Y = 0).
 *   info: host pointer, filled on return (may be NULL).
 * Errors: INVALID_ARG for null/ill-formed arguments, SHAPE when n or n'
 * exceed the handle's bounds or ld < columns, NUMERIC on NaN/Inf, TIMEOUT if
 * a device wait gave up, UNSUPPORTED when max(n, n') > 4096 (a team of 256
 * workgroups of 256 x 256 tiles is the largest); X is unspecified after an
 * error. */
fastpfp_status fastpfp_solve(fastpfp_t h, int n, int np,
                             const float* A, int lda,
                             const float* B, int ldb,
                             const float* K, int ldk,
                             const fastpfp_params* p,
                             float* X, int ldx,
                             float* Y_state,
                             fastpfp_info* info);

/* fastpfp_solve without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and meaning as fastpfp_solve, and the
 * same kernels, so the results are bitwise those of fastpfp_solve with the
 * same team size.  Limit: max(n, n') <= FASTPFP_NOALLOC_MAX_N.
 * Instead of the handle's workspace the call uses a library-owned device
 * array of FASTPFP_NOALLOC_SCRATCH_BYTES per GPU (each GPU the library runs
 * on holds it until the process ends); what must start at zero is cleared by
 * a kernel on every call, and nothing is allocated or freed.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (from any
 * handle or host thread) race, so the caller must serialise them.
 * Errors: SHAPE when max(n, n') > FASTPFP_NOALLOC_MAX_N or the launch's
 * workspace would not fit the array; otherwise those of fastpfp_solve.
 * Does not record the eps1 trace that fastpfp_get_trace returns. */
#define FASTPFP_NOALLOC_MAX_N 1024
#define FASTPFP_NOALLOC_SCRATCH_BYTES (17u << 20)
fastpfp_status fastpfp_solve_noalloc(fastpfp_t h, int n, int np,
                                     const float* A, int lda,
                                     const float* B, int ldb,
                                     const float* K, int ldk,
                                     const fastpfp_params* p,
                                     float* X, int ldx,
                                     float* Y_state,
                                     fastpfp_info* info);

/* Solves `batch` independent pairs in one persistent launch.
 *   n_host[b], np_host[b]: sizes of pair b.
 *   A + offA_host[b]: pair b's A, dense n x n (row pitch n); likewise
 *   B + offB_host[b] (n' x n'), K + offK_host[b] (n x n'; K may be NULL iff
 *   lambda == 0), X + offX_host[b] (n x n', in/out as in fastpfp_solve).
 *   Offsets are element counts.  infos_host: batch entries (may be NULL).
 * Every pair runs the same arithmetic as fastpfp_solve with the same team
 * size, so a pair's result does not depend on its batch mates.  A pair that
 * fails (e.g. NUMERIC) is reported in its info.status; the others complete,
 * and the call returns the first failing status. */
fastpfp_status fastpfp_solve_batched(fastpfp_t h, int batch,
                                     const int* n_host, const int* np_host,
                                     const float* A, const int64_t* offA_host,
                                     const float* B, const int64_t* offB_host,
                                     const float* K, const int64_t* offK_host,
                                     const fastpfp_params* p,
                                     float* X, const int64_t* offX_host,
                                     fastpfp_info* infos_host);

/* Runs Algorithm 1's inner repeat (steps 4-7: eqs. P1 then P2 per pass) on
 * one square N x N matrix Y (row pitch N), in place, until
 * max|Y_{u+1} - Y_u| < tol or max_inner passes; with projection =
 * FASTPFP_PROJ_DYKSTRA, Dykstra's passes instead (Y receives the projection,
 * the stopping measure is the change of the projected iterate).
 * info->inner_iters_total receives the pass count and info->eps2_last the
 * last max|dY|.  Exposed so the projection can be checked and timed on its
 * own. */
fastpfp_status fastpfp_project(fastpfp_t h, int N, float* Y, double tol,
                               int max_inner, int team_size, int projection,
                               fastpfp_info* info);

/* The same inner repeat with Y kept in device memory instead of on chip:
 * every pass reads and writes the N x N matrix once (8 N^2 bytes), so it is
 * bound by HBM bandwidth and has no size limit beyond the handle's
 * (N <= max(max_n, max_np)) and memory.  fastpfp_project takes this path by
 * itself for N > 4096 with team_size = 0.  Same arithmetic per entry as the
 * on-chip path (row and column sums reduced in another fixed order; s in
 * float64), same stopping rule and pass count; info->kernel_ms covers the
 * whole call.  Y (device, row pitch N) must hold N x N floats.  Grows a
 * handle-owned scratch of about 4 N (N/64 + N/1024 + 3) bytes.  Returns
 * FASTPFP_ERR_NUMERIC if a sum or max|dY| turns non-finite. */
fastpfp_status fastpfp_project_stream(fastpfp_t h, int N, float* Y, double tol,
                                      int max_inner, int projection,
                                      fastpfp_info* info);

/* Team-size autotuner.  A pair is solved by a team of W workgroups cut
 * into a TR x TC grid of tiles; larger teams finish one pair faster but
 * leave fewer teams for the rest of a batch.  For pairs of size
 * N = max(n, n') in batches of `batch`, this times every power-of-two W from
 * the smallest whose tiles fit N up to the workgroups the device holds,
 * running min(batch, workgroups / W) concurrent projections (Algorithm 1,
 * steps 4-7) of an N x N matrix for `passes` passes each, and returns in
 * *team_size_out the W with the most pair-passes per second (earliest on
 * ties).  W_host / rate_host (cap entries each; may be NULL iff cap == 0)
 * receive every candidate and its rate; *count (nullable) the number
 * written.  Pass the result as fastpfp_params.team_size.  Allocates and
 * frees a scratch buffer of min(batch, workgroups / W) N x N floats. */
fastpfp_status fastpfp_autotune(fastpfp_t h, int N, int batch, int passes,
                                int* team_size_out, int* W_host,
                                double* rate_host, int cap, int* count);

/* Discretises a host matrix X (n x n', ldx) into a partial permutation
 * (Sec. 4.5).  method: FASTPFP_HUNGARIAN (maximise sum_i X[i, m(i)] over
 * injective maps of the smaller side) or FASTPFP_GREEDY (repeatedly take
 * the largest remaining entry, ties to the smallest row-major index, and
 * remove its row and column).  match_host[i] receives the column matched to
 * row i, or -1.  score (nullable) receives sum_i X[i, match[i]] in float64.
 * Host-only; needs no handle or GPU. */
fastpfp_status fastpfp_discretize(int n, int np, const float* X_host, int ldx,
                                  int method, int32_t* match_host,
                                  double* score);

/* The greedy rule of FASTPFP_GREEDY (Sec. 4.5) on the device, for a packed
 * ragged batch of results: pair b's X is n_host[b] x np_host[b], row-major
 * with row pitch np_host[b], at X + offX_host[b] (device float32, as the
 * solver leaves it); its matching is written to match + offM_host[b]
 * (device int32, n_host[b] entries: the column of row i, or -1).  The
 * matching is identical to fastpfp_discretize(..., FASTPFP_GREEDY, ...):
 * entries taken by value, ties to the smaller row-major index.  It is found
 * by parallel row-proposing deferred acceptance on that order, whose unique
 * stable matching is the greedy one.  Sizes must satisfy
 * 1 <= n <= max_n, 1 <= n' <= max_np of the handle.  status_host (nullable,
 * batch entries) receives FASTPFP_OK or FASTPFP_ERR_NUMERIC (X holds a
 * non-finite entry; that pair's match is all -1); the call returns the first
 * non-OK pair status.  Grows a handle-owned scratch of about 8 (n'_1 + ... +
 * n'_batch) bytes; runs on the handle's stream and waits for it. */
fastpfp_status fastpfp_discretize_greedy_batched(
    fastpfp_t h, int batch, const int* n_host, const int* np_host,
    const float* X, const int64_t* offX_host, int32_t* match,
    const int64_t* offM_host, int* status_host);

/* Copies the eps1 trace (max|X_{t+1} - X_t| per outer step) of the last
 * fastpfp_solve on this handle into out_host (up to cap values); returns the
 * number written in *count. */
fastpfp_status fastpfp_get_trace(fastpfp_t h, double* out_host, int cap,
                                 int* count);

/* ------------------------------------------------------------------------
 * Learned warm start.  Not part of the paper's method: it replaces the
 * uniform X0 of Algorithm 1 (the paper notes the result depends on the
 * starting point, Sec. 4.5) by a softmax of similarities between per-node
 * embeddings, and is trained on fixed points of the plain method.
 *
 * Features of node i (48 floats): over i's neighbours k (A[i,k] != 0), a
 * 16-bin histogram of bin(deg(k)) and one of bin(wdeg(k)), each divided by
 * deg(i); bin(v) = clip(floor((4 v) / mean), 0, 15) in float64, with deg the
 * nonzero count and wdeg the sum of a row and mean their average over the
 * graph (a histogram is zero when its mean is <= 0, both are zero when
 * deg(i) = 0); then the first min(fdim, 16) attributes, zero-padded to 16.
 * Network (FASTPFP_WS_NPARAMS floats, in this order, weights row-major
 * out x in): W1 128x48, b1, W2 128x128, b2, W3 64x128, b3, logtau;
 * h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), e = W3 h2 + b3.
 * X0 = softmax of S = E E'^T exp(-logtau) over j for each row i when
 * n <= n' (rows sum to one), over i for each column j otherwise.
 * Training loss for a target T (n x n', positive sums along that axis): with
 * P = T normalised along the same axis, L = -sum P log X0 / min(n, n').
 * Every call synchronises the handle's stream before it returns.  Results
 * are deterministic (fixed-order reductions, no floating-point atomics).
 * ---------------------------------------------------------------------- */
#define FASTPFP_WS_NPARAMS 31041
enum { FASTPFP_WS_BF16_WEIGHTS = 1 }; /* round W1..W3 to bfloat16 (RNE) */

/* Copies FASTPFP_WS_NPARAMS host floats (bytes must equal 4x that) to the
 * handle's device copy and resets the gradient and the Adam moments.
 * INVALID_ARG if a value is not finite, SHAPE if bytes is wrong. */
fastpfp_status fastpfp_warmstart_load(fastpfp_t h, const void* blob_host,
                                      size_t bytes);

/* Copies the parameters and/or the accumulated gradient (either pointer may
 * be NULL) to the host; count must equal FASTPFP_WS_NPARAMS. */
fastpfp_status fastpfp_warmstart_get(fastpfp_t h, float* params_host,
                                     float* grad_host, size_t count);

/* Features of one graph: A (n x n, lda), attributes F (n x fdim, ldf; NULL
 * iff fdim == 0) -> x_out (n x 48, row pitch ldx >= 48, device). */
fastpfp_status fastpfp_warmstart_features(fastpfp_t h, int n, const float* A,
                                          int lda, const float* F, int ldf,
                                          int fdim, float* x_out, int ldx);

/* Forms X0 (n x n', ldx, device) for the pair (A, B) with attributes F
 * (n x fdim) and G (n' x fdim), both NULL iff fdim == 0.  flags:
 * 0 or FASTPFP_WS_BF16_WEIGHTS.  Feed X0 to fastpfp_solve with
 * init = FASTPFP_INIT_USER.  NUMERIC if an entry of X0 is not finite (the
 * caller then falls back to the uniform start). */
fastpfp_status fastpfp_warmstart(fastpfp_t h, int n, int np, const float* A,
                                 int lda, const float* B, int ldb,
                                 const float* F, int ldf, const float* G,
                                 int ldg, int fdim, int flags, float* X0,
                                 int ldx);

/* fastpfp_warmstart for a packed batch, with one synchronisation at the
 * end: the pairs' forward passes run on four streams of the handle at once
 * (pair b on stream b % 4, after the work already on the handle's stream;
 * that stream waits for all four before the call returns, and the results
 * are the same as one pair at a time).  Pair b: A + offA_host[b] (n x n,
 * pitch n), B + offB_host[b] (n' x n', pitch n'), F + offF_host[b]
 * (n x fdim, pitch fdim), G + offG_host[b] (n' x fdim), X + offX_host[b]
 * (n x n', pitch n').
 * F, G and their offsets may be NULL iff fdim == 0.  status_host (nullable,
 * batch entries) receives OK or NUMERIC per pair; every pair is computed and
 * the call returns the first failing status. */
fastpfp_status fastpfp_warmstart_batched(
    fastpfp_t h, int batch, const int* n_host, const int* np_host,
    const float* A, const int64_t* offA_host, const float* B,
    const int64_t* offB_host, const float* F, const int64_t* offF_host,
    const float* G, const int64_t* offG_host, int fdim, int flags, float* X,
    const int64_t* offX_host, int* status_host);

/* Adds the gradient of L for target T (n x n', ldt, device) to the handle's
 * gradient buffer (float32 weights, no rounding); loss_host (nullable)
 * receives L.  NUMERIC if a softmax output or a target sum is not finite or
 * a target sum is <= 0. */
fastpfp_status fastpfp_warmstart_grad(fastpfp_t h, int n, int np,
                                      const float* A, int lda, const float* B,
                                      int ldb, const float* F, int ldf,
                                      const float* G, int ldg, int fdim,
                                      const float* T, int ldt,
                                      double* loss_host);

fastpfp_status fastpfp_warmstart_zero_grad(fastpfp_t h);

/* One Adam step (Kingma & Ba) on the parameters with gradient
 * grad_scale * (accumulated gradient); the handle counts the steps for the
 * bias correction.  lr > 0, 0 <= beta < 1, eps > 0. */
fastpfp_status fastpfp_warmstart_adam(fastpfp_t h, double lr, double beta1,
                                      double beta2, double eps,
                                      double grad_scale);

const char* fastpfp_status_string(fastpfp_status s);
const char* fastpfp_last_error(fastpfp_t h);
int fastpfp_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FASTPFP_H */
