"""Benchmark: matched pairs/s of the FastPFP iteration at n = n' = 1000.

One step solves the whole n=1000 metric set (32 seeded synthetic pairs of
the config-1 workload: Bernoulli(0.1) U(0,1) weighted graphs, relabelled
copies with N(0, 0.05^2) edge noise, 16-d attributes, Gaussian K, lambda 1,
alpha 0.5) to convergence in one persistent launch, inputs resident in HBM.
Discretisation (Hungarian) runs after the timed region.

Prints one JSON line.  ``value`` is the plain method: FP32 products, uniform
start, eps1 = 1e-6.  ``roofline`` describes the persistent kernel (the only
kernel of a step): its inner projection passes are ALU-bound with Y held on
chip, so ``achieved`` counts 7 float32 operations per entry per pass (P1: 2
adds, P2: 1 max, row/column sums: 2 adds, max|dY|: 1 sub + 1 max) over the
kernel's average launch time measured with HIP events on the library's
stream; ``traffic`` is the HBM bytes of one launch from counter runs.
Further legs on the same pairs: ``fp32_tol_5e-4`` (FP32 at the BF16 legs'
eps1, the control that separates the tolerance from the precision),
``bf16`` (BF16 products, uniform start), ``bf16_warmstart`` (BF16 products
from the learned start, the batched warm start inside the timed step,
uniform re-solve of any pair it fails; its speed-up split into tolerance,
BF16 and learned-start factors).  Other workloads: ``config2`` (one
n = 1000 x 1200 pair with outliers), ``config4`` (n = 2000, plain against
BF16 + learned start) and ``config3`` (512 ragged pairs in one launch).
Every leg that has a stored FP64 oracle run reports its error against it on
every entry; ``phases`` gives the per-pair team time of step 3, steps 4-7
and the rest from device clock stamps, and the products' rate within step
3.  ``cpu_baseline`` times full FP64 oracle solves on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("matched pairs/s at n=1000 (plain FP32 vs BF16+warm start); "
          "A·X·B TFLOP/s")
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz for non-FMA, non-packed
# float32 VALU instructions (the 157.3 TFLOP/s vector figure counts an FMA
# as two operations and packed FP32 as two lanes; this build uses neither).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
OPS_PER_ENTRY_PASS = 7
# With bfloat16 products max|X_{t+1} - X_t| wanders on a plateau instead of
# falling below 1e-6 (bfloat16 rounding of X and T moves the fixed point each
# step); the largest plateau value seen over 32 pairs at n = 1000 was 3.1e-4,
# so the BF16 legs stop at 5e-4.
BF16_TOL_OUTER = 5e-4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--pairs", type=int, default=32)
    ap.add_argument("--n", type=int, default=1000)
    ap.add_argument("--team-size", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-passes", type=int, default=300,
                    help="inner passes of the one-thread oracle sample")
    ap.add_argument("--cpu-repeats", type=int, default=1,
                    help="full oracle solves timed (median reported)")
    ap.add_argument("--stream-only", action="store_true",
                    help="run only the streaming-projection leg (N = 8192, "
                         "16384) and an in-place elementwise add on the same "
                         "matrices for reference, print one JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for "
                         "HBM byte counters) and exit")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the BF16, warm-start and ragged-batch legs")
    ap.add_argument("--products-only", action="store_true",
                    help="run only the products leg (8 outer steps x 1 inner "
                         "pass on the metric set, FP32 and BF16) and print "
                         "it as one JSON line")
    return ap.parse_args()


def make_inputs(torch, n_pairs, n):
    from paper_1207_1114_amd import synth
    pairs = [synth.config1_pair(i, n=n) for i in range(n_pairs)]
    N = n * n
    A = torch.empty(n_pairs * N, dtype=torch.float32, device="cuda:0")
    B = torch.empty_like(A)
    K = torch.empty_like(A)
    X = torch.zeros_like(A)
    for i, p in enumerate(pairs):
        sl = slice(i * N, (i + 1) * N)
        A[sl] = torch.from_numpy(p.A.ravel().astype(np.float32))
        B[sl] = torch.from_numpy(p.B.ravel().astype(np.float32))
        K[sl] = torch.from_numpy(p.K.ravel().astype(np.float32))
    offs = [i * N for i in range(n_pairs)]
    return pairs, A.view(-1, 1), B.view(-1, 1), K.view(-1, 1), X.view(-1, 1), offs


def cpu_baseline(pair, gpu_infos, passes, repeats):
    """The FP64 oracle on the host: `repeats` full solves of config-1 pair 0
    (median reported), all host cores for the products (NumPy's elementwise
    passes run on one thread), and a one-thread figure from a bounded sample
    (one gradient and `passes` inner passes with BLAS held to one thread,
    scaled to the pair's outer / inner counts)."""
    from oracle import fastpfp_oracle as O
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        blas_threads = max([d.get("num_threads", 1)
                            for d in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        blas_threads = os.cpu_count()
    times, r = [], None
    for _ in range(max(1, repeats)):
        t0 = time.perf_counter()
        r = O.fastpfp(pair.A, pair.B, pair.K, pair.lam)
        times.append(time.perf_counter() - t0)
    t_pair = float(np.median(times))
    one = None
    if threadpool_limits is not None:
        n, m = pair.n, pair.np_
        with threadpool_limits(limits=1):
            X = O.uniform_x0(n, m)
            t0 = time.perf_counter()
            G = O.gradient(pair.A, X, pair.B, pair.K, pair.lam)
            t_gemm = time.perf_counter() - t0
            Y = np.zeros((max(n, m), max(n, m)))
            Y[:n, :m] = G
            t0 = time.perf_counter()
            O.inner_projection(Y, 1e-300, passes)
            t_pass = (time.perf_counter() - t0) / passes
        one = 1.0 / (r.outer_iters * t_gemm + sum(r.inner_iters) * t_pass)
    return {"value": 1.0 / t_pair, "unit": "pairs/s",
            "cores": int(blas_threads), "kind": "oracle",
            "sample": (f"FP64 oracle, full solve of config-1 pair 0 "
                       f"({r.outer_iters} outer steps, {sum(r.inner_iters)} "
                       f"inner passes), median of {len(times)}: "
                       f"{t_pair:.1f} s; products on {blas_threads} BLAS "
                       f"threads, elementwise NumPy on 1 thread"),
            "seconds_per_pair": t_pair, "runs_s": times,
            "one_thread_pairs_per_s": one,
            "one_thread_sample": (f"1 gradient + {passes} inner passes with "
                                  "BLAS on 1 thread, scaled to the same "
                                  "outer / inner counts"),
            "gpu_outer_iters": int(gpu_infos[0]["outer_iters"]),
            "gpu_inner_iters": int(gpu_infos[0]["inner_iters_total"]),
            "host_cpu_count": os.cpu_count()}


def ragged_batch(torch, F, steps):
    """Config 3: 512 ragged pairs (n ~ U{50..400}, n' = n + U{0..40}) of
    distance-weighted 8-NN point graphs, BF16 products, one launch."""
    from paper_1207_1114_amd import scores, synth
    pairs = [synth.config3_pair(i) for i in range(512)]
    offs, cur = {k: [] for k in "ABKX"}, {k: 0 for k in "ABKX"}
    bufs = {k: [] for k in "ABKX"}
    for p in pairs:
        for k, m in (("A", p.A), ("B", p.B), ("K", p.K),
                     ("X", np.zeros((p.n, p.np_)))):
            offs[k].append(cur[k])
            bufs[k].append(m.ravel().astype(np.float32))
            cur[k] += m.size
    d = {k: torch.from_numpy(np.concatenate(v)).cuda().view(-1, 1)
         for k, v in bufs.items()}
    S = F.Solver(512, 512)
    prm = F.default_params(lambda_=1.0, precision=F.BF16,
                           tol_outer=BF16_TOL_OUTER)
    args = ([p.n for p in pairs], [p.np_ for p in pairs], d["A"], offs["A"],
            d["B"], offs["B"], d["K"], offs["K"], d["X"], offs["X"], prm)
    S.solve_batched(*args)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos = S.solve_batched(*args)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S.close()
    Xall = d["X"].cpu().numpy().ravel()
    acc = []
    for p, o in zip(pairs, offs["X"]):
        m, _ = F.discretize(Xall[o:o + p.n * p.np_].reshape(p.n, p.np_))
        acc.append(scores.accuracy(m, p.perm))
    p0 = pairs[0]
    err0 = error_vs_oracle(Xall[:p0.n * p0.np_].reshape(p0.n, p0.np_),
                           "config3_pair0")
    flops = sum(2.0 * p.n * p.np_ * (p.n + p.np_) * i["outer_iters"]
                for p, i in zip(pairs, infos))
    # ALU roofline of the launch: 7 operations per entry of each pair's own
    # N x N matrix per inner pass (the padding of its tiles not counted)
    ops = sum(OPS_PER_ENTRY_PASS * float(max(p.n, p.np_)) ** 2
              * i["inner_iters_total"] for p, i in zip(pairs, infos))
    alu = ops / (infos[0]["kernel_ms"] * 1e-3) / 1e12
    return {"value": steps * len(pairs) / dt, "unit": "pairs/s",
            "roofline": {"bound": "alu", "achieved": alu,
                         "peak": ALU_PEAK_TOPS, "unit": "T ops/s",
                         "frac": alu / ALU_PEAK_TOPS},
            "pairs": len(pairs), "precision": "bf16",
            "tol_outer": BF16_TOL_OUTER,
            "accuracy_mean": float(np.mean(acc)),
            "outer_iters_mean": float(np.mean([i["outer_iters"] for i in infos])),
            "converged": int(sum(i["converged"] for i in infos)),
            "pair0_max_abs_err_vs_fp64_oracle": err0,
            "product_tflops_in_launch": flops / (infos[0]["kernel_ms"] * 1e-3) / 1e12}


# HBM bytes of one launch of the persistent kernel on this workload, from
# two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE; profiles/ holds the
# summaries), each scaled by the factor the same counter reads for a plain
# 1 GiB copy.  Valid only for the kernel source they were taken on.
TRAFFIC = {"kernel_sha256":
           "620bbf8c28049f944db17000c292cd8e260c250ad8e2288055d5dc43d1be9a78",
           "fetch_kib": 7756930.8125 * 2.0,    # copy calibration: x 2.0
           "write_kib": 4845545.53125 * 1.0,   # copy calibration: x 1.0
           "team_size": 16}


def kernel_sha256() -> str:
    import hashlib
    path = os.path.join(ROOT, "paper_1207_1114_amd", "csrc",
                        "fastpfp_kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_bytes(args, team):
    """HBM bytes per launch (read + written), or None when not measured for
    this kernel source, workload and team size."""
    if (TRAFFIC is None or TRAFFIC["kernel_sha256"] != kernel_sha256()
            or args.pairs != 32 or args.n != 1000
            or team != TRAFFIC["team_size"]):
        return None
    return (TRAFFIC["fetch_kib"] + TRAFFIC["write_kib"]) * 1024.0


MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}  # MI355X dense
HBM_PEAK_GBS = 8000.0                                 # MI355X HBM3E


def products_leg(torch, F, S, ns, nps, A, B, K, X, offs, team, steps):
    """The products A X B (step 3) on their own: the same pairs with one
    inner pass per outer step and 8 outer steps, so the launch is almost all
    MFMA work; TFLOP/s = 2 n n' (n + n') x outer steps x pairs / launch."""
    out = {}
    for name, prec in (("fp32", F.FP32), ("bf16", F.BF16)):
        prm = F.default_params(lambda_=1.0, team_size=team, precision=prec,
                               tol_outer=1e-30, max_outer=8, max_inner=1)
        S.solve_batched(ns, nps, A, offs, B, offs, K, offs, X, offs, prm)
        ms = []
        for _ in range(steps):
            infos = S.solve_batched(ns, nps, A, offs, B, offs, K, offs, X,
                                    offs, prm)
            ms.append(infos[0]["kernel_ms"])
        flops = sum(2.0 * n * m * (n + m) * i["outer_iters"]
                    for n, m, i in zip(ns, nps, infos))
        tf = flops / (np.mean(ms) * 1e-3) / 1e12
        out[name] = {"tflops": tf, "peak": MFMA_PEAK_TFLOPS[name],
                     "frac": tf / MFMA_PEAK_TFLOPS[name],
                     "avg_launch_ms": float(np.mean(ms)),
                     "phases": phases(infos, ns, nps, team, name)}
    out["work"] = ("8 outer steps x 1 inner pass per pair; tflops/frac: the "
                   "whole launch (the pass and the update inside the time); "
                   "phases: step 3 alone, on the team's compute units")
    return out


def products_large(torch, F, steps, n=4000):
    """The products leg at n = n' = 4000 (configuration 4's largest size):
    one synthetic pair on one team of every compute unit, the only team that
    holds N = 4000 on chip."""
    _, A, B, K, X, offs = make_inputs(torch, 1, n)
    S = F.Solver(n, n)
    team, _ = S.autotune(n, 1)
    res = products_leg(torch, F, S, [n], [n], A, B, K, X, offs, team, steps)
    S.close()
    res["n"] = n
    return res


def warm_leg(torch, F, pairs, steps, team):
    """BF16 products from the learned warm start on the same pairs as the
    FP32 leg: the timed step is the batched warm start (X0 of every pair),
    the batched solve from it, and the uniform re-solve of any pair the
    learned start did not bring to convergence."""
    from paper_1207_1114_amd import warmstart as W
    try:
        params, meta = W.load_params()
    except (FileNotFoundError, RuntimeError) as e:
        return {"skipped": str(e)}, None
    b = W.pack(torch, pairs)
    n = max(max(b.ns), max(b.nps))
    S = F.Solver(n, n)
    S.warmstart_load(params)
    prm = W.warm_params()
    prm.team_size = team
    W.solve_batched_warm(S, b, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos, extra = W.solve_batched_warm(S, b, prm)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S.close()
    Xs = [b.x(i).cpu().numpy() for i in range(len(pairs))]
    out = {"value": steps * len(pairs) / dt, "unit": "pairs/s",
           "precision": "bf16", "tol_outer": W.BF16_TOL_OUTER,
           "fallbacks": extra["fallbacks"],
           "sharpening_beta": meta.get("beta"),
           "accepted_on_heldout": bool(meta.get("accepted"))}
    return out, (infos, Xs)


def quality(F, pairs, Xs):
    """Hungarian matching of every result: objective (trace form) and
    accuracy against the planted correspondence."""
    from paper_1207_1114_amd import scores
    obj, acc = [], []
    for p, X in zip(pairs, Xs):
        m, _ = F.discretize(X)
        obj.append(scores.matching_objective(p.A, p.B, p.K, p.lam, m))
        acc.append(scores.accuracy(m, p.perm))
    return obj, acc


def error_vs_oracle(X, name):
    """Upper bound of max|X - X_oracle| over every entry, against the stored
    FP64 oracle iterate tests/golden/<name>.npz (entries above tau stored
    exactly, the others within [-tau, tau]); None if the file is absent."""
    path = os.path.join(ROOT, "tests", "golden", name + ".npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    flat = np.asarray(X, np.float64).ravel()
    idx, tau = g["idx"], float(g["tau"])
    err = float(np.abs(flat[idx] - g["val"]).max()) if idx.size else 0.0
    rest = np.ones(flat.size, dtype=bool)
    rest[idx] = False
    rmax = float(np.abs(flat[rest]).max()) if rest.any() else 0.0
    return max(err, rmax + tau) / float(g["xmax"])


def phases(infos, ns, nps, W, prec):
    """Mean per-pair team time in each phase (device wall-clock stamps) and
    the products' rate within their phase: 2 n n' (n + n') flops per outer
    step over the team's step-3 time, against the MFMA peak of the team's
    W compute units."""
    g = np.array([i["gemm_ms"] for i in infos])
    pj = np.array([i["proj_ms"] for i in infos])
    al = np.array([i["pair_ms"] for i in infos])
    flops = np.array([2.0 * n * m * (n + m) * i["outer_iters"]
                      for n, m, i in zip(ns, nps, infos)])
    tf = flops / np.maximum(g * 1e-3, 1e-12) / 1e12
    peak = MFMA_PEAK_TFLOPS[prec] * W / 256.0
    passes = np.array([i["inner_iters_total"] for i in infos])
    return {"team_size": W, "gemm_ms_per_pair": float(g.mean()),
            "proj_ms_per_pair": float(pj.mean()),
            "other_ms_per_pair": float((al - g - pj).mean()),
            "pair_ms": float(al.mean()),
            "proj_us_per_pass": float((pj / np.maximum(passes, 1)).mean()
                                      * 1e3),
            "products_tflops_in_phase": float(tf.mean()),
            "products_frac_of_team_peak": float(tf.mean() / peak),
            "team_peak_tflops": peak}


def discretize_leg(torch, F, S, Xh, X, offs, n, steps):
    """The paper's greedy discretisation (Sec. 4.5) of the batch's results
    on the device, one call for all pairs, against the host greedy and
    Hungarian discretisers on the same matrices."""
    b = Xh.shape[0]
    match = torch.empty(b * n, dtype=torch.int32, device="cuda:0")
    offm = [i * n for i in range(b)]
    args = ([n] * b, [n] * b, X.view(-1), offs, match, offm)
    S.discretize_greedy_batched(*args)
    t0 = time.perf_counter()
    for _ in range(steps):
        S.discretize_greedy_batched(*args)
    dev_ms = (time.perf_counter() - t0) / steps * 1e3
    got = match.view(b, n).cpu().numpy()
    t0 = time.perf_counter()
    host = [F.discretize(Xh[i], F.GREEDY)[0] for i in range(b)]
    greedy_ms = (time.perf_counter() - t0) / b * 1e3
    t0 = time.perf_counter()
    hung = [F.discretize(Xh[i], F.HUNGARIAN)[0] for i in range(b)]
    hung_ms = (time.perf_counter() - t0) / b * 1e3
    return {"device_greedy_ms_per_batch": dev_ms,
            "device_greedy_ms_per_pair": dev_ms / b,
            "host_greedy_ms_per_pair": greedy_ms,
            "host_hungarian_ms_per_pair": hung_ms,
            "device_equals_host_greedy": bool(all(
                (got[i] == host[i]).all() for i in range(b))),
            "greedy_equals_hungarian_pairs": int(sum(
                (host[i] == hung[i]).all() for i in range(b))),
            "pairs": b, "n": n}


def projection_leg(torch, F, S, n, team):
    """Device time per inner pass of the alternating projection (Algorithm 1)
    and of the exact one (Dykstra) on one n x n matrix, team `team`, 1000
    passes each from the same seeded input."""
    rng = np.random.default_rng([1207, 1114, 5, n])
    Y0 = (rng.normal(size=(n, n)) * 2.0 + 0.5).astype(np.float32)
    out = {"n": n, "team_size": team, "passes": 1000}
    for name, proj in (("alternating", F.ALTERNATING),
                       ("dykstra", F.DYKSTRA)):
        Y = torch.tensor(Y0, device="cuda:0")
        S.project(Y, 1e-30, 8, team, projection=proj)      # warm
        Y = torch.tensor(Y0, device="cuda:0")
        info = S.project(Y, 1e-30, 1000, team, projection=proj)
        out[name + "_us_per_pass"] = (info["kernel_ms"] * 1e3
                                      / max(1, info["inner_iters_total"]))
    out["dykstra_over_alternating"] = (out["dykstra_us_per_pass"]
                                       / out["alternating_us_per_pass"])
    return out


def stream_leg(torch, F, sizes=(8192, 16384), passes=50):
    """Steps 4-7 with Y in HBM (fastpfp_project_stream) on random nonnegative
    N x N matrices too large for the on-chip path: 8 N^2 algorithmic bytes
    per pass (read Y, write D) against the 8 TB/s HBM peak.  The time is the
    whole call (launches, and a flag check every 32 passes, included)."""
    out = {"passes": passes, "bytes_per_pass": "8 N^2"}
    S = F.Solver(max(sizes), max(sizes))
    g = torch.Generator(device="cuda:0")
    for N in sizes:
        g.manual_seed(N)
        Y = torch.rand(N, N, device="cuda:0", generator=g)
        S.project_stream(Y, 1e-30, 2)                      # warm
        info = S.project_stream(Y, 1e-30, passes)
        us = info["kernel_ms"] * 1e3 / info["inner_iters_total"]
        gbs = 8.0 * N * N / (us * 1e-6) / 1e9
        out[str(N)] = {"us_per_pass": us, "GB_per_s": gbs,
                       "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
        del Y
    S.close()
    return out


def elementwise_reference(torch, sizes=(8192, 16384), reps=20):
    """In-place Y += 1 on the same N x N float32 matrices (8 N^2 bytes per
    call, like a projection pass): what a plain streaming kernel reaches."""
    out = {}
    for N in sizes:
        Y = torch.rand(N, N, device="cuda:0")
        for _ in range(3):
            Y.add_(1.0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            Y.add_(1.0)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        out[str(N)] = {"us": us, "GB_per_s": 8.0 * N * N / (us * 1e-6) / 1e9}
        del Y
    return out


def batch_run(torch, S, ns, nps, A, B, K, X, offs, prm, steps):
    """Warm-up plus `steps` timed batched solves; returns (pairs/s, infos of
    the last solve, the mean launch time of the timed solves)."""
    S.solve_batched(ns, nps, A, offs, B, offs, K, offs, X, offs, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = []
    for _ in range(steps):
        infos = S.solve_batched(ns, nps, A, offs, B, offs, K, offs, X, offs,
                                prm)
        ms.append(infos[0]["kernel_ms"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return steps * len(ns) / dt, infos, float(np.mean(ms))


def single_pair_leg(torch, F, p, name, steps, team=0):
    """One pair of another configuration solved alone, FP32 (eps1 1e-6) and
    BF16 (eps1 5e-4): pairs/s, iteration counts, error against the stored
    FP64 oracle, matching quality."""
    dev = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda:0")
    S = F.Solver(p.n, p.np_)
    A, B, K = dev(p.A), dev(p.B), dev(p.K)
    out = {"n": p.n, "n_prime": p.np_}
    for tag, prec, tol in (("fp32", F.FP32, 1e-6),
                           ("bf16", F.BF16, BF16_TOL_OUTER)):
        prm = F.default_params(lambda_=p.lam, precision=prec, tol_outer=tol,
                               team_size=team)
        X = torch.zeros(p.n, p.np_, device="cuda:0")
        S.solve(A, B, K, X, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = S.solve(A, B, K, X, prm)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        Xh = X.cpu().numpy()
        obj, acc = quality(F, [p], [Xh])
        out[tag] = {"pairs_per_s": steps / dt, "tol_outer": tol,
                    "outer_iters": info["outer_iters"],
                    "inner_iters": info["inner_iters_total"],
                    "max_abs_err_vs_fp64_oracle": error_vs_oracle(Xh, name),
                    "objective": obj[0], "accuracy": acc[0],
                    "gemm_ms": info["gemm_ms"], "proj_ms": info["proj_ms"]}
    S.close()
    return out


def config4_leg(torch, F, steps, n=2000, count=4):
    """Configuration 4 at its evaluation size: `count` held-out pairs at
    n = n' = 2000, the plain method (FP32, uniform start, eps1 1e-6) against
    BF16 products from the learned start (eps1 5e-4), both batched; pair 0
    is compared with the stored FP64 oracle run."""
    from paper_1207_1114_amd import synth
    from paper_1207_1114_amd import warmstart as W
    params, _ = W.load_params()
    pairs = [synth.config4_pair(i, n) for i in range(count)]
    b = W.pack(torch, pairs)
    S = F.Solver(n, n)
    W.solve_batched(S, b, F.default_params(lambda_=1.0))      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pinfos = W.solve_batched(S, b, F.default_params(lambda_=1.0))
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / steps
    Xp = [b.x(i).cpu().numpy() for i in range(count)]
    S.warmstart_load(params)
    prm = W.warm_params()
    W.solve_batched_warm(S, b, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        winfos, extra = W.solve_batched_warm(S, b, prm)
    torch.cuda.synchronize()
    t_warm = (time.perf_counter() - t0) / steps
    Xw = [b.x(i).cpu().numpy() for i in range(count)]
    S.close()
    op, ap = quality(F, pairs, Xp)
    ow, aw = quality(F, pairs, Xw)
    return {"n": n, "pairs": count,
            "plain_fp32": {"pairs_per_s": count / t_plain,
                           "outer_iters_mean": float(np.mean(
                               [i["outer_iters"] for i in pinfos])),
                           "accuracy_mean": float(np.mean(ap)),
                           "pair0_max_abs_err_vs_fp64_oracle":
                               error_vs_oracle(Xp[0], f"config4_n{n}_pair0"),
                           "phases": phases(pinfos, [n] * count,
                                            [n] * count, 64, "fp32")},
            "bf16_warmstart": {"pairs_per_s": count / t_warm,
                               "outer_iters_mean": float(np.mean(
                                   [i["outer_iters"] for i in winfos])),
                               "accuracy_mean": float(np.mean(aw)),
                               "fallbacks": extra["fallbacks"],
                               "pair0_max_abs_err_vs_fp64_oracle":
                                   error_vs_oracle(Xw[0],
                                                   f"config4_n{n}_pair0"),
                               "phases": phases(winfos, [n] * count,
                                                [n] * count, 64, "bf16")},
            "speedup": t_plain / t_warm,
            "objective_rel_diff": float((np.mean(ow) - np.mean(op))
                                        / abs(np.mean(op))),
            "accuracy_diff": float(np.mean(aw) - np.mean(ap))}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); "
              "sharding pairs over several GPUs is not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.stream_only:
        from paper_1207_1114_amd import fastpfp as F
        print(json.dumps({"projection_stream": stream_leg(torch, F),
                          "elementwise_add_reference":
                              elementwise_reference(torch)}), flush=True)
        return
    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4,
                          "copy_bytes_written": y.numel() * 4}), flush=True)
        return
    from paper_1207_1114_amd import fastpfp as F
    from paper_1207_1114_amd import synth

    torch.cuda.init()
    pairs, A, B, K, X, offs = make_inputs(torch, args.pairs, args.n)
    n = args.n
    S = F.Solver(n, n)
    # team size: the autotuner's pick for this batch unless one is given
    tuned = None
    team = args.team_size
    if team == 0:
        team, cands = S.autotune(n, args.pairs)
        tuned = {"chosen": team, "pair_passes_per_s": dict(cands)}
    prm = F.default_params(lambda_=1.0, team_size=team)
    ns, nps = [n] * args.pairs, [n] * args.pairs
    if args.products_only:
        res = products_leg(torch, F, S, ns, nps, A, B, K, X, offs, team,
                           args.steps)
        S.close()
        print(json.dumps({"products": res, "team_size": team}), flush=True)
        return

    def step():
        return S.solve_batched(ns, nps, A, offs, B, offs, K, offs, X, offs,
                               prm)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_infos = []
    for _ in range(args.steps):
        all_infos.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps * args.pairs / dt

    infos = all_infos[-1]
    kernel_ms = float(np.mean([inf[0]["kernel_ms"] for inf in all_infos]))
    passes = sum(i["inner_iters_total"] for i in infos)
    ops = OPS_PER_ENTRY_PASS * float(n * n) * passes
    achieved = ops / (kernel_ms * 1e-3) / 1e12
    gemm_flops = sum(i["outer_iters"] for i in infos) * 2.0 * n * n * (2 * n)

    Xh = X.view(args.pairs, n, n).cpu().numpy()
    obj, acc = quality(F, pairs, list(Xh))

    out = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "node_matches_per_s": value * n, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"config-1 metric set: {args.pairs} seeded "
                                f"synthetic pairs, n=n'={n}, edge p=0.1, "
                                "noise 0.05, 16-d attributes, lambda=1, "
                                "alpha=0.5, eps1=1e-6, eps2=1e-8, "
                                "I0=I1=1000, FP32 products"),
                   "pairs_per_step": args.pairs, "n": n, "precision": "fp32",
                   "team_size": team,
                   "team_size_from": "autotuner" if tuned else "argument"},
        "roofline": {"bound": "alu", "achieved": achieved,
                     "peak": ALU_PEAK_TOPS, "unit": "T ops/s",
                     "frac": achieved / ALU_PEAK_TOPS,
                     "traffic": traffic_bytes(args, team),
                     "kernel": "fastpfp_persistent",
                     "avg_launch_ms": kernel_ms,
                     "work_per_launch": (f"{passes} inner passes x {n}^2 "
                                         f"entries x {OPS_PER_ENTRY_PASS} ops")},
        "gemm_tflops_in_launch": gemm_flops / (kernel_ms * 1e-3) / 1e12,
        "phases": phases(infos, ns, nps, team, "fp32"),
        "outer_iters_mean": float(np.mean([i["outer_iters"] for i in infos])),
        "inner_iters_mean": float(np.mean([i["inner_iters_total"]
                                           for i in infos])),
        "accuracy_mean": float(np.mean(acc)),
        "objective_mean": float(np.mean(obj)),
        "pair0_max_abs_err_vs_fp64_oracle": (
            error_vs_oracle(Xh[0], "config1_pair0") if n == 1000 else None),
        "converged": int(sum(i["converged"] for i in infos)),
        "autotune": tuned,
    }
    if not args.no_extra:
        out["discretize"] = discretize_leg(torch, F, S, Xh, X, offs, n,
                                           args.steps)
        out["projection"] = projection_leg(torch, F, S, n, team)
        out["projection_stream"] = stream_leg(torch, F)
        out["projection_stream"]["elementwise_add_reference"] = \
            elementwise_reference(torch)
        # the same pairs: FP32 at the BF16 legs' eps1 (the control that
        # separates the looser tolerance from the BF16 products), then BF16
        legs = {}
        for tag, prec in (("fp32_tol_5e-4", F.FP32), ("bf16", F.BF16)):
            pr = F.default_params(lambda_=1.0, team_size=team, precision=prec,
                                  tol_outer=BF16_TOL_OUTER)
            v, inf, _ = batch_run(torch, S, ns, nps, A, B, K, X, offs, pr,
                                  args.steps)
            Xl = X.view(args.pairs, n, n).cpu().numpy()
            ob, ac = quality(F, pairs, list(Xl))
            legs[tag] = {"value": v, "unit": "pairs/s",
                         "tol_outer": BF16_TOL_OUTER,
                         "accuracy_mean": float(np.mean(ac)),
                         "objective_rel_diff_vs_fp32": float(
                             (np.mean(ob) - np.mean(obj)) / abs(np.mean(obj))),
                         "outer_iters_mean": float(np.mean(
                             [i["outer_iters"] for i in inf])),
                         "pair0_max_abs_err_vs_fp64_oracle": (
                             error_vs_oracle(Xl[0], "config1_pair0")
                             if n == 1000 else None),
                         "phases": phases(inf, ns, nps, team,
                                          "bf16" if prec == F.BF16
                                          else "fp32")}
        out.update(legs)
        warm, res = warm_leg(torch, F, pairs, args.steps, team)
        if res is not None:
            winf, Xw = res
            ob, ac = quality(F, pairs, Xw)
            warm.update({
                "outer_iters_mean": float(np.mean([i["outer_iters"]
                                                   for i in winf])),
                "accuracy_mean": float(np.mean(ac)),
                "accuracy_diff_vs_fp32": float(np.mean(ac) - np.mean(acc)),
                "objective_rel_diff_vs_fp32": float(
                    (np.mean(ob) - np.mean(obj)) / abs(np.mean(obj))),
                "pair0_max_abs_err_vs_fp64_oracle": (
                    error_vs_oracle(Xw[0], "config1_pair0")
                    if n == 1000 else None),
                "speedup_vs_fp32": warm["value"] / value,
                "speedup_vs_fp32_tol_5e-4":
                    warm["value"] / legs["fp32_tol_5e-4"]["value"],
                # the speed-up split into its three factors (their product)
                "factor_tolerance": legs["fp32_tol_5e-4"]["value"] / value,
                "factor_bf16_products":
                    legs["bf16"]["value"] / legs["fp32_tol_5e-4"]["value"],
                "factor_learned_start": warm["value"] / legs["bf16"]["value"],
                "phases": phases(winf, ns, nps, team, "bf16")})
        out["bf16_warmstart"] = warm
        out["config2"] = single_pair_leg(torch, F, synth.config2_pair(0),
                                         "config2_pair0", args.steps)
        out["config4"] = config4_leg(torch, F, args.steps)
        out["config3"] = ragged_batch(torch, F, args.steps)
        out["products"] = products_leg(torch, F, S, ns, nps, A, B, K, X, offs,
                                       team, args.steps)
        out["products_n4000"] = products_large(torch, F, args.steps)
    S.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pairs[0], infos, args.cpu_passes,
                                           args.cpu_repeats)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
