"""The paper's synthetic benchmark (Sec. 5.1) on the GPU solver.

Unweighted random graphs with 50% connectivity, n = 100 .. 1500, in four
cases: (a) isomorphic, (b) n edge flips, (c) 10% of the first graph's nodes
deleted (subgraph isomorphism), (d) both.  Every (n, case) setting is solved
in one batched launch with the paper's settings: FP32 products, lambda = 0,
alpha = 0.5, the recommended start X0 = 1 1^T / (n n') (the initialisation
paragraph after Algorithm 1), eps1 = 1e-6, eps2 = 1e-8, I0 = I1 = 1000, with
Algorithm 1's alternating inner projection or the exact one (Dykstra), and
discretised with both the greedy method the paper's experiments use and the
Hungarian method.

Reported per setting: the device time per pair (launch time / pairs), the
mean outer steps, the matching error ||A - X A' X^T||_F^2 minus that of the
planted correspondence (<= 0: a match at least as good as the ground truth,
which the paper reports for FastPFP in all four cases) and the fraction of
nodes matched to their planted partner.

    python -m paper_1207_1114_amd.paper_benchmark [--sizes 100,500,1000,1500]
        [--pairs 4] [--cases abcd] [--projection alternating|dykstra|both]
        [--method fastpfp|pg] [--alpha 0.5[,0.7,...]]

The same runner gives the step-size study of Sec. 6.2 (FastPFP with
alpha in [0.1, 1]) and the Projected Gradient comparison of Sec. 5
(--method pg, alpha its step size) on these synthetic pairs.
"""
from __future__ import annotations

import json

import numpy as np

from . import fastpfp as F
from . import scores, synth

CASES = {"a": (False, False), "b": (True, False), "c": (False, True),
         "d": (True, True)}
SIZES = (100, 300, 500, 700, 900, 1100, 1300, 1500)
NUMERIC = 5  # FASTPFP_ERR_NUMERIC


def pairs_for(n: int, case: str, count: int) -> list:
    flips, deletion = CASES[case]
    return [synth.paper_synthetic_pair(i, n, flips, deletion)
            for i in range(count)]


def solve(S, torch, pairs, prm_kw: dict | None = None):
    """One batched launch over `pairs` (lambda = 0, no K) with the paper's
    start; returns (list of X as float64 arrays, infos)."""
    offs = {k: [] for k in "ABX"}
    cur = {k: 0 for k in "ABX"}
    bufs = {k: [] for k in "ABX"}
    for p in pairs:
        for k, m in (("A", p.A), ("B", p.B), ("X", np.zeros((p.n, p.np_)))):
            offs[k].append(cur[k])
            bufs[k].append(np.asarray(m, np.float32).ravel())
            cur[k] += m.size
    d = {k: torch.from_numpy(np.concatenate(v)).to("cuda").view(-1, 1)
         for k, v in bufs.items()}
    # the recommended start 1 1^T / (n n'): one scale for a batch of one size
    n0, m0 = pairs[0].n, pairs[0].np_
    assert all((p.n, p.np_) == (n0, m0) for p in pairs)
    kw = dict(lambda_=0.0, init_scale=1.0 / (n0 * m0))
    kw.update(prm_kw or {})
    try:
        infos = S.solve_batched([p.n for p in pairs], [p.np_ for p in pairs],
                                d["A"], offs["A"], d["B"], offs["B"], None,
                                None, d["X"], offs["X"],
                                F.default_params(**kw))
    except F.FastPFPError as e:
        # pairs whose iterates overflowed (status NUMERIC) are reported as
        # failed; the rest of the batch is complete
        if e.status != NUMERIC or not hasattr(e, "infos"):
            raise
        infos = e.infos
    Xall = d["X"].cpu().numpy().ravel().astype(np.float64)
    Xs = [Xall[o:o + p.n * p.np_].reshape(p.n, p.np_)
          for p, o in zip(pairs, offs["X"])]
    return Xs, infos


def evaluate(pairs, Xs, method: int = F.HUNGARIAN, infos=None) -> dict:
    """Scores of the discretised results; `solved` counts pairs whose error
    is at most the planted correspondence's.  A pair whose solve ended with
    non-finite values scores as no match (every node unmatched)."""
    diff, acc = [], []
    for k, (p, X) in enumerate(zip(pairs, Xs)):
        if infos is not None and infos[k]["status"] != 0:
            m = np.full(p.n, -1, dtype=np.int32)
        else:
            m, _ = F.discretize(X, method)
        diff.append(scores.frobenius_error(p.A, p.B, m)
                    - scores.frobenius_error(p.A, p.B, p.perm))
        acc.append(scores.accuracy(m, p.perm))
    return {"error_minus_ground_truth_mean": float(np.mean(diff)),
            "error_minus_ground_truth_max": float(np.max(diff)),
            "solved": int(sum(d <= 0.0 for d in diff)),
            "accuracy_mean": float(np.mean(acc))}


PROJECTIONS = {"alternating": F.ALTERNATING, "dykstra": F.DYKSTRA}
METHODS = {"fastpfp": F.METHOD_FASTPFP, "pg": F.METHOD_PG}


def run(sizes=SIZES, count: int = 4, projection: str = "alternating",
        method: str = "fastpfp", alpha: float = 0.5, cases=tuple(CASES),
        log=print) -> list:
    """One batched launch per (n, case).  method "pg" runs eq. (pg) with
    step alpha and no step 9; "fastpfp" runs Algorithm 1 with damping
    alpha."""
    import torch
    S = F.Solver(max(sizes), max(sizes))
    prm = {"projection": PROJECTIONS[projection], "method": METHODS[method],
           "alpha": alpha}
    if method == "pg":
        prm["normalize_max"] = 0
    rows = []
    for n in sizes:
        for case in cases:
            pairs = pairs_for(n, case, count)
            Xs, infos = solve(S, torch, pairs, prm)
            row = {"n": n, "case": case, "pairs": count, "method": method,
                   "alpha": alpha, "projection": projection,
                   "ms_per_pair": infos[0]["kernel_ms"] / count,
                   "outer_mean": float(np.mean([i["outer_iters"]
                                                for i in infos])),
                   "converged": int(sum(i["converged"] for i in infos)),
                   "non_finite": int(sum(i["status"] == NUMERIC
                                         for i in infos)),
                   "hungarian": evaluate(pairs, Xs, F.HUNGARIAN, infos),
                   "greedy": evaluate(pairs, Xs, F.GREEDY, infos)}
            rows.append(row)
            log(json.dumps(row))
    S.close()
    return rows


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default=",".join(str(s) for s in SIZES))
    ap.add_argument("--pairs", type=int, default=4)
    ap.add_argument("--cases", default="abcd")
    ap.add_argument("--projection", choices=[*PROJECTIONS, "both"],
                    default="both")
    ap.add_argument("--method", choices=list(METHODS), default="fastpfp")
    ap.add_argument("--alpha", default="0.5",
                    help="FastPFP damping or PG step; a comma list sweeps")
    a = ap.parse_args()
    sizes = tuple(int(v) for v in a.sizes.split(","))
    for proj in (PROJECTIONS if a.projection == "both" else [a.projection]):
        for alpha in (float(v) for v in a.alpha.split(",")):
            run(sizes, a.pairs, proj, a.method, alpha, tuple(a.cases))


if __name__ == "__main__":
    main()
