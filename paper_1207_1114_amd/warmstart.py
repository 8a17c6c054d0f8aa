"""Learned warm start: training it on fixed points of the plain method, and
solving with it while the uniform start stays the fallback and the reference.

The network and its kernels live in the library (``fastpfp_warmstart*``
entry points); this module only orchestrates them.

* Runtime (``solve_batched_warm``): X0 of every pair from the network, then
  Algorithm 1 from that X0 (init = USER).  A pair whose X0 is not finite, or
  whose solve fails or does not converge, is solved again from the uniform
  start, so the learned start can only replace the plain one, never lose a
  pair.
* Training (``train``): seeded training pairs of the config-4 model
  (Bernoulli(0.05) graphs, n = n' ~ U{100..500}, noise 0.05, 16-d
  attributes) are generated in chunks, solved in one batched FP32 launch
  from the uniform start, and their fixed points X* are the targets of the
  cross-entropy loss; Adam steps over minibatches run on the GPU through the
  library's forward and backward kernels.
* Acceptance (``evaluate``): on held-out pairs, BF16 products with the
  learned start must reach the plain FP32 run's objective within 1e-3
  relative and its matching accuracy within 0.5 percentage points.  The
  verdict is stored with the parameters; ``load_params`` refuses parameters
  that were not accepted unless asked otherwise.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import fastpfp as F
from . import scores, synth

HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_NPY = os.path.join(HERE, "warmstart_params.npy")
PARAMS_JSON = os.path.join(HERE, "warmstart_params.json")

# With bfloat16 products max|X_{t+1} - X_t| wanders on a plateau (up to
# 3.1e-4 over 32 pairs at n = 1000) instead of falling to the paper's 1e-6,
# so runs with BF16 products stop at 5e-4; float32 runs keep 1e-6.
BF16_TOL_OUTER = 5e-4
# A learned start that has not converged after this many outer steps is
# abandoned and the pair solved again from the uniform start.
WARM_MAX_OUTER = 100
OBJ_REL_TOL = 1e-3      # acceptance: objective within 1e-3 relative
ACC_TOL = 0.005         # acceptance: accuracy within 0.5 percentage points


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases, tau = 8 (log tau = log 8)."""
    rng = np.random.default_rng([1207, 1114, 4444, seed])
    parts = []
    for shape in ((128, 48), (128,), (128, 128), (128,), (64, 128), (64,)):
        if len(shape) == 2:
            b = np.sqrt(6.0 / shape[1])
            parts.append(rng.uniform(-b, b, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    parts.append(np.array([np.log(8.0)]))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == F.WS_NPARAMS
    return flat


def load_params(require_accepted: bool = True) -> tuple[np.ndarray, dict]:
    if not os.path.exists(PARAMS_NPY):
        raise FileNotFoundError(
            f"{PARAMS_NPY} is missing: train the warm start first "
            "(python -m paper_1207_1114_amd.warmstart --train)")
    flat = np.load(PARAMS_NPY, allow_pickle=False).astype(np.float32)
    meta = {}
    if os.path.exists(PARAMS_JSON):
        with open(PARAMS_JSON) as f:
            meta = json.load(f)
    if require_accepted and not meta.get("accepted", False):
        raise RuntimeError("the stored warm-start parameters did not pass "
                           "the acceptance check against the uniform start")
    return flat, meta


# ---------------------------------------------------------------- batches
@dataclass
class Batch:
    """Pairs packed densely on the device (row pitch = number of columns)."""
    pairs: list
    ns: list
    nps: list
    A: object
    B: object
    K: object
    Fa: object
    Gb: object
    X: object
    offA: list
    offB: list
    offK: list
    offF: list
    offG: list
    fdim: int

    def view(self, buf, off, rows, cols):
        return buf[off:off + rows * cols].view(rows, cols)

    def x(self, i):
        return self.view(self.X, self.offK[i], self.ns[i], self.nps[i])


def pack(torch, pairs, fdim: int = 16) -> Batch:
    offs = {k: [] for k in "ABKFG"}
    cur = {k: 0 for k in "ABKFG"}
    bufs = {k: [] for k in "ABKFG"}
    for p in pairs:
        Fp = p.F if p.F is not None else np.zeros((p.n, fdim))
        Gp = p.G if p.G is not None else np.zeros((p.np_, fdim))
        for k, m in (("A", p.A), ("B", p.B), ("K", p.K), ("F", Fp),
                     ("G", Gp)):
            offs[k].append(cur[k])
            bufs[k].append(np.asarray(m, np.float32).ravel())
            cur[k] += m.size
    d = {k: torch.from_numpy(np.concatenate(v)).to("cuda")
         for k, v in bufs.items()}
    X = torch.zeros_like(d["K"])
    return Batch(pairs, [p.n for p in pairs], [p.np_ for p in pairs],
                 d["A"], d["B"], d["K"], d["F"], d["G"], X, offs["A"],
                 offs["B"], offs["K"], offs["F"], offs["G"], fdim)


def solve_batched(S, b: Batch, prm) -> list:
    return S.solve_batched(b.ns, b.nps, b.A.view(-1, 1), b.offA,
                           b.B.view(-1, 1), b.offB, b.K.view(-1, 1), b.offK,
                           b.X.view(-1, 1), b.offK, prm)


def _attrs(b: Batch, i):
    Fa = b.view(b.Fa, b.offF[i], b.ns[i], b.fdim)
    Gb = b.view(b.Gb, b.offG[i], b.nps[i], b.fdim)
    return Fa, Gb


def warm_x0(S, b: Batch, i: int, bf16_weights: bool = True) -> bool:
    """Writes the learned X0 of pair i into b.X; False if it is not finite
    (X0 is then the uniform start)."""
    A = b.view(b.A, b.offA[i], b.ns[i], b.ns[i])
    B = b.view(b.B, b.offB[i], b.nps[i], b.nps[i])
    Fa, Gb = _attrs(b, i)
    try:
        S.warmstart(A, B, Fa, Gb, b.x(i), bf16_weights=bf16_weights)
        return True
    except F.FastPFPError as e:
        if e.status != 5:
            raise
        b.x(i).fill_(1.0 / max(b.ns[i], b.nps[i]))
        return False


def solve_batched_warm(S, b: Batch, prm, bf16_weights: bool = True
                       ) -> tuple[list, dict]:
    """Learned X0 for every pair, one batched solve from it, and a uniform
    re-solve of every pair the learned start did not bring to convergence.
    ``prm`` must have init = INIT_USER."""
    import ctypes
    torch = _torch()
    status = S.warmstart_batched(b.ns, b.nps, b.A.view(-1, 1), b.offA,
                                 b.B.view(-1, 1), b.offB, b.Fa.view(-1, 1),
                                 b.offF, b.Gb.view(-1, 1), b.offG, b.fdim,
                                 b.X.view(-1, 1), b.offK, bf16_weights)
    warm_ok = [st == 0 for st in status]
    for i, ok in enumerate(warm_ok):
        if not ok:      # non-finite X0: this pair starts uniform
            b.x(i).fill_(1.0 / max(b.ns[i], b.nps[i]))
    try:
        infos = solve_batched(S, b, prm)
    except F.FastPFPError as e:
        infos = e.infos
    redo = [i for i, inf in enumerate(infos)
            if inf["status"] != 0 or not inf["converged"]]
    if redo:
        uni = F.Params()
        ctypes.memmove(ctypes.byref(uni), ctypes.byref(prm),
                       ctypes.sizeof(F.Params))
        uni.init = F.INIT_UNIFORM
        uni.max_outer = 1000        # the plain method's own cap
        sub = Batch([b.pairs[i] for i in redo], [b.ns[i] for i in redo],
                    [b.nps[i] for i in redo], b.A, b.B, b.K, b.Fa, b.Gb,
                    b.X, [b.offA[i] for i in redo], [b.offB[i] for i in redo],
                    [b.offK[i] for i in redo], [b.offF[i] for i in redo],
                    [b.offG[i] for i in redo], b.fdim)
        try:
            again = solve_batched(S, sub, uni)
        except F.FastPFPError as e:
            again = e.infos
        for i, inf in zip(redo, again):
            inf["fallback"] = 1
            infos[i] = inf
    torch.cuda.synchronize()
    return infos, {"warm_ok": int(sum(warm_ok)), "fallbacks": len(redo)}


def _torch():
    import torch
    return torch


# ---------------------------------------------------------------- training
def train_size(idx: int) -> int:
    """n = n' of training pair idx, U{100..500}."""
    return int(np.random.default_rng([1207, 1114, 41, idx]).integers(100, 501))


def _gen_train(idx: int):
    return synth.config4_pair(idx, train_size(idx), train=True)


def _generate(indices, workers: int):
    if workers <= 1:
        return [_gen_train(i) for i in indices]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        return pool.map(_gen_train, indices, chunksize=8)


def train(num_pairs: int = 20000, chunk: int = 512, epochs: int = 8,
          minibatch: int = 8, lr: float = 2e-3, lr_end: float = 1e-4,
          seed: int = 0, workers: int = 16, log=print,
          init: Optional[np.ndarray] = None) -> tuple[np.ndarray, dict]:
    """Trains the warm start; returns (parameters, training log).

    All training pairs are generated and solved once (chunks of `chunk`
    pairs stay resident on the device with their fixed points), then
    `epochs` passes of minibatch Adam run over them in a seeded random
    order, with a cosine learning-rate decay from lr to lr_end."""
    torch = _torch()
    S = F.Solver(512, 512)
    S.warmstart_load(init if init is not None else init_params(seed))
    prm = F.default_params(lambda_=1.0)
    t_start = time.perf_counter()
    chunks, hist = [], []
    for c0 in range(0, num_pairs, chunk):
        idx = list(range(c0, min(num_pairs, c0 + chunk)))
        t0 = time.perf_counter()
        pairs = _generate(idx, workers)
        t_gen = time.perf_counter() - t0
        b = pack(torch, pairs)
        b.pairs = None              # training needs only the device copies
        del pairs
        t0 = time.perf_counter()
        infos = solve_batched(S, b, prm)
        torch.cuda.synchronize()
        rec = {"targets": c0 + len(idx), "gen_s": t_gen,
               "solve_s": time.perf_counter() - t0,
               "converged": int(sum(i["converged"] for i in infos))}
        log(json.dumps(rec))
        chunks.append(b)
    items = [(c, i) for c, b in enumerate(chunks) for i in range(len(b.ns))]
    steps_total = max(1, epochs * ((len(items) + minibatch - 1) // minibatch))
    rng = np.random.default_rng([1207, 1114, 42, seed])
    step = 0
    for ep in range(epochs):
        t0 = time.perf_counter()
        order = rng.permutation(len(items))
        losses = []
        for m0 in range(0, len(order), minibatch):
            mb = order[m0:m0 + minibatch]
            S.warmstart_zero_grad()
            for k in mb:
                c, i = items[k]
                b = chunks[c]
                A = b.view(b.A, b.offA[i], b.ns[i], b.ns[i])
                B = b.view(b.B, b.offB[i], b.nps[i], b.nps[i])
                Fa, Gb = _attrs(b, i)
                losses.append(S.warmstart_grad(A, B, Fa, Gb, b.x(i)))
            frac = step / steps_total
            cur = lr_end + 0.5 * (lr - lr_end) * (1 + np.cos(np.pi * frac))
            S.warmstart_adam(cur, 0.9, 0.999, 1e-8, grad_scale=1.0 / len(mb))
            step += 1
        rec = {"epoch": ep, "loss": float(np.mean(losses)),
               "loss_last_tenth": float(np.mean(losses[-len(losses) // 10:])),
               "seconds": time.perf_counter() - t0}
        hist.append(rec)
        log(json.dumps(rec))
    params, _ = S.warmstart_get()
    del chunks
    S.close()
    return params, {"history": hist, "seconds": time.perf_counter() - t_start,
                    "num_pairs": num_pairs, "epochs": epochs,
                    "minibatch": minibatch, "lr": lr, "lr_end": lr_end,
                    "chunk": chunk}


# -------------------------------------------------------------- acceptance
def sharpened(params: np.ndarray, beta: float) -> np.ndarray:
    """The same network with its similarities divided by tau / beta
    (log tau - log beta): an inference temperature, chosen on held-out
    pairs, that sharpens X0 without changing any row's ranking."""
    p = np.array(params, dtype=np.float32, copy=True)
    p[-1] = np.float32(float(p[-1]) - np.log(beta))
    return p


def warm_params():
    """Solver parameters of the learned-start runs: BF16 products, X0 from
    the caller, eps1 above the bfloat16 plateau, a short outer cap."""
    return F.default_params(lambda_=1.0, precision=F.BF16, init=F.INIT_USER,
                            tol_outer=BF16_TOL_OUTER, max_outer=WARM_MAX_OUTER)


def run_plain(S, torch, b: Batch, prm=None, repeats: int = 1) -> dict:
    """The reference run: FP32 products from the uniform start."""
    prm = prm or F.default_params(lambda_=1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(repeats):
        infos = solve_batched(S, b, prm)
    torch.cuda.synchronize()
    return _scored(b, infos, (time.perf_counter() - t0) / repeats, {})


def run_warm(S, torch, b: Batch, params: np.ndarray, prm=None,
             repeats: int = 1) -> dict:
    """BF16 products from the learned start (uniform fallback per pair)."""
    prm = prm or warm_params()
    S.warmstart_load(params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(repeats):
        infos, extra = solve_batched_warm(S, b, prm)
    return _scored(b, infos, (time.perf_counter() - t0) / repeats, extra)


def _scored(b: Batch, infos, seconds, extra) -> dict:
    obj, acc = [], []
    for i, p in enumerate(b.pairs):
        m, _ = F.discretize(b.x(i).cpu().numpy())
        obj.append(scores.matching_objective(p.A, p.B, p.K, p.lam, m))
        acc.append(scores.accuracy(m, p.perm))
    return {"objective": obj, "accuracy": acc,
            "outer": [i["outer_iters"] for i in infos],
            "converged": int(sum(i["converged"] for i in infos)),
            "seconds": seconds, "pairs_per_s": len(b.pairs) / seconds,
            **extra}


def x0_quality(S, torch, b: Batch, params: np.ndarray) -> dict:
    """How close the learned X0 is to the planted matching: the fraction of
    rows whose largest entry sits on the planted partner, and the smallest
    and median probability the softmax gives that partner."""
    S.warmstart_load(params)
    top1, pm = [], []
    for i, p in enumerate(b.pairs):
        warm_x0(S, b, i)
        X0 = b.x(i).cpu().numpy()
        rows = np.nonzero(p.perm >= 0)[0]
        top1.append(float(np.mean(X0[rows].argmax(1) == p.perm[rows])))
        pm.append(X0[rows, p.perm[rows]])
    pm = np.concatenate(pm)
    return {"x0_top1": float(np.mean(top1)), "x0_pmatch_min": float(pm.min()),
            "x0_pmatch_median": float(np.median(pm)),
            "x0_pmatch_p01": float(np.quantile(pm, 0.01))}


def verdict(plain: dict, warm: dict) -> dict:
    """Acceptance: objective within OBJ_REL_TOL relative and accuracy within
    ACC_TOL of the plain run (means over the pairs)."""
    op, ow = np.mean(plain["objective"]), np.mean(warm["objective"])
    ap, aw = np.mean(plain["accuracy"]), np.mean(warm["accuracy"])
    ok = bool(ow >= op - OBJ_REL_TOL * abs(op) and aw >= ap - ACC_TOL)
    return {"accepted": ok, "objective_plain": float(op),
            "objective_warm": float(ow),
            "objective_rel_diff": float((ow - op) / abs(op)),
            "accuracy_plain": float(ap), "accuracy_warm": float(aw),
            "outer_plain": float(np.mean(plain["outer"])),
            "outer_warm": float(np.mean(warm["outer"])),
            "speedup": warm["pairs_per_s"] / plain["pairs_per_s"],
            "fallbacks": warm.get("fallbacks", 0)}


def evaluate(params: np.ndarray, sizes=((1000, 16),),
             betas=(1.0, 2.0, 4.0, 8.0), log=print) -> dict:
    """Held-out pairs of the config-4 model (evaluation seeds) at each
    (n, count): the plain run once, the learned start at every sharpening
    beta.  The chosen beta is the accepted one (at every size) with the
    largest smallest speedup; None if no beta is accepted."""
    torch = _torch()
    nmax = max(n for n, _ in sizes)
    S = F.Solver(nmax, nmax)
    rows = {}
    for n, count in sizes:
        b = pack(torch, [synth.config4_pair(i, n) for i in range(count)])
        plain = run_plain(S, torch, b)
        for beta in betas:
            pb = sharpened(params, beta)
            q = x0_quality(S, torch, b, pb)
            v = {**verdict(plain, run_warm(S, torch, b, pb)), **q}
            rows.setdefault(beta, {})[str(n)] = v
            log(json.dumps({"n": n, "beta": beta, **v}))
        del b
    S.close()
    best, best_speed = None, 0.0
    for beta, per in rows.items():
        if all(v["accepted"] for v in per.values()):
            sp = min(v["speedup"] for v in per.values())
            if sp > best_speed:
                best, best_speed = beta, sp
    return {"accepted": best is not None, "beta": best,
            "min_speedup": best_speed,
            "by_beta": {str(k): v for k, v in rows.items()}}


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--minibatch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--init", default=None,
                    help="continue from these raw parameters (.npy)")
    ap.add_argument("--evaluate-only", default=None,
                    help="skip training: run the acceptance check on these "
                         "raw parameters (.npy) and keep their training log "
                         "from the .json beside them")
    ap.add_argument("--eval", default="1000:16,2000:4",
                    help="held-out n:count list for the acceptance check")
    ap.add_argument("--betas", default="1,2,4,8")
    ap.add_argument("--out", default=HERE,
                    help="directory for warmstart_params.npy/.json")
    a = ap.parse_args()
    if a.evaluate_only:
        raw = np.load(a.evaluate_only, allow_pickle=False).astype(np.float32)
        with open(os.path.join(os.path.dirname(a.evaluate_only),
                               "warmstart_params.json")) as f:
            old = json.load(f)
        log = {"history": [{"loss": old["loss_first"]},
                           {"loss": old["loss_last"]}], **old["training"]}
    else:
        init = (np.load(a.init, allow_pickle=False).astype(np.float32)
                if a.init else None)
        raw, log = train(a.pairs, epochs=a.epochs, minibatch=a.minibatch,
                         lr=a.lr, workers=a.workers, init=init)
    sizes = [tuple(int(v) for v in s.split(":")) for s in a.eval.split(",")]
    betas = [float(v) for v in a.betas.split(",")]
    rep = evaluate(raw, sizes, betas)
    os.makedirs(a.out, exist_ok=True)
    beta = rep["beta"] if rep["accepted"] else 1.0
    deployed = sharpened(raw, beta)
    np.save(os.path.join(a.out, "warmstart_params.npy"), deployed)
    # the trained (unsharpened) parameters only when they differ from the
    # deployed ones
    raw_path = os.path.join(a.out, "warmstart_params_raw.npy")
    if beta != 1.0:
        np.save(raw_path, raw)
    elif os.path.exists(raw_path):
        os.remove(raw_path)
    meta = {"accepted": rep["accepted"], "beta": rep["beta"],
            "evaluation": rep,
            "training": {k: v for k, v in log.items() if k != "history"},
            "continued_from": a.init,
            "loss_first": log["history"][0]["loss"],
            "loss_last": log["history"][-1]["loss"],
            "recipe": ("config-4 model training pairs (train seeds), "
                       "n = n' ~ U{100..500}, targets = FP32 FastPFP fixed "
                       "points from the uniform start, lambda = 1")}
    with open(os.path.join(a.out, "warmstart_params.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps({"accepted": rep["accepted"], "beta": rep["beta"],
                      "min_speedup": rep["min_speedup"]}), flush=True)


if __name__ == "__main__":
    main()
