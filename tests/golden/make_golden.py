"""Writes the stored oracle results used by the full-size GPU parity tests.

    python tests/golden/make_golden.py            # all files
    python tests/golden/make_golden.py config1

Only ``oracle/`` and the seeded input generators are imported; nothing here
touches the GPU library.  Each output is a compressed .npz holding the
oracle's outer/inner iteration counts, its eps1 trace, its Hungarian matching,
objective and accuracy, and its final X in full, in a sparse form that loses
nothing the parity bound needs: every entry with |X| > TAU is stored (flat
index and float64 value), and every other entry is known to satisfy
|X| <= TAU.  A converged iterate is close to a partial permutation (at
n = 1000 about n entries are near 1 and the rest are ~1e-11), so the file is
a few kilobytes where the dense matrix would be 8 MB.  With the parity bound
|X_gpu - X_ref| <= tol, an unstored entry passes exactly when
|X_gpu| <= tol - TAU (then |X_gpu - X_ref| <= |X_gpu| + TAU <= tol).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fastpfp_oracle as O  # noqa: E402
from paper_1207_1114_amd import synth  # noqa: E402

TAU = 1e-6   # entries at or below this magnitude are not stored


def write(job: str, name: str, pair, **kw) -> None:
    t0 = time.time()
    r = O.fastpfp(pair.A, pair.B, pair.K, pair.lam, **kw)
    dt = time.time() - t0
    match = O.hungarian_discretize(r.X)
    flat = r.X.ravel()
    idx = np.flatnonzero(np.abs(flat) > TAU)
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(
        out, outer=r.outer_iters, inner=np.array(r.inner_iters),
        eps1=np.array(r.eps1_trace), match=match, shape=np.array(r.X.shape),
        tau=TAU, idx=idx.astype(np.int64), val=flat[idx], xmax=r.X.max(),
        xsum_rows=r.X.sum(1), xsum_cols=r.X.sum(0), converged=r.converged,
        seconds=dt, accuracy=O.accuracy(match, pair.perm),
        objective=O.objective(pair.A, pair.B, pair.K, pair.lam, match),
        command=f"python tests/golden/make_golden.py {job}")
    print(f"{out}: outer {r.outer_iters} inner {sum(r.inner_iters)} "
          f"acc {O.accuracy(match, pair.perm):.4f} stored {idx.size} of "
          f"{flat.size} entries ({dt:.1f} s)")


JOBS = {
    "config1": lambda: write("config1", "config1_pair0", synth.config1_pair(0)),
    "config2": lambda: write("config2", "config2_pair0", synth.config2_pair(0)),
    # configuration 4's evaluation size n = n' = 2000, plain FP32 settings
    "config4": lambda: write("config4", "config4_n2000_pair0",
                             synth.config4_pair(0, 2000)),
    # the first pair of configuration 3's ragged batch (n = 57, n' = 73)
    "config3": lambda: write("config3", "config3_pair0", synth.config3_pair(0)),
}

if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    for nm in names:
        JOBS[nm]()
