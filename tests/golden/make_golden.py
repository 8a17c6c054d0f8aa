"""Writes the stored oracle results used by the full-size GPU parity tests.

    python tests/golden/make_golden.py            # all files
    python tests/golden/make_golden.py config1

Only ``oracle/`` and the seeded input generators are imported; nothing here
touches the GPU library.  Each output is a compressed .npz holding the
oracle's outer/inner iteration counts, its eps1 trace, its Hungarian matching,
and the final X at a fixed seeded sample of positions (the full 1000 x 1000
iterate would be 8 MB).
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

SAMPLES = 20000


def sample_positions(n: int, m: int, k: int = SAMPLES) -> tuple:
    rng = np.random.default_rng([1207, 1114, 777, n, m])
    return rng.integers(0, n, size=k), rng.integers(0, m, size=k)


def write(name: str, pair, **kw) -> None:
    t0 = time.time()
    r = O.fastpfp(pair.A, pair.B, pair.K, pair.lam, **kw)
    dt = time.time() - t0
    match = O.hungarian_discretize(r.X)
    ii, jj = sample_positions(pair.n, pair.np_)
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(
        out, outer=r.outer_iters, inner=np.array(r.inner_iters),
        eps1=np.array(r.eps1_trace), match=match, rows=ii, cols=jj,
        xs=r.X[ii, jj], xmax=r.X.max(), xsum_rows=r.X.sum(1),
        xsum_cols=r.X.sum(0), converged=r.converged, seconds=dt,
        accuracy=O.accuracy(match, pair.perm),
        objective=O.objective(pair.A, pair.B, pair.K, pair.lam, match))
    print(f"{out}: outer {r.outer_iters} inner {sum(r.inner_iters)} "
          f"acc {O.accuracy(match, pair.perm):.4f} ({dt:.1f} s)")


JOBS = {
    "config1": lambda: write("config1_pair0", synth.config1_pair(0)),
    "config2": lambda: write("config2_pair0", synth.config2_pair(0)),
}

if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    for nm in names:
        JOBS[nm]()
