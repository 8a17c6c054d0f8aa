"""Configuration 4's evaluation size on the GPU: n = n' = 2000, Bernoulli(0.05)
graphs with noise 0.05 and the configuration-1 attribute model.

* The plain method (FP32 products, uniform start, eps1 = 1e-6) against the
  stored FP64 oracle run of pair 0: every entry within 1e-4 max X, the same
  Hungarian matching, the eps1 trace and the outer step count.
* BF16 products from the learned warm start against the plain run on four
  held-out pairs: the acceptance rule of the learned start (mean objective
  within 1e-3 relative, mean matching accuracy within 0.5 pp), fewer outer
  steps, and the BF16 iterate's error against the FP64 oracle on pair 0.
"""
import os

import numpy as np
import pytest

from oracle import fastpfp_oracle as O
from paper_1207_1114_amd import synth
from parity_util import BF16_X_ERR, assert_full_parity, full_error

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
N = 2000


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1207_1114_amd import fastpfp as F
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    S = F.Solver(N, N)
    yield torch, F, S
    S.close()


def test_config4_n2000_fp32_every_entry_against_stored_oracle(env):
    torch, F, S = env
    g = np.load(os.path.join(GOLD, "config4_n2000_pair0.npz"))
    p = synth.config4_pair(0, N)
    dev = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda:0")
    X = torch.zeros(N, N, device="cuda:0")
    info = S.solve(dev(p.A), dev(p.B), dev(p.K), X,
                   F.default_params(lambda_=p.lam))
    Xh = X.cpu().numpy().astype(np.float64)
    tr, ref = S.trace(), g["eps1"]
    print("eps1 gpu   ", " ".join(f"{v:.3e}" for v in tr))
    print("eps1 oracle", " ".join(f"{v:.3e}" for v in ref))
    # eps1 is a max of differences of entries near 1 that carry float32
    # rounding of ~1000 passes per step (a few 1e-6): agreement to 1e-5
    k = min(len(tr), len(ref))
    assert np.all(np.abs(tr[:k] - ref[:k]) <= 1e-5 + 1e-3 * ref[:k])
    assert abs(info["outer_iters"] - int(g["outer"])) <= 1
    assert info["converged"] == 1
    assert_full_parity(Xh, g)
    np.testing.assert_array_equal(O.hungarian_discretize(Xh), g["match"])


def test_config4_n2000_bf16_learned_start_acceptance(env):
    torch, F, S = env
    from paper_1207_1114_amd import warmstart as W
    params, meta = W.load_params()
    b = W.pack(torch, [synth.config4_pair(i, N) for i in range(4)])
    plain = W.run_plain(S, torch, b)
    X_plain0 = b.x(0).cpu().numpy().astype(np.float64)
    warm = W.run_warm(S, torch, b, params)
    X_warm0 = b.x(0).cpu().numpy().astype(np.float64)
    v = W.verdict(plain, warm)
    g = np.load(os.path.join(GOLD, "config4_n2000_pair0.npz"))
    e_plain = full_error(X_plain0, g)[2]
    e_warm = full_error(X_warm0, g)[2]
    print(f"n={N}: plain FP32 outer {v['outer_plain']:.2f} acc "
          f"{v['accuracy_plain']:.4f}; BF16 + learned start outer "
          f"{v['outer_warm']:.2f} acc {v['accuracy_warm']:.4f} objective "
          f"rel diff {v['objective_rel_diff']:.2e} fallbacks "
          f"{v['fallbacks']}; pair 0 max|X - X_fp64|: FP32 {e_plain:.2e}, "
          f"BF16 + learned start {e_warm:.2e}")
    assert v["accepted"], v
    assert v["outer_warm"] < v["outer_plain"], v
    assert warm["converged"] == len(b.pairs)
    assert e_plain <= 1e-4 * float(g["xmax"])
    assert e_warm <= BF16_X_ERR * float(g["xmax"])
