"""What the trained warm start gains over the method without it.

Held-out pairs of the config-4 model (evaluation seeds 100-107, outside the
pairs the acceptance check used) at n = 1000 are solved three ways: the
plain method (FP32 products, uniform start, eps1 = 1e-6) -- the reference; BF16
products from the uniform start; and BF16 products from the shipped learned
start (both with the BF16 eps1).  The learned start must match the reference's
objective (1e-3 relative) and accuracy (0.5 pp) with at most 0.6 of its
outer steps (about half were measured), and take fewer outer steps than the uniform start at the same
precision, which isolates what the network itself contributes.
"""
import numpy as np
import pytest

from paper_1207_1114_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def runs():
    import torch
    from paper_1207_1114_amd import fastpfp as F
    from paper_1207_1114_amd import warmstart as W
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    params, meta = W.load_params()
    S = F.Solver(1000, 1000)
    b = W.pack(torch, [synth.config4_pair(i, 1000) for i in range(100, 108)])
    bf16_uniform = F.default_params(lambda_=1.0, precision=F.BF16,
                                    tol_outer=W.BF16_TOL_OUTER)
    out = {"uniform_bf16": W.run_plain(S, torch, b, bf16_uniform),
           "plain_fp32": W.run_plain(S, torch, b),
           "warm_bf16": W.run_warm(S, torch, b, params)}
    S.close()
    return W, out


def test_learned_start_beats_the_uniform_start_at_the_same_precision(runs):
    W, r = runs
    uni, warm = r["uniform_bf16"], r["warm_bf16"]
    v = W.verdict(uni, warm)
    assert v["accepted"], v
    assert np.mean(warm["outer"]) < np.mean(uni["outer"]), v
    assert warm["converged"] == len(warm["outer"])
    assert warm.get("fallbacks", 0) == 0


def test_learned_start_matches_the_plain_fp32_reference(runs):
    W, r = runs
    v = W.verdict(r["plain_fp32"], r["warm_bf16"])
    assert v["accepted"], v
    assert v["outer_warm"] <= 0.6 * v["outer_plain"], v
