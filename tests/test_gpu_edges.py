"""Edge cases of the solver through the C ABI: empty and single-node
problems, graphs with no edges, the largest supported size (N = 4096, one
team of 256 workgroups) and one beyond it.  Tolerances as in the parity
tests: |X_gpu - X_ref| <= 1e-4 max|X_ref|."""
import numpy as np
import pytest

from oracle import fastpfp_oracle as O
from paper_1207_1114_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1207_1114_amd import fastpfp as F
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, F


def dev(torch, a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda:0")


def solve(torch, F, S, A, B, K, lam, X0=None, **kw):
    n, m = A.shape[0], B.shape[0]
    X = dev(torch, X0) if X0 is not None else torch.zeros(n, m,
                                                           device="cuda:0")
    prm = F.default_params(lambda_=lam, **kw)
    info = S.solve(dev(torch, A), dev(torch, B),
                   dev(torch, K) if K is not None else None, X, prm)
    return X.cpu().numpy().astype(np.float64), info


def test_empty_inputs_are_shape_errors(env):
    torch, F = env
    S = F.Solver(16, 16)
    z = torch.zeros(0, 0, device="cuda:0")
    one = torch.zeros(1, 1, device="cuda:0")
    with pytest.raises(F.FastPFPError) as e:
        S.solve(z, one, None, torch.zeros(0, 1, device="cuda:0"),
                F.default_params())
    assert e.value.status == 2
    with pytest.raises(F.FastPFPError) as e:
        S.project(z, 1e-6, 5)
    assert e.value.status == 2
    S.warmstart_load(np.zeros(F.WS_NPARAMS, np.float32))
    with pytest.raises(F.FastPFPError) as e:
        S.warmstart(z, one, None, None, torch.zeros(0, 1, device="cuda:0"))
    assert e.value.status == 2
    S.close()


@pytest.mark.parametrize("n,m", [(1, 1), (1, 5), (5, 1), (2, 3)])
def test_tiny_problems_match_oracle(env, n, m):
    torch, F = env
    S = F.Solver(8, 8)
    rng = np.random.default_rng([n, m, 11])
    A = synth.random_weighted_graph(rng, n, 0.7)
    B = synth.random_weighted_graph(rng, m, 0.7)
    K = rng.random((n, m))
    X, info = solve(torch, F, S, A, B, K, 1.0)
    ref = O.fastpfp(A, B, K, 1.0)
    assert info["status"] == 0 and info["converged"] == int(ref.converged)
    assert np.abs(X - ref.X).max() <= 1e-4 * np.abs(ref.X).max()
    # slow tiny problems (ratio ~0.7 per step) may cross eps1 a step apart
    assert abs(info["outer_iters"] - ref.outer_iters) <= 2
    S.close()


def test_graphs_without_edges_give_the_uniform_fixed_point(env):
    """A = B = 0, lambda = 0: the gradient is 0, its projection is 1/N
    everywhere, and after step 9 every entry of X is 1."""
    torch, F = env
    S = F.Solver(64, 64)
    n, m = 40, 52
    X, info = solve(torch, F, S, np.zeros((n, n)), np.zeros((m, m)), None,
                    0.0)
    ref = O.fastpfp(np.zeros((n, n)), np.zeros((m, m)), None, 0.0)
    assert info["converged"] == 1 and ref.converged
    assert info["outer_iters"] == ref.outer_iters
    np.testing.assert_allclose(X, 1.0, atol=1e-6)
    np.testing.assert_allclose(ref.X, 1.0, atol=1e-12)
    S.close()


def test_largest_supported_size(env):
    """N = 4096 (one team of 256 workgroups, 256 x 256 tiles): one outer
    step with 10 inner passes against the oracle on every entry."""
    torch, F = env
    n = 4096
    p = synth.config4_pair(7, n)
    S = F.Solver(n, n)
    kw = dict(max_outer=1, max_inner=10, tol_outer=1e-30)
    X, info = solve(torch, F, S, p.A, p.B, p.K, p.lam, **kw)
    A32, B32, K32 = (np.asarray(a, np.float32).astype(np.float64)
                     for a in (p.A, p.B, p.K))
    ref = O.fastpfp(A32, B32, K32, p.lam, eps1=1e-30, max_outer=1,
                    max_inner=10)
    assert info["status"] == 0 and info["inner_iters_total"] == 10
    assert np.abs(X - ref.X).max() <= 1e-4 * np.abs(ref.X).max()
    S.close()


def test_bf16_products_at_n4000_against_recipe_oracle(env):
    """Configuration 4's largest size with BF16 products: one team of 256
    workgroups (T = A X in 128 x 256 output tiles handed to the XCDs in
    8 x 4 blocks, the second product in 128 x 128 tiles in 4 x 8 blocks), a
    random start X0 so that every output tile differs, two outer
    steps of 10 inner passes, against the oracle's bfloat16 recipe on every
    entry (one bfloat16 ulp of the largest entry, as in the small recipe
    tests)."""
    torch, F = env
    n = 4000
    p = synth.config4_pair(11, n)
    rng = synth.rng_for(4000, 11)
    X0 = rng.random((n, n))
    S = F.Solver(n, n)
    kw = dict(max_outer=2, max_inner=10, tol_outer=1e-30)
    X, info = solve(torch, F, S, p.A, p.B, p.K, p.lam, X0=X0,
                    init=F.INIT_USER, precision=F.BF16, **kw)
    A32, B32, K32, X032 = (np.asarray(a, np.float32).astype(np.float64)
                           for a in (p.A, p.B, p.K, X0))
    ref = O.fastpfp(A32, B32, K32, p.lam, eps1=1e-30, max_outer=2,
                    max_inner=10, X0=X032, products="bf16")
    print(f"n={n} BF16: max|X - ref| {np.abs(X - ref.X).max():.3e}, "
          f"max|ref| {np.abs(ref.X).max():.3e}", flush=True)
    assert info["status"] == 0 and info["inner_iters_total"] == 20
    assert np.abs(X - ref.X).max() <= 2.0 ** -8 * np.abs(ref.X).max()
    S.close()


def test_beyond_the_largest_team_is_unsupported(env):
    torch, F = env
    S = F.Solver(4097, 4097)
    A = torch.zeros(4097, 4097, device="cuda:0")
    X = torch.zeros(4097, 4097, device="cuda:0")
    with pytest.raises(F.FastPFPError) as e:
        S.solve(A, A, None, X, F.default_params())
    assert e.value.status == 7
    S.close()
