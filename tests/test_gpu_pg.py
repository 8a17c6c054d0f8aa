"""The Projected Gradient iteration (eq. pg; method = METHOD_PG) on the GPU
against the FP64 oracle's ``projected_gradient``, through the C ABI.

Same bounds as the FastPFP solves: |X_gpu - X_ref| <= 1e-4 max|X_ref|,
identical outer step counts and Hungarian matchings.
"""
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
    S = F.Solver(512, 512)
    yield torch, F, S
    S.close()


def dev(torch, a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda:0")


def _solve(env, A, B, K, lam, **kw):
    torch, F, S = env
    prm = F.default_params(method=F.METHOD_PG, normalize_max=0, lambda_=lam,
                           **kw)
    X = torch.zeros(A.shape[0], B.shape[0], device="cuda:0")
    info = S.solve(dev(torch, A), dev(torch, B),
                   dev(torch, K) if lam > 0 else None, X, prm)
    return X.cpu().numpy().astype(np.float64), info


def _assert_parity(X, info, ref):
    err = np.abs(X - ref.X).max()
    print(f"outer {info['outer_iters']} (oracle {ref.outer_iters}) "
          f"max|dX| {err:.2e}")
    assert info["outer_iters"] == ref.outer_iters
    assert err <= 1e-4 * np.abs(ref.X).max()
    np.testing.assert_array_equal(O.hungarian_discretize(X),
                                  O.hungarian_discretize(ref.X))


@pytest.mark.parametrize("step", [0.05, 0.5])
def test_pg_parity_config0(env, step):
    """Attributed pair (lambda > 0), default start, no step 9."""
    p = synth.config0_pair(0)
    X, info = _solve(env, p.A, p.B, p.K, p.lam, alpha=step)
    ref = O.projected_gradient(p.A, p.B, p.K, p.lam, step)
    assert info["converged"] == ref.converged
    _assert_parity(X, info, ref)


@pytest.mark.parametrize("flips,deletion", [(False, False), (True, True)])
@pytest.mark.parametrize("projection", ["alternating", "dykstra"])
def test_pg_parity_sec51(env, flips, deletion, projection):
    torch, F, S = env
    p = synth.paper_synthetic_pair(0, 64, flips, deletion)
    c = 1.0 / (p.n * p.np_)
    proj = {"alternating": F.ALTERNATING, "dykstra": F.DYKSTRA}[projection]
    X, info = _solve(env, p.A, p.B, None, 0.0, alpha=0.1, init_scale=c,
                     projection=proj)
    ref = O.projected_gradient(p.A, p.B, None, 0.0, 0.1,
                               X0=O.uniform_x0(p.n, p.np_, c),
                               projection=projection)
    assert info["converged"] and ref.converged
    _assert_parity(X, info, ref)


def test_pg_linear_objective_reaches_the_assignment(env):
    """A = A' = 0: PG with the exact projection converges to the optimal
    assignment of K (scipy), 30 x 40."""
    from scipy.optimize import linear_sum_assignment
    torch, F, S = env
    rng = np.random.default_rng(53)
    n, m = 30, 40
    K = rng.random((n, m))
    X, info = _solve(env, np.zeros((n, n)), np.zeros((m, m)), K, 1.0,
                     alpha=2.0, projection=F.DYKSTRA, tol_inner=1e-7,
                     max_inner=20_000)
    ri, ci = linear_sum_assignment(K, maximize=True)
    P = np.zeros((n, m))
    P[ri, ci] = 1.0
    print(f"outer {info['outer_iters']} max|X - P| {np.abs(X - P).max():.2e}")
    assert info["converged"]
    assert np.abs(X - P).max() <= 1e-3


def test_pg_argument_checks(env):
    torch, F, S = env
    A = dev(torch, np.zeros((4, 4)))
    X = torch.zeros(4, 4, device="cuda:0")
    # a PG step above 1 is valid; FastPFP's alpha must lie in (0, 1]
    S.solve(A, A, None, X, F.default_params(method=F.METHOD_PG, alpha=3.0,
                                            max_outer=2))
    for kw in ({"alpha": 3.0}, {"method": 7},
               {"method": F.METHOD_PG, "alpha": 0.0},
               {"method": F.METHOD_PG, "alpha": float("inf")}):
        with pytest.raises(F.FastPFPError):
            S.solve(A, A, None, X, F.default_params(max_outer=2, **kw))


def test_pg_with_bf16_products_matches_recipe_oracle(env):
    """PG with BF16 products against the oracle running the same bfloat16
    recipe: one bfloat16 ulp of the largest entry, as for FastPFP."""
    torch, F, S = env
    rng = synth.rng_for(98, 70 * 1000 + 90 + 11)
    A = synth.random_weighted_graph(rng, 70, 0.3)
    B = synth.random_weighted_graph(rng, 90, 0.3)
    K = rng.random((70, 90))
    kw = dict(max_outer=5, max_inner=120)
    X, info = _solve(env, A, B, K, 0.5, alpha=0.1, precision=F.BF16, **kw)
    ref = O.projected_gradient(A, B, K, 0.5, 0.1, products="bf16", **kw)
    assert np.abs(X - ref.X).max() <= 2.0 ** -8 * np.abs(ref.X).max()
    assert info["outer_iters"] == ref.outer_iters
