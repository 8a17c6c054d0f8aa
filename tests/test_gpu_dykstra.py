"""The exact projection (Dykstra's algorithm, projection = DYKSTRA) on the GPU
against the FP64 oracle's ``dykstra_inner`` and ``fastpfp(projection=
"dykstra")``, through the C ABI.

Tolerances as for the alternating path: float32 rounding per pass, damped by
the projection's non-expansiveness, so |Y_gpu - Y_ref| <= 1e-4 max|Y_ref| for
projections and |X_gpu - X_ref| <= 1e-4 max|X_ref| plus identical outer step
counts and Hungarian matchings for solves.
"""
import itertools

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
    S = F.Solver(1024, 1024)
    yield torch, F, S
    S.close()


def dev(torch, a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda:0")


@pytest.mark.parametrize("N,T,team", [(1, 5, 0), (2, 40, 0), (17, 120, 0),
                                      (129, 60, 0), (200, 30, 0),
                                      (257, 40, 0), (300, 40, 0),
                                      (300, 40, 16), (470, 30, 0),
                                      (513, 30, 0), (900, 20, 0),
                                      (1000, 20, 0)])
def test_dykstra_projection_parity(env, N, T, team):
    torch, F, S = env
    rng = np.random.default_rng([N, T, 7])
    Y = rng.normal(size=(N, N)) * 2.0 + 0.5
    Yg = dev(torch, Y)
    info = S.project(Yg, 1e-30, T, team, projection=F.DYKSTRA)
    ref = O.dykstra_inner(Y, 1e-30, T)
    got = Yg.cpu().numpy()
    scale = max(1.0, np.abs(ref.Y).max())
    err = np.abs(got - ref.Y).max()
    print(f"N={N} T={T} team={team}: max|dY| {err:.2e} "
          f"passes {info['inner_iters_total']} (oracle {ref.iters})")
    assert err <= 1e-4 * scale
    assert np.all(got >= 0)
    # both stop early only on an exact fixed point (max|dY| = 0 < 1e-30),
    # which float32 rounding may reach a pass before or after float64
    it = info["inner_iters_total"]
    # an early stop is only allowed on an exact float32 fixed point
    # (max|dY| = 0), which float64 may reach a little later or not at all
    assert it == ref.iters or (info["eps2_last"] == 0.0 and (
        it < ref.iters or (ref.converged and it - ref.iters <= 2)))


def _certificate(Y, D):
    """max over permutation matrices Z of <Y - D, Z - D> (<= 0 iff D is the
    nearest doubly stochastic matrix, D feasible)."""
    N = Y.shape[0]
    worst = -np.inf
    for p in itertools.permutations(range(N)):
        Z = np.zeros((N, N))
        Z[np.arange(N), p] = 1.0
        worst = max(worst, float(np.sum((Y - D) * (Z - D))))
    return worst


def test_dykstra_reaches_the_nearest_point_alternation_does_not(env):
    torch, F, S = env
    rng = np.random.default_rng(17)
    rng.normal(size=(4, 4))         # the oracle pin's second draw
    Y = rng.normal(size=(4, 4)) * 2
    out = {}
    for proj in (F.ALTERNATING, F.DYKSTRA):
        Yg = dev(torch, Y)
        info = S.project(Yg, 1e-7, 200_000, projection=proj)
        D = Yg.cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(D.sum(0), 1.0, atol=1e-5)
        np.testing.assert_allclose(D.sum(1), 1.0, atol=1e-5)
        out[proj] = _certificate(Y, D)
        print(f"projection {proj}: passes {info['inner_iters_total']} "
              f"certificate {out[proj]:.2e}")
    assert out[F.DYKSTRA] <= 1e-4
    assert out[F.ALTERNATING] > 1e-2


def _solve(env, p, **kw):
    torch, F, S = env
    prm = F.default_params(projection=F.DYKSTRA, **kw)
    A, B = dev(torch, p.A), dev(torch, p.B)
    K = dev(torch, p.K) if (p.K is not None and prm.lambda_ > 0) else None
    X = torch.zeros(p.n, p.np_, device="cuda:0")
    info = S.solve(A, B, K, X, prm)
    return X.cpu().numpy().astype(np.float64), info


def _assert_parity(X, info, ref):
    err = np.abs(X - ref.X).max()
    print(f"outer {info['outer_iters']} (oracle {ref.outer_iters}) "
          f"max|dX| {err:.2e}")
    assert info["outer_iters"] == ref.outer_iters
    assert err <= 1e-4 * np.abs(ref.X).max()
    np.testing.assert_array_equal(O.hungarian_discretize(X),
                                  O.hungarian_discretize(ref.X))


def test_dykstra_solve_parity_config0(env):
    """Attributed pair (lambda > 0), default start."""
    p = synth.config0_pair(0)
    X, info = _solve(env, p, lambda_=p.lam)
    ref = O.fastpfp(p.A, p.B, p.K, p.lam, projection="dykstra")
    assert info["converged"] and ref.converged
    _assert_parity(X, info, ref)


@pytest.mark.parametrize("flips,deletion", [(False, False), (True, False),
                                            (False, True), (True, True)])
def test_dykstra_solve_parity_sec51(env, flips, deletion):
    """The synthetic benchmark's four cases at n = 64 (58 x 64 with node
    deletion) from the recommended start X0 = 1 1^T / (n n')."""
    p = synth.paper_synthetic_pair(0, 64, flips, deletion)
    c = 1.0 / (p.n * p.np_)
    X, info = _solve(env, p, lambda_=0.0, init_scale=c)
    ref = O.fastpfp(p.A, p.B, None, 0.0, X0=O.uniform_x0(p.n, p.np_, c),
                    projection="dykstra")
    assert info["converged"] and ref.converged
    _assert_parity(X, info, ref)


@pytest.mark.parametrize("n,m", [(70, 90), (90, 70)])
def test_dykstra_with_bf16_products_matches_recipe_oracle(env, n, m):
    """BF16 products with the exact projection against the oracle running
    the same bfloat16 recipe; one bfloat16 ulp of the largest entry, as for
    the alternating projection."""
    torch, F, S = env
    rng = synth.rng_for(98, n * 1000 + m + 7)
    A = synth.random_weighted_graph(rng, n, 0.3)
    B = synth.random_weighted_graph(rng, m, 0.3)
    K = rng.random((n, m))
    p = synth.GraphPair(A, B, K, 0.5, np.full(n, -1))
    kw = dict(max_outer=5, max_inner=120)
    X, info = _solve(env, p, lambda_=0.5, precision=F.BF16, **kw)
    ref = O.fastpfp(A, B, K, 0.5, products="bf16", projection="dykstra", **kw)
    assert np.abs(X - ref.X).max() <= 2.0 ** -8 * np.abs(ref.X).max()
    assert info["outer_iters"] == ref.outer_iters


@pytest.mark.parametrize("method", ["dykstra", "pg"])
def test_batched_equals_single_for_the_variants(env, method):
    """A ragged batch with the exact projection or the PG iteration gives
    every pair bit for bit what a solve of that pair alone gives."""
    torch, F, S = env
    pairs = [synth.config3_pair(i) for i in range(4)]
    pairs += [synth.config3_pair(100, n=50, n_extra=0),
              synth.config3_pair(101, n=300, n_extra=40)]
    kw = dict(lambda_=1.0, max_outer=6, max_inner=150, team_size=16)
    if method == "dykstra":
        kw["projection"] = F.DYKSTRA
    else:
        kw.update(method=F.METHOD_PG, alpha=0.05, normalize_max=0)
    prm = F.default_params(**kw)
    offs = {k: [] for k in "ABKX"}
    bufs = {k: [] for k in "ABKX"}
    cur = {k: 0 for k in "ABKX"}
    for p in pairs:
        for k, mtx in dict(A=p.A, B=p.B, K=p.K,
                           X=np.zeros((p.n, p.np_))).items():
            offs[k].append(cur[k])
            bufs[k].append(np.asarray(mtx, np.float32).ravel())
            cur[k] += mtx.size
    d = {k: dev(torch, np.concatenate(v)).view(-1, 1)
         for k, v in bufs.items()}
    infos = S.solve_batched([p.n for p in pairs], [p.np_ for p in pairs],
                            d["A"], offs["A"], d["B"], offs["B"], d["K"],
                            offs["K"], d["X"], offs["X"], prm)
    Xall = d["X"].cpu().numpy().ravel()
    for p, o, inf in zip(pairs, offs["X"], infos):
        Xs = torch.zeros(p.n, p.np_, device="cuda:0")
        info = S.solve(dev(torch, p.A), dev(torch, p.B), dev(torch, p.K), Xs,
                       prm)
        np.testing.assert_array_equal(
            Xall[o:o + p.n * p.np_].reshape(p.n, p.np_), Xs.cpu().numpy())
        assert inf["outer_iters"] == info["outer_iters"]
        assert inf["inner_iters_total"] == info["inner_iters_total"]
