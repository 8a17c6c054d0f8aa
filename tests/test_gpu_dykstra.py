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
                                      (129, 60, 0), (257, 40, 0),
                                      (300, 40, 0), (300, 40, 16),
                                      (513, 30, 0), (1000, 20, 0)])
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
    assert it == ref.iters or (info["eps2_last"] == 0.0 and ref.converged
                               and abs(it - ref.iters) <= 2)


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
