"""Device greedy discretisation (fastpfp_discretize_greedy_batched) against
the host rule (fastpfp_discretize, FASTPFP_GREEDY) and the FP64 oracle's
greedy_discretize: matchings must be identical, entry for entry, including
the tie-break (equal values go to the smaller row-major index)."""
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
    S = F.Solver(1200, 1200)
    yield torch, F, S
    S.close()


def _device(env, X):
    torch, F, S = env
    Xd = torch.tensor(np.asarray(X, np.float32), device="cuda:0")
    return S.discretize_greedy(Xd).cpu().numpy()


def _host(env, X):
    torch, F, S = env
    m, _ = F.discretize(np.asarray(X, np.float32), F.GREEDY)
    return m


def _check(env, X):
    X32 = np.asarray(X, np.float32)
    got = _device(env, X32)
    np.testing.assert_array_equal(got, _host(env, X32))
    np.testing.assert_array_equal(
        got, O.greedy_discretize(X32.astype(np.float64)))
    return got


@pytest.mark.parametrize("n,m", [(1, 1), (1, 7), (7, 1), (5, 8), (8, 5),
                                 (64, 64), (300, 257), (257, 300),
                                 (1000, 1000)])
def test_random_matrices(env, n, m):
    rng = np.random.default_rng([n, m, 61])
    _check(env, rng.random((n, m)))


def test_ties_zeros_and_negatives(env):
    rng = np.random.default_rng(67)
    _check(env, rng.integers(0, 3, size=(120, 90)).astype(np.float32))
    X = rng.normal(size=(80, 100)).astype(np.float32)
    X[rng.random(X.shape) < 0.3] = 0.0
    X[rng.random(X.shape) < 0.1] = -0.0
    _check(env, X)
    _check(env, -rng.random((50, 40)))


def test_all_equal_entries(env):
    """Every entry ties: the rule matches row i to column i (smallest
    index first), the longest proposal chains the device path can see."""
    got = _check(env, np.full((200, 230), 0.25))
    np.testing.assert_array_equal(got, np.arange(200))


def test_on_solver_output(env):
    torch, F, S = env
    p = synth.config0_pair(0)
    dev = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda:0")
    X = torch.zeros(p.n, p.np_, device="cuda:0")
    K = dev(p.K) if p.K is not None and p.lam > 0 else None
    S.solve(dev(p.A), dev(p.B), K, X, F.default_params(lambda_=p.lam))
    got = S.discretize_greedy(X).cpu().numpy()
    Xh = X.cpu().numpy()
    np.testing.assert_array_equal(got, _host(env, Xh))
    assert O.accuracy(got, p.perm) == 1.0


def test_ragged_batch_and_a_non_finite_pair(env):
    torch, F, S = env
    rng = np.random.default_rng(71)
    shapes = [(int(rng.integers(1, 400)), int(rng.integers(1, 400)))
              for _ in range(20)]
    mats = [rng.random(s).astype(np.float32) for s in shapes]
    mats[7][3, 4] = np.nan
    offX = np.cumsum([0] + [a.size for a in mats[:-1]]).tolist()
    offM = np.cumsum([0] + [s[0] for s in shapes[:-1]]).tolist()
    Xd = torch.tensor(np.concatenate([a.ravel() for a in mats]),
                      device="cuda:0")
    match = torch.zeros(sum(s[0] for s in shapes), dtype=torch.int32,
                        device="cuda:0")
    with pytest.raises(F.FastPFPError) as e:
        S.discretize_greedy_batched([s[0] for s in shapes],
                                    [s[1] for s in shapes], Xd, offX, match,
                                    offM)
    st = e.value.statuses
    assert st[7] == 5 and all(s == 0 for k, s in enumerate(st) if k != 7)
    got = match.cpu().numpy()
    for k, (a, s) in enumerate(zip(mats, shapes)):
        mk = got[offM[k]:offM[k] + s[0]]
        if k == 7:
            assert np.all(mk == -1)
        else:
            np.testing.assert_array_equal(mk, _host(env, a))
    # the same batch without the bad entry, twice: repeatable and complete
    mats[7][3, 4] = 0.5
    Xd = torch.tensor(np.concatenate([a.ravel() for a in mats]),
                      device="cuda:0")
    for _ in range(2):
        assert S.discretize_greedy_batched(
            [s[0] for s in shapes], [s[1] for s in shapes], Xd, offX,
            match, offM) == [0] * len(shapes)
        got = match.cpu().numpy()
        for k, (a, s) in enumerate(zip(mats, shapes)):
            np.testing.assert_array_equal(got[offM[k]:offM[k] + s[0]],
                                          _host(env, a))


def test_argument_errors(env):
    torch, F, S = env
    X = torch.zeros(4, device="cuda:0")
    m = torch.zeros(2, dtype=torch.int32, device="cuda:0")
    with pytest.raises(F.FastPFPError):
        S.discretize_greedy_batched([2000], [2], X, [0], m, [0])
    with pytest.raises(F.FastPFPError):
        S.discretize_greedy_batched([0], [2], X, [0], m, [0])
    with pytest.raises(TypeError):
        S.discretize_greedy_batched([2], [2], X, [0], m.float(), [0])
