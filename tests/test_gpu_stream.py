"""The streaming projection (fastpfp_project_stream: steps 4-7 with Y in
device memory, any N) against the FP64 oracle, through the C ABI.  Same
bounds as the on-chip projection: |Y_gpu - Y_ref| <= 1e-4 max|Y_ref| and equal
pass counts (or both at an exact fixed point)."""
import numpy as np
import pytest

from oracle import fastpfp_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1207_1114_amd import fastpfp as F
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    S = F.Solver(4100, 4100)
    yield torch, F, S
    S.close()


def dev(torch, a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda:0")


def _cmp(info, got, ref):
    scale = max(1.0, np.abs(ref.Y).max())
    err = np.abs(got - ref.Y).max()
    it = info["inner_iters_total"]
    print(f"max|dY| {err:.2e} passes {it} (oracle {ref.iters})")
    assert err <= 1e-4 * scale
    assert np.all(got >= 0)
    # an early stop is only allowed on an exact float32 fixed point
    # (max|dY| = 0), which float64 may reach a little later or not at all
    assert it == ref.iters or (info["eps2_last"] == 0.0 and (
        it < ref.iters or (ref.converged and it - ref.iters <= 2)))


@pytest.mark.parametrize("N,T", [(1, 5), (2, 40), (17, 120), (300, 40),
                                 (1000, 20), (1500, 15), (2049, 10)])
@pytest.mark.parametrize("projection", ["alternating", "dykstra"])
def test_stream_parity(env, N, T, projection):
    torch, F, S = env
    rng = np.random.default_rng([N, T, 11])
    Y = rng.normal(size=(N, N)) * 2.0 + 0.5
    Yg = dev(torch, Y)
    proj = {"alternating": F.ALTERNATING, "dykstra": F.DYKSTRA}[projection]
    info = S.project_stream(Yg, 1e-30, T, projection=proj)
    inner = {"alternating": O.inner_projection,
             "dykstra": O.dykstra_inner}[projection]
    _cmp(info, Yg.cpu().numpy(), inner(Y, 1e-30, T))


def test_stream_stopping_rule(env):
    torch, F, S = env
    Y = np.array([[3.0, -1.0], [0.5, 2.5]])
    Yg = dev(torch, Y)
    info = S.project_stream(Yg, 1e-6, 10_000)
    ref = O.inner_projection(Y, 1e-6, 10_000)
    assert info["converged"] == 1
    assert info["inner_iters_total"] == ref.iters
    np.testing.assert_allclose(Yg.cpu().numpy(), ref.Y, atol=1e-6)


def test_large_n_routes_to_the_stream(env):
    """N = 4100 fits no on-chip team: fastpfp_project streams it."""
    torch, F, S = env
    N, T = 4100, 4
    rng = np.random.default_rng(13)
    Y = rng.random((N, N)).astype(np.float32)
    Yg = dev(torch, Y)
    info = S.project(Yg, 1e-30, T)
    _cmp(info, Yg.cpu().numpy(), O.inner_projection(Y.astype(np.float64),
                                                    1e-30, T))


def test_stream_non_finite_input(env):
    torch, F, S = env
    Y = np.ones((40, 40))
    Y[3, 5] = np.inf
    with pytest.raises(F.FastPFPError) as e:
        S.project_stream(dev(torch, Y), 1e-6, 10)
    assert e.value.status == 5


def test_large_n_exact_projection_routes_to_the_stream(env):
    torch, F, S = env
    N, T = 4100, 3
    rng = np.random.default_rng(17)
    Y = (rng.random((N, N)) * 2.0 - 0.5).astype(np.float32)
    Yg = dev(torch, Y)
    info = S.project(Yg, 1e-30, T, projection=F.DYKSTRA)
    _cmp(info, Yg.cpu().numpy(), O.dykstra_inner(Y.astype(np.float64),
                                                 1e-30, T))


@pytest.mark.parametrize("N,T,projection", [(6000, 3, "alternating"),
                                            (8200, 3, "alternating"),
                                            (6000, 2, "dykstra")])
def test_stream_parity_past_the_cache(N, T, projection):
    """Matrices larger than half (N = 6000, 144 MB) and than all (N = 8200,
    269 MB) of the 256 MiB last-level cache: the pass reads Y with
    non-temporal loads, and at 8200 also writes it with non-temporal stores.
    Both sizes leave ragged tiles (N % 64 and N % 1024 are not 0), so the
    bounds-checked edge path runs beside the unchecked one.  (Dykstra's pass
    takes the same accesses with other arithmetic; its float64 oracle is too
    slow for more than two passes at N = 6000 here.)"""
    import torch
    from paper_1207_1114_amd import fastpfp as F
    rng = np.random.default_rng([N, 23])
    Y = (rng.random((N, N)) * 2.0 - 0.5).astype(np.float32)
    proj = {"alternating": F.ALTERNATING, "dykstra": F.DYKSTRA}[projection]
    inner = {"alternating": O.inner_projection,
             "dykstra": O.dykstra_inner}[projection]
    S = F.Solver(N, N)
    try:
        Yg = dev(torch, Y)
        info = S.project_stream(Yg, 1e-30, T, projection=proj)
        got = Yg.cpu().numpy()
        del Yg
    finally:
        S.close()
    _cmp(info, got, inner(Y.astype(np.float64), 1e-30, T))
