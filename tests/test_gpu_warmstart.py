"""GPU parity of the learned warm start, called through the C ABI, against the
FP64 warm-start oracle (whose gradients are pinned by central differences).

Tolerances.  Features are counts divided by a degree: the kernel's float32
result must equal the oracle's value rounded to float32, bit for bit (the
bins are taken in float64 on both sides).  The network runs in float32: with
|S| <= ~15 for these parameters, S carries an absolute error of about 64
products x 2^-24 x |S| ~ 1e-5, which moves each softmax output by a relative
~2e-5, so X0 is compared with a relative bound of 2e-4.  Gradients sum
n n' terms of float32 products: each parameter tensor must match the oracle
within 1e-3 of that tensor's largest gradient, and the loss within 1e-5
relative.
"""
import numpy as np
import pytest

from oracle import warmstart_oracle as W
from paper_1207_1114_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1207_1114_amd import fastpfp as F
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    S = F.Solver(1024, 1024)
    return torch, F, S


def dev(torch, a):
    if a is None:
        return None
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda:0")


def f32(a):
    """The float32 copy the GPU receives, back in float64 for the oracle."""
    return None if a is None else np.asarray(a, np.float32).astype(np.float64)


def params(seed, logtau=np.log(2.0)):
    flat = W.init_params(seed)
    flat[-1] = logtau
    # small nonzero biases so every bias path is exercised
    rng = np.random.default_rng(seed + 77)
    p = W.unpack(flat)
    for b in ("b1", "b2", "b3"):
        p[b] = rng.normal(0.0, 0.1, size=p[b].shape)
    return W.pack(p).astype(np.float32).astype(np.float64)


def pair(kind, n, m, seed):
    rng = np.random.default_rng([kind, n, m, seed])
    if kind == 0:       # config-1 model: Bernoulli(0.1), 16-d attributes
        A = synth.random_weighted_graph(rng, n, 0.1)
        B = synth.random_weighted_graph(rng, m, 0.1)
        F, G = rng.normal(size=(n, 16)), rng.normal(size=(m, 16))
    elif kind == 1:     # 8-NN distance graphs, 8-d attributes
        A = synth.knn_distance_graph(rng.random((n, 2)), 8)
        B = synth.knn_distance_graph(rng.random((m, 2)), 8)
        F, G = rng.normal(size=(n, 8)), rng.normal(size=(m, 8))
    else:               # isolated nodes, negative weights, no attributes
        A = synth.random_weighted_graph(rng, n, 0.05) - 0.3 * (
            synth.random_weighted_graph(rng, n, 0.05) > 0)
        A = np.triu(A, 1)
        A = A + A.T
        B = synth.random_weighted_graph(rng, m, 0.05)
        F = G = None
    return f32(A), f32(B), f32(F), f32(G)


# -------------------------------------------------------------- features
@pytest.mark.parametrize("kind,n", [(0, 1), (0, 2), (0, 70), (0, 300),
                                    (1, 150), (2, 90), (2, 1000)])
def test_features_bit_exact(env, kind, n):
    torch, F, S = env
    A, _, Fa, _ = pair(kind, n, 3, 0)
    x = S.warmstart_features(dev(torch, A), dev(torch, Fa)).cpu().numpy()
    want = W.node_features(A, Fa).astype(np.float32)
    np.testing.assert_array_equal(x, want)


# -------------------------------------------------------------------- X0
@pytest.mark.parametrize("kind,n,m", [(0, 1, 1), (0, 70, 90), (0, 130, 100),
                                      (1, 150, 170), (2, 64, 64),
                                      (0, 300, 300), (1, 257, 200)])
@pytest.mark.parametrize("bf16", [False, True])
def test_x0_parity(env, kind, n, m, bf16):
    torch, F, S = env
    A, B, Fa, Gb = pair(kind, n, m, 1)
    prm = params(3)
    S.warmstart_load(prm)
    X = torch.full((n, m + 3), -7.0, device="cuda:0")[:, :m]  # ragged pitch
    S.warmstart(dev(torch, A), dev(torch, B), dev(torch, Fa), dev(torch, Gb),
                X, bf16_weights=bf16)
    Xg = X.cpu().numpy().astype(np.float64)
    Xo = W.x0(W.unpack(prm), A, B, Fa, Gb, bf16=bf16)
    assert np.all(np.abs(Xg - Xo) <= 2e-4 * Xo + 1e-30), np.abs(Xg - Xo).max()
    axis = 1 if n <= m else 0
    np.testing.assert_allclose(Xg.sum(axis=axis), 1.0, atol=1e-5)


def test_x0_non_finite_input_reports_numeric(env):
    torch, F, S = env
    A, B, Fa, Gb = pair(0, 40, 40, 2)
    Fa = Fa.copy()
    Fa[3, 0] = np.nan
    S.warmstart_load(params(0))
    X = torch.zeros(40, 40, device="cuda:0")
    with pytest.raises(F.FastPFPError) as e:
        S.warmstart(dev(torch, A), dev(torch, B), dev(torch, Fa),
                    dev(torch, Gb), X)
    assert e.value.status == 5


def test_warmstart_argument_errors(env):
    torch, F, S = env
    fresh = F.Solver(64, 64)
    A = torch.zeros(8, 8, device="cuda:0")
    X = torch.zeros(8, 8, device="cuda:0")
    with pytest.raises(F.FastPFPError) as e:
        fresh.warmstart(A, A, None, None, X)          # nothing loaded
    assert e.value.status == 1
    with pytest.raises(ValueError):
        fresh.warmstart_load(np.zeros(10, np.float32))
    bad = np.zeros(F.WS_NPARAMS, np.float32)
    bad[5] = np.inf
    with pytest.raises(F.FastPFPError) as e:
        fresh.warmstart_load(bad)
    assert e.value.status == 1
    fresh.warmstart_load(np.zeros(F.WS_NPARAMS, np.float32))
    big = torch.zeros(65, 65, device="cuda:0")
    with pytest.raises(F.FastPFPError) as e:
        fresh.warmstart(big, big, None, None, big)
    assert e.value.status == 2
    fresh.close()


# -------------------------------------------------------------- gradient
@pytest.mark.parametrize("kind,n,m", [(0, 70, 90), (0, 130, 100),
                                      (1, 150, 170), (2, 60, 60)])
def test_gradient_parity(env, kind, n, m):
    torch, F, S = env
    A, B, Fa, Gb = pair(kind, n, m, 4)
    prm = params(5)
    rng = np.random.default_rng([n, m])
    T = f32(rng.random((n, m)) ** 4)          # positive, uneven target
    S.warmstart_load(prm)
    S.warmstart_zero_grad()
    loss = S.warmstart_grad(dev(torch, A), dev(torch, B), dev(torch, Fa),
                            dev(torch, Gb), dev(torch, T))
    _, g = S.warmstart_get()
    lo, go = W.loss_and_grad(W.unpack(prm), A, B, Fa, Gb, T)
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    gu = W.unpack(g.astype(np.float64))
    for name, _ in W.SHAPES:
        ref = go[name]
        err = np.abs(gu[name] - ref).max()
        assert err <= 1e-3 * np.abs(ref).max() + 1e-9, (name, err,
                                                        np.abs(ref).max())


def test_gradient_is_deterministic_and_accumulates(env):
    """Repeated from zero, the gradient is bitwise identical; a second call
    adds to it (the two graph sides accumulate into one buffer, so the sum
    is 2 g up to rounding, not bitwise)."""
    torch, F, S = env
    A, B, Fa, Gb = (dev(torch, a) for a in pair(0, 100, 120, 6))
    T = dev(torch, np.random.default_rng(6).random((100, 120)))
    S.warmstart_load(params(6))
    S.warmstart_zero_grad()
    l1 = S.warmstart_grad(A, B, Fa, Gb, T)
    _, g1 = S.warmstart_get()
    S.warmstart_zero_grad()
    l2 = S.warmstart_grad(A, B, Fa, Gb, T)
    _, g1b = S.warmstart_get()
    assert l1 == l2
    np.testing.assert_array_equal(g1, g1b)
    S.warmstart_grad(A, B, Fa, Gb, T)
    _, g2 = S.warmstart_get()
    np.testing.assert_allclose(g2, 2.0 * g1, rtol=1e-5,
                               atol=1e-6 * np.abs(g1).max())


def test_adam_step_matches_torch_adam(env):
    torch, F, S = env
    A, B, Fa, Gb = (dev(torch, a) for a in pair(1, 80, 80, 7))
    T = dev(torch, np.random.default_rng(7).random((80, 80)))
    p0 = params(7).astype(np.float32)
    S.warmstart_load(p0)
    ref = torch.nn.Parameter(torch.tensor(p0))
    opt = torch.optim.Adam([ref], lr=1e-3, betas=(0.9, 0.99), eps=1e-8)
    for _ in range(3):
        S.warmstart_zero_grad()
        S.warmstart_grad(A, B, Fa, Gb, T)
        S.warmstart_grad(A, B, Fa, Gb, T)
        _, g = S.warmstart_get()
        ref.grad = torch.tensor(g) * 0.5
        opt.step()
        S.warmstart_adam(1e-3, 0.9, 0.99, 1e-8, grad_scale=0.5)
        p, _ = S.warmstart_get()
        np.testing.assert_allclose(p, ref.detach().numpy(), rtol=1e-5,
                                   atol=1e-7)


def test_a_few_adam_steps_lower_the_loss(env):
    """On a planted pair whose attributes identify the permutation, thirty
    Adam steps towards the permutation matrix must halve the loss."""
    torch, F, S = env
    p = synth.config4_pair(0, 120, train=True)
    A, B, Fa, Gb = (dev(torch, a) for a in (p.A, p.B, p.F, p.G))
    T = np.zeros((120, 120))
    T[np.arange(120), p.perm] = 1.0
    T = dev(torch, T)
    S.warmstart_load(params(8))
    losses = []
    for _ in range(30):
        S.warmstart_zero_grad()
        losses.append(S.warmstart_grad(A, B, Fa, Gb, T))
        S.warmstart_adam(3e-3)
    assert losses[-1] < 0.5 * losses[0], losses[::6]


def test_batched_x0_on_every_stream_equals_single(env):
    """Twelve pairs of mixed sizes: the batched call spreads them over its
    four streams (three pairs each, of different sizes, sharing that
    stream's node buffers in turn); every X0 equals the one-pair call bit
    for bit."""
    torch, F, S = env
    shapes = [(40, 60), (300, 280), (17, 17), (128, 200), (250, 250),
              (90, 33), (64, 64), (199, 301), (5, 9), (260, 140), (120, 120),
              (77, 150)]
    pairs = [pair(0, n, m, 30 + k) for k, (n, m) in enumerate(shapes)]
    S.warmstart_load(params(4))
    cat = lambda xs: dev(torch, np.concatenate([np.ravel(x) for x in xs]))
    offs = lambda xs: np.cumsum([0] + [np.size(x) for x in xs[:-1]])
    As, Bs = [p[0] for p in pairs], [p[1] for p in pairs]
    Fs, Gs = [p[2] for p in pairs], [p[3] for p in pairs]
    Xs = [np.zeros(s) for s in shapes]
    X = cat(Xs)
    st = S.warmstart_batched([s[0] for s in shapes], [s[1] for s in shapes],
                             cat(As), offs(As), cat(Bs), offs(Bs), cat(Fs),
                             offs(Fs), cat(Gs), offs(Gs), 16, X, offs(Xs),
                             bf16_weights=True)
    assert st == [0] * len(shapes)
    Xh = X.cpu().numpy()
    for k, ((n, m), o) in enumerate(zip(shapes, offs(Xs))):
        Xk = torch.zeros(n, m, device="cuda:0")
        S.warmstart(*(dev(torch, a) for a in pairs[k]), Xk, bf16_weights=True)
        np.testing.assert_array_equal(Xh[o:o + n * m].reshape(n, m),
                                      Xk.cpu().numpy())


def test_batched_x0_equals_single_and_isolates_a_bad_pair(env):
    torch, F, S = env
    shapes = [(70, 90), (130, 100), (1, 1), (64, 64), (200, 257)]
    pairs = [pair(0, n, m, 9 + k) for k, (n, m) in enumerate(shapes)]
    # pair 3 gets a NaN attribute: only its status may fail
    Fa3 = pairs[3][2].copy()
    Fa3[0, 0] = np.nan
    pairs[3] = (pairs[3][0], pairs[3][1], Fa3, pairs[3][3])
    S.warmstart_load(params(9))
    cat = lambda xs: dev(torch, np.concatenate([np.ravel(x) for x in xs]))
    offs = lambda xs: np.cumsum([0] + [np.size(x) for x in xs[:-1]])
    As, Bs = [p[0] for p in pairs], [p[1] for p in pairs]
    Fs, Gs = [p[2] for p in pairs], [p[3] for p in pairs]
    Xs = [np.zeros(s) for s in shapes]
    X = cat(Xs)
    st = S.warmstart_batched([s[0] for s in shapes], [s[1] for s in shapes],
                             cat(As), offs(As), cat(Bs), offs(Bs), cat(Fs),
                             offs(Fs), cat(Gs), offs(Gs), 16, X, offs(Xs),
                             bf16_weights=True)
    assert st == [0, 0, 0, 5, 0]
    Xh = X.cpu().numpy()
    for k, ((n, m), o) in enumerate(zip(shapes, offs(Xs))):
        if k == 3:
            continue
        Xk = torch.zeros(n, m, device="cuda:0")
        S.warmstart(*(dev(torch, a) for a in pairs[k]), Xk, bf16_weights=True)
        np.testing.assert_array_equal(Xh[o:o + n * m].reshape(n, m),
                                      Xk.cpu().numpy())
