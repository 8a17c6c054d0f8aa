"""Pins of the warm-start oracle: features on a hand-worked graph, the
softmax constraint, permutation equivariance, and backpropagated gradients
against float64 central differences."""
import numpy as np
import pytest

from oracle import warmstart_oracle as W
from paper_1207_1114_amd import synth


def test_features_path_graph_by_hand():
    """Path 0-1-2-3, unit weights: degrees 1,2,2,1 (mean 1.5), so a degree-1
    neighbour falls in bin floor(4/1.5) = 2 and a degree-2 one in bin
    floor(8/1.5) = 5; weighted degrees equal degrees."""
    A = np.zeros((4, 4))
    for i in range(3):
        A[i, i + 1] = A[i + 1, i] = 1.0
    F = np.arange(8.0).reshape(4, 2)
    x = W.node_features(A, F)
    want = np.zeros((4, 48))
    for h in (0, 16):
        want[0, h + 5] = 1.0            # node 0: neighbour 1 (deg 2)
        want[1, h + 2] = want[1, h + 5] = 0.5   # node 1: nodes 0 and 2
        want[2, h + 2] = want[2, h + 5] = 0.5
        want[3, h + 5] = 1.0
    want[:, 32:34] = F
    np.testing.assert_array_equal(x, want)


def test_features_last_bin_is_open_and_isolated_nodes_are_zero():
    A = np.zeros((6, 6))
    for k in range(1, 5):                 # star centre 0, leaves 1..4
        A[0, k] = A[k, 0] = 2.0
    x = W.node_features(A)
    # mean degree 8/6; centre has degree 4: 4*4/(8/6) = 12 -> bin 12;
    # leaves have degree 1: 4/(8/6) = 3 -> bin 3
    assert x[1, 12] == 1.0 and x[0, 3] == 1.0
    assert np.all(x[5] == 0.0)            # isolated node
    A2 = np.zeros((5, 5))
    A2[0, 1:] = A2[1:, 0] = 1.0
    A2[1, 2] = A2[2, 1] = 1.0
    x2 = W.node_features(A2)
    # degrees 4,2,2,1,1 (mean 2): node 1 sees node 0 (bin 8) and node 2 (bin 4)
    assert x2[1, 8] == 0.5 and x2[1, 4] == 0.5 and x2[1, :16].sum() == 1.0
    A3 = np.zeros((40, 40))
    A3[0, 1:] = A3[1:, 0] = 1.0           # hub of degree 39, mean ~1.95
    assert W.node_features(A3)[1, 15] == 1.0   # floor(80) clipped to 15


def test_negative_weighted_degree_falls_in_bin_zero():
    """Edge noise can make a row sum negative: its bin clips to 0."""
    A = np.zeros((4, 4))
    A[0, 1] = A[1, 0] = -0.5
    A[2, 3] = A[3, 2] = 2.0
    A[1, 2] = A[2, 1] = 1.0
    x = W.node_features(A)
    # wdeg = -0.5, 0.5, 3, 2 (mean 1.25): node 0's only neighbour (node 1)
    # has 4*0.5/1.25 = 1.6 -> bin 1; node 1 sees node 0 (-1.6 -> bin 0)
    # and node 2 (9.6 -> bin 9)
    assert x[0, 16 + 1] == 1.0
    assert x[1, 16 + 0] == 0.5 and x[1, 16 + 9] == 0.5


def test_bf16_weight_recipe_moves_x0_by_little():
    rng = np.random.default_rng(8)
    A = synth.random_weighted_graph(rng, 20, 0.3)
    B = synth.random_weighted_graph(rng, 24, 0.3)
    p = W.unpack(W.init_params(0))
    X, Xb = W.x0(p, A, B), W.x0(p, A, B, bf16=True)
    assert not np.array_equal(X, Xb)
    np.testing.assert_allclose(Xb.sum(1), 1.0, atol=1e-12)
    assert np.abs(X - Xb).max() < 0.05 * X.max()


def test_x0_constraint_axis_and_permutation_equivariance():
    rng = np.random.default_rng(3)
    p = W.unpack(W.init_params(1))
    for n, m in ((9, 12), (12, 9)):
        A = synth.random_weighted_graph(rng, n, 0.4)
        B = synth.random_weighted_graph(rng, m, 0.4)
        F, G = rng.normal(size=(n, 16)), rng.normal(size=(m, 16))
        X = W.x0(p, A, B, F, G)
        axis = 1 if n <= m else 0
        np.testing.assert_allclose(X.sum(axis=axis), 1.0, atol=1e-12)
        q, s = rng.permutation(n), rng.permutation(m)
        Xp = W.x0(p, A[np.ix_(q, q)], B[np.ix_(s, s)], F[q], G[s])
        np.testing.assert_allclose(Xp, X[np.ix_(q, s)], atol=1e-12)


@pytest.mark.parametrize("n,m", [(6, 8), (8, 6)])
def test_gradient_matches_central_differences(n, m):
    rng = np.random.default_rng(n * 10 + m)
    A = synth.random_weighted_graph(rng, n, 0.5)
    B = synth.random_weighted_graph(rng, m, 0.5)
    F, G = rng.normal(size=(n, 16)), rng.normal(size=(m, 16))
    T = rng.random((n, m)) + 0.1
    flat = W.init_params(2)
    flat[-1] = np.log(3.0)
    p = W.unpack(flat)
    loss, g = W.loss_and_grad(p, A, B, F, G, T)
    gflat = W.pack(g)
    h = 1e-6
    pick = np.concatenate([rng.choice(W.NPARAMS - 1, 60, replace=False),
                           [W.NPARAMS - 1]])
    for k in pick:
        e = np.zeros(W.NPARAMS)
        e[k] = h
        lp, _ = W.loss_and_grad(W.unpack(flat + e), A, B, F, G, T)
        lm, _ = W.loss_and_grad(W.unpack(flat - e), A, B, F, G, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gflat[k]) <= 1e-6 + 1e-5 * abs(fd), (k, fd, gflat[k])


def test_loss_is_minimal_when_softmax_equals_target():
    rng = np.random.default_rng(5)
    n, m = 5, 7
    A = synth.random_weighted_graph(rng, n, 0.5)
    B = synth.random_weighted_graph(rng, m, 0.5)
    p = W.unpack(W.init_params(4))
    X = W.x0(p, A, B)
    loss, g = W.loss_and_grad(p, A, B, None, None, X * 3.0)
    # the target normalises to X itself: dS = 0, so every gradient vanishes
    assert np.abs(W.pack(g)).max() < 1e-12
    ent = -np.sum(X * np.log(X)) / n
    assert abs(loss - ent) < 1e-12


def test_network_forward_by_hand():
    """Hand-set weights: unit 0 = relu(f0 - 0.5), unit 1 = relu(-f0), passed
    through layer 2 unchanged, and e0 = h0 - 2 h1; every other weight 0.  So
    S_ij = e0(f_i) e0(g_j) / tau and X0 is its row softmax, computed here
    directly from the attributes."""
    p = W.unpack(np.zeros(W.NPARAMS))
    a0 = 2 * W.NBINS                      # column of attribute 0
    p["W1"][0, a0], p["b1"][0] = 1.0, -0.5
    p["W1"][1, a0] = -1.0
    p["W2"][0, 0] = p["W2"][1, 1] = 1.0
    p["W3"][0, 0], p["W3"][0, 1] = 1.0, -2.0
    p["b3"][0] = 0.25
    p["logtau"][0] = np.log(0.5)
    rng = np.random.default_rng(9)
    n, m = 6, 9
    A = synth.random_weighted_graph(rng, n, 0.5)
    B = synth.random_weighted_graph(rng, m, 0.5)
    F, G = rng.normal(size=(n, 3)), rng.normal(size=(m, 3))
    e = lambda f: (np.maximum(f - 0.5, 0) - 2 * np.maximum(-f, 0) + 0.25)
    S = np.outer(e(F[:, 0]), e(G[:, 0])) / 0.5
    want = np.exp(S - S.max(1, keepdims=True))
    want /= want.sum(1, keepdims=True)
    np.testing.assert_allclose(W.x0(p, A, B, F, G), want, rtol=1e-12)
    # transposed orientation: softmax over each column
    S2 = S.T
    want2 = np.exp(S2 - S2.max(0, keepdims=True))
    want2 /= want2.sum(0, keepdims=True)
    np.testing.assert_allclose(W.x0(p, B, A, G, F), want2, rtol=1e-12)
