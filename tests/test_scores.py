"""The package's matching scores agree with the oracle's trace-form
definitions of eq. (3) and of accuracy."""
import numpy as np
import pytest

from oracle import fastpfp_oracle as O
from paper_1207_1114_amd import scores, synth


@pytest.mark.parametrize("n,m", [(7, 7), (6, 9), (9, 6), (40, 52)])
def test_objective_and_accuracy_match_oracle(n, m):
    rng = np.random.default_rng([n, m])
    A = synth.random_weighted_graph(rng, n, 0.4)
    B = synth.random_weighted_graph(rng, m, 0.4)
    K = rng.random((n, m))
    if n <= m:
        match = rng.permutation(m)[:n]
    else:
        match = -np.ones(n, dtype=np.int64)
        match[rng.permutation(n)[:m]] = rng.permutation(m)
    perm = rng.permutation(max(n, m))[:n] if n <= m else match.copy()
    perm[0] = -1
    for lam in (0.0, 0.7):
        assert scores.matching_objective(A, B, K, lam, match) == pytest.approx(
            O.objective(A, B, K, lam, match), rel=1e-12, abs=1e-12)
    assert scores.accuracy(match, perm) == O.accuracy(match, perm)


@pytest.mark.parametrize("n,m", [(6, 6), (5, 8), (30, 33)])
def test_frobenius_error_matches_oracle(n, m):
    rng = np.random.default_rng([n, m, 5])
    A = synth.random_weighted_graph(rng, n, 0.5)
    B = synth.random_weighted_graph(rng, m, 0.5)
    match = rng.permutation(m)[:n]
    match[1] = -1
    # Sec. 5.1 reports ||A - X A' X^T||_F^2; eq. (1) carries a factor 1/2
    assert scores.frobenius_error(A, B, match) == pytest.approx(
        2.0 * O.matching_error(A, B, match), rel=1e-12, abs=1e-12)
