"""Seeded synthetic graph pairs shaped like the FastPFP paper's workloads.

This module only *generates inputs*; it holds none of the matching method's
arithmetic, so both the FP64 oracle and the GPU path may import it.

Problem statement (paper, Sec. 3, eqs. 1-4): two undirected graphs with
symmetric adjacency matrices A (n x n) and A' (n' x n'), here called ``B``,
plus a node-similarity matrix K (n x n') weighted by lambda.  Every generator
plants a known correspondence ``perm``: node i of the first graph is node
``perm[i]`` of the second one, so matching accuracy can be scored.

Every random draw comes from ``np.random.default_rng([1207, 1114, cfg, idx])``
so that a (config, pair index) names one pair for good.

Workload recipes (parameters of the five benchmark configurations):

* ``config0_pair``  n=n'=100, Bernoulli(0.2) edges, U(0,1) weights, B is a
  relabelled copy of A with N(0, 0.02^2) noise on the existing edges (added
  once per undirected edge and mirrored), lambda = 0.
* ``config1_pair``  n=n'=1000, Bernoulli(0.1), noise sigma 0.05, 16-d N(0,1)
  node attributes, the second graph's copies perturbed by N(0, 0.1^2),
  K_ij = exp(-||f_i - g_j||^2), lambda = 1.  (The paper's K is an inner
  product of SIFT descriptors, Sec. 5.3; a Gaussian kernel keeps K bounded.)
* ``config2_pair``  n=1000, n'=1200: config 1 plus 200 outlier nodes in the
  second graph, each joined to every other node by a Bernoulli(0.1) U(0,1)
  edge, with N(0, I) attributes.
* ``config3_pair``  ragged batch member: n ~ U{50..400}, n' = n + U{0..40};
  graphs are symmetric 8-NN graphs of U[0,1]^2 point sets whose edge weights
  are Euclidean distances (the paper's point graphs, Sec. 5.3-5.4, use the
  distance as the weight); the second point set is the first one rotated by
  U(-pi/4, pi/4), scaled by U(0.8, 1.2), jittered by N(0, 0.01^2), plus
  outliers drawn uniformly in its bounding box; 8-d attributes.
* ``config4_pair``  n=n', Bernoulli(0.05), noise 0.05, config 1's attribute
  model (training sizes n ~ U{100..500}, evaluation n = 2000 or 4000).
* ``paper_synthetic_pair``  the paper's Sec. 5.1 benchmark: unweighted
  random graphs with 50% connectivity, optional n edge flips and 10% node
  deletion.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_ROOT = (1207, 1114)


def rng_for(cfg: int, idx: int) -> np.random.Generator:
    """The generator that names pair ``idx`` of configuration ``cfg``."""
    return np.random.default_rng([SEED_ROOT[0], SEED_ROOT[1], int(cfg), int(idx)])


@dataclass
class GraphPair:
    """One matching problem.  Arrays are float64, row-major.

    A: (n, n) symmetric; B: (np_, np_) symmetric; K: (n, np_) or None when
    lam == 0; perm[i] is the planted partner of node i in the second graph,
    or -1 when node i has none.  F (n, d) and G (np_, d) are node attributes
    (None when the configuration has none).
    """

    A: np.ndarray
    B: np.ndarray
    K: Optional[np.ndarray]
    lam: float
    perm: np.ndarray
    F: Optional[np.ndarray] = None
    G: Optional[np.ndarray] = None
    cfg: int = -1
    idx: int = -1
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def np_(self) -> int:
        return self.B.shape[0]


# ---------------------------------------------------------------- helpers
def random_weighted_graph(rng: np.random.Generator, n: int, p: float,
                          weighted: bool = True) -> np.ndarray:
    """Symmetric adjacency, zero diagonal, Bernoulli(p) edges on i<k."""
    mask = np.triu(rng.random((n, n)) < p, k=1)
    if weighted:
        w = np.triu(rng.random((n, n)), k=1)
        A = np.where(mask, w, 0.0)
    else:
        A = mask.astype(np.float64)
    return A + A.T


def relabel(rng: np.random.Generator, A: np.ndarray, n2: int,
            noise: float) -> tuple[np.ndarray, np.ndarray]:
    """Place graph A's nodes at random positions of an n2-node graph.

    Returns (B, perm) with B[perm[i], perm[k]] = A[i, k] + noise on every
    existing edge (noise drawn once per undirected edge and mirrored).
    Positions not hit by perm are left empty for the caller to fill.
    """
    n = A.shape[0]
    perm = rng.permutation(n2)[:n]
    An = A.copy()
    if noise > 0:
        e = np.triu(rng.normal(0.0, noise, size=(n, n)), k=1)
        e = e + e.T
        An = np.where(A != 0, A + e, 0.0)
    B = np.zeros((n2, n2))
    B[np.ix_(perm, perm)] = An
    return B, perm


def gaussian_similarity(F: np.ndarray, G: np.ndarray) -> np.ndarray:
    """K_ij = exp(-||f_i - g_j||^2) in float64."""
    d2 = (np.sum(F * F, 1)[:, None] + np.sum(G * G, 1)[None, :]
          - 2.0 * F @ G.T)
    return np.exp(-np.maximum(d2, 0.0))


def attributes(rng: np.random.Generator, n: int, n2: int, perm: np.ndarray,
               dim: int, noise: float) -> tuple[np.ndarray, np.ndarray]:
    """N(0,I) attributes; partners copy them with N(0, noise^2) added."""
    F = rng.normal(size=(n, dim))
    G = rng.normal(size=(n2, dim))
    G[perm] = F + rng.normal(0.0, noise, size=(n, dim))
    return F, G


def knn_distance_graph(P: np.ndarray, k: int) -> np.ndarray:
    """Symmetric k-NN graph of points P with Euclidean-distance weights."""
    n = P.shape[0]
    d = np.sqrt(np.maximum(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1), 0))
    dd = d + np.diag(np.full(n, np.inf))
    kk = min(k, n - 1)
    nbr = np.argpartition(dd, kk - 1, axis=1)[:, :kk]
    M = np.zeros((n, n), dtype=bool)
    M[np.repeat(np.arange(n), kk), nbr.ravel()] = True
    M = M | M.T
    return np.where(M, d, 0.0)


# ---------------------------------------------------------------- configs
def config0_pair(idx: int = 0, n: int = 100) -> GraphPair:
    rng = rng_for(0, idx)
    A = random_weighted_graph(rng, n, 0.2)
    B, perm = relabel(rng, A, n, 0.02)
    return GraphPair(A, B, None, 0.0, perm, cfg=0, idx=idx)


def config1_pair(idx: int = 0, n: int = 1000) -> GraphPair:
    rng = rng_for(1, idx)
    A = random_weighted_graph(rng, n, 0.1)
    B, perm = relabel(rng, A, n, 0.05)
    F, G = attributes(rng, n, n, perm, 16, 0.1)
    return GraphPair(A, B, gaussian_similarity(F, G), 1.0, perm, F, G,
                     cfg=1, idx=idx)


def config2_pair(idx: int = 0, n: int = 1000, n_out: int = 200) -> GraphPair:
    rng = rng_for(2, idx)
    n2 = n + n_out
    A = random_weighted_graph(rng, n, 0.1)
    B, perm = relabel(rng, A, n2, 0.05)
    outl = np.setdiff1d(np.arange(n2), perm)
    # Outliers: Bernoulli(0.1) U(0,1) edges to every other node.
    for o in outl:
        row = np.where(rng.random(n2) < 0.1, rng.random(n2), 0.0)
        row[o] = 0.0
        # keep earlier outlier rows symmetric: only write where still empty
        for j in np.nonzero(row)[0]:
            if B[o, j] == 0.0:
                B[o, j] = B[j, o] = row[j]
    F, G = attributes(rng, n, n2, perm, 16, 0.1)
    return GraphPair(A, B, gaussian_similarity(F, G), 1.0, perm, F, G,
                     cfg=2, idx=idx)


def config3_pair(idx: int, n: Optional[int] = None,
                 n_extra: Optional[int] = None) -> GraphPair:
    rng = rng_for(3, idx)
    if n is None:
        n = int(rng.integers(50, 401))
    if n_extra is None:
        n_extra = int(rng.integers(0, 41))
    n2 = n + n_extra
    P = rng.random((n, 2))
    th = rng.uniform(-np.pi / 4, np.pi / 4)
    sc = rng.uniform(0.8, 1.2)
    R = sc * np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    Q_in = P @ R.T + rng.normal(0.0, 0.01, size=(n, 2))
    lo, hi = Q_in.min(0), Q_in.max(0)
    Q_out = lo + (hi - lo) * rng.random((n_extra, 2))
    perm = rng.permutation(n2)[:n]
    Q = np.zeros((n2, 2))
    Q[perm] = Q_in
    outl = np.setdiff1d(np.arange(n2), perm)
    Q[outl] = Q_out
    A = knn_distance_graph(P, 8)
    B = knn_distance_graph(Q, 8)
    F, G = attributes(rng, n, n2, perm, 8, 0.1)
    return GraphPair(A, B, gaussian_similarity(F, G), 1.0, perm, F, G,
                     cfg=3, idx=idx)


def config3_sizes(batch: int = 512) -> list[tuple[int, int]]:
    """(n, n') of each member of the ragged batch, without building it."""
    out = []
    for i in range(batch):
        rng = rng_for(3, i)
        n = int(rng.integers(50, 401))
        out.append((n, n + int(rng.integers(0, 41))))
    return out


def config4_pair(idx: int, n: int, train: bool = False) -> GraphPair:
    rng = rng_for(4 if not train else 40, idx)
    A = random_weighted_graph(rng, n, 0.05)
    B, perm = relabel(rng, A, n, 0.05)
    F, G = attributes(rng, n, n, perm, 16, 0.1)
    return GraphPair(A, B, gaussian_similarity(F, G), 1.0, perm, F, G,
                     cfg=4, idx=idx)


def planted_isomorphic_pair(idx: int, n: int, p: float = 0.2) -> GraphPair:
    """Noiseless weighted relabelled copy (lambda = 0)."""
    rng = rng_for(90, idx * 100000 + n)
    A = random_weighted_graph(rng, n, p)
    B, perm = relabel(rng, A, n, 0.0)
    return GraphPair(A, B, None, 0.0, perm, cfg=90, idx=idx)


def paper_synthetic_pair(idx: int, n: int, edge_flips: bool,
                         node_deletion: bool) -> GraphPair:
    """Sec. 5.1: unweighted 50%-connectivity random graphs.

    edge_flips: n entries A_ik (i<k) toggled after relabelling.
    node_deletion: 10% of the first graph's nodes removed (subgraph case).
    """
    rng = rng_for(91, idx * 100000 + n * 4 + 2 * int(edge_flips)
                  + int(node_deletion))
    A = random_weighted_graph(rng, n, 0.5, weighted=False)
    B, perm = relabel(rng, A, n, 0.0)
    if edge_flips:
        iu = np.array(np.triu_indices(n, 1)).T
        pick = iu[rng.choice(len(iu), size=n, replace=False)]
        for i, k in pick:
            v = 1.0 - B[i, k]
            B[i, k] = B[k, i] = v
    if node_deletion:
        keep = np.sort(rng.permutation(n)[: n - n // 10])
        A = A[np.ix_(keep, keep)]
        perm = perm[keep]
    return GraphPair(A, B, None, 0.0, perm, cfg=91, idx=idx)


def make_pair(cfg: int, idx: int = 0, **kw) -> GraphPair:
    return {0: config0_pair, 1: config1_pair, 2: config2_pair,
            3: config3_pair}[cfg](idx, **kw)
