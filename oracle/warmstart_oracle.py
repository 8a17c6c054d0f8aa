"""FP64 oracle of the learned warm start -- TEST INFRASTRUCTURE ONLY.

The warm start is not part of the paper: it is a small per-node network whose
output replaces Algorithm 1's uniform initialisation X0 (the paper notes the
method is sensitive to initialisation, Sec. 4.5).  Only the tests may import
this module.

Definitions (shared with the HIP implementation only through this text):

* Node features, 48 per node.  deg(k) = number of nonzero entries of row k
  of the adjacency, wdeg(k) = sum of row k; md, mw their means over the graph.
  For node i, over its neighbours k (A_ik != 0):
    h_deg[b]  = #{k : clip(floor(4 deg(k) / md), 0, 15) = b} / deg(i)
    h_wdeg[b] = #{k : clip(floor(4 wdeg(k) / mw), 0, 15) = b} / deg(i)
  (16 bins each, zero when deg(i) = 0 or the mean is <= 0; the lower clip
  only matters for a negative weighted degree), followed by the node's
  attributes, zero-padded to 16.  The bin index is taken in float64 as
  written: (4 v) / m, then floor.
* Network: h1 = relu(W1 x + b1) (128), h2 = relu(W2 h1 + b2) (128),
  e = W3 h2 + b3 (64).  For inference the three weight matrices may be
  stored in bfloat16 (round to nearest even); biases and tau stay float.
* X0 = softmax of S = E E'^T / tau (tau = exp(logtau)) along the larger side:
  over j for each row i when n <= n', over i for each column j otherwise, so
  the smaller side sums to one as in the relaxed constraint set (Sec. 4).
* Training loss for a target X* (the solver's fixed point): with P = X*
  normalised along the same axis, L = -(1/ns) sum P * log(X0), ns = min(n,n').
"""
from __future__ import annotations

import numpy as np

from .fastpfp_oracle import bf16_round

NBINS = 16
ATTR = 16
D_IN = 2 * NBINS + ATTR
H1, H2, D_OUT = 128, 128, 64
SHAPES = [("W1", (H1, D_IN)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)),
          ("W3", (D_OUT, H2)), ("b3", (D_OUT,)), ("logtau", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel()
                           for name, _ in SHAPES])


def node_features(A: np.ndarray, F=None) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    nz = A != 0
    deg = nz.sum(1).astype(np.float64)
    wdeg = A.sum(1)
    md, mw = deg.sum() / n, wdeg.sum() / n
    feat = np.zeros((n, D_IN))

    def bins(v, m):
        if m <= 0:
            return None
        return np.clip(np.floor(4.0 * v / m), 0, 15).astype(np.int64)

    bd, bw = bins(deg, md), bins(wdeg, mw)
    for i in range(n):
        if deg[i] == 0:
            continue
        nb = np.nonzero(nz[i])[0]
        if bd is not None:
            feat[i, :NBINS] = np.bincount(bd[nb], minlength=NBINS) / deg[i]
        if bw is not None:
            feat[i, NBINS:2 * NBINS] = (np.bincount(bw[nb], minlength=NBINS)
                                        / deg[i])
    if F is not None:
        d = min(ATTR, F.shape[1])
        feat[:, 2 * NBINS:2 * NBINS + d] = F[:, :d]
    return feat


def mlp_forward(p: dict, x: np.ndarray):
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    e = h2 @ p["W3"].T + p["b3"]
    return e, (x, h1, h2)


def softmax_x0(E, Ep, logtau):
    """Returns (X0, S, axis): the softmax axis is 1 (rows) when n <= n'."""
    S = (E @ Ep.T) * np.exp(-logtau)
    axis = 1 if E.shape[0] <= Ep.shape[0] else 0
    m = S.max(axis=axis, keepdims=True)
    Z = np.exp(S - m)
    return Z / Z.sum(axis=axis, keepdims=True), S, axis


def bf16_weights(p: dict) -> dict:
    """The inference copy: W1, W2, W3 rounded to bfloat16."""
    return {k: (bf16_round(v) if k.startswith("W") else v)
            for k, v in p.items()}


def x0(p: dict, A, B, F=None, G=None, bf16: bool = False) -> np.ndarray:
    if bf16:
        p = bf16_weights(p)
    E, _ = mlp_forward(p, node_features(A, F))
    Ep, _ = mlp_forward(p, node_features(B, G))
    return softmax_x0(E, Ep, float(p["logtau"][0]))[0]


def loss_and_grad(p: dict, A, B, F, G, target):
    """Loss and its exact gradient (dict like p) by backpropagation."""
    xa, xb = node_features(A, F), node_features(B, G)
    E, ca = mlp_forward(p, xa)
    Ep, cb = mlp_forward(p, xb)
    logtau = float(p["logtau"][0])
    Q, S, axis = softmax_x0(E, Ep, logtau)
    P = target / target.sum(axis=axis, keepdims=True)
    ns = min(E.shape[0], Ep.shape[0])
    loss = -float(np.sum(P * np.log(Q))) / ns
    dS = (Q - P) / ns
    inv = np.exp(-logtau)
    dE = dS @ Ep * inv
    dEp = dS.T @ E * inv
    g = {k: np.zeros_like(v) for k, v in p.items()}
    g["logtau"][0] = -float(np.sum(dS * S))
    for de, (x, h1, h2) in ((dE, ca), (dEp, cb)):
        g["W3"] += de.T @ h2
        g["b3"] += de.sum(0)
        d2 = (de @ p["W3"]) * (h2 > 0)
        g["W2"] += d2.T @ h1
        g["b2"] += d2.sum(0)
        d1 = (d2 @ p["W2"]) * (h1 > 0)
        g["W1"] += d1.T @ x
        g["b1"] += d1.sum(0)
    return loss, g


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases, tau = sqrt(64) (a fixed seed)."""
    rng = np.random.default_rng([1207, 1114, 4444, seed])
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-bound, bound, size=shp)
        elif name == "logtau":
            p[name] = np.array([np.log(8.0)])
        else:
            p[name] = np.zeros(shp)
    return pack(p)
