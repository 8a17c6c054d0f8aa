"""FP64 CPU oracle for the FastPFP iteration -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The product path (the HIP library and its binding) never
imports it and shares no code with it.

It follows Lu, Huang & Liu, "A Fast Projected Fixed-Point Algorithm for Large
Graph Matching" (arXiv 1207.1114) step by step, in float64, with NumPy
matrix products as the only library primitive:

* ``gradient``            Sec. 4.1: grad f(X) = A X A' + lambda K.
* ``p1``                  Sec. 4.3, eq. (P1): closed-form projection onto
                          {D 1 = 1, D^T 1 = 1}.
* ``p2``                  Sec. 4.3, eq. (P2): (Y + |Y|) / 2.
* ``inner_projection``    Algorithm 1, inner repeat: P1 then P2 until
                          max|Y_{u+1} - Y_u| < eps2 or I1 passes (Sec. 5).
* ``dykstra_inner``       the projection P_D of eq. (DSP) itself, by Dykstra's
                          algorithm over the same two sets (P1, then P2 with a
                          correction term), under the same stopping rule.  The
                          paper's plain alternation only reaches a nearby
                          feasible point (Sec. 4.3 invokes von Neumann's lemma,
                          which is a statement about subspaces, and the set of
                          P2 is a cone); ``projection="dykstra"`` of
                          ``fastpfp`` selects this one.
* ``fastpfp``             Algorithm 1, outer repeat: slack-embedded gradient,
                          inner projection, damped update (eq. fastPFP),
                          max-normalisation (remark after Theorem 1), stop on
                          max|X_{t+1} - X_t| < eps1 or I0 steps (Sec. 5).
* ``projected_gradient``  eq. (pg), Sec. 4.2: X <- P_d(X + alpha grad f(X)),
                          the iteration FastPFP is compared with; same
                          gradient, projection and stopping rule.
* ``greedy_discretize``   Sec. 4.5, steps 1-3 (greedy, from SM).
* ``hungarian_discretize`` the assignment that maximises sum_i X[i, pi(i)],
                          via scipy's linear_sum_assignment (library routine).
* ``objective``           eq. (3): 1/2 tr(P^T A P A') + lambda tr(P^T K).
* ``matching_error``      eq. (1): 1/2 ||A - P A' P^T||^2 + lambda ||F - P G||^2.

Readings taken where the paper is loose:

* Orientation.  The paper assumes n >= n' (columns of X sum to one, rows to
  at most one).  Both orientations are handled natively: Y is N x N with
  N = max(n, n') and the gradient is written into its leading n x n' block;
  the remaining rows (n < n') or columns (n > n') are the slack.  The side
  with fewer nodes therefore gets the "= 1" sums.
* P1 as printed uses 1^T X 1; Algorithm 1 uses 1^T Y 1 over the whole slacked
  N x N matrix, with N in place of n.  The latter is used.
* The slack block starts at zero (the paper initialises Y = 0) and, since
  Algorithm 1 only overwrites the leading block, carries over between outer
  steps.
* The inner stopping test compares the matrix before P1 with the matrix after
  P2 of the same pass.
* eps1 is measured on the stored (normalised) iterates; at t = 1 against X0.
* X0 defaults to c 1 1^T with c = 1 / max(n, n'); the paper's 1/(n n') is
  ``init_scale = 1/(n*n')``.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

DEFAULT_EPS1 = 1e-6
DEFAULT_EPS2 = 1e-8
DEFAULT_I0 = 1000
DEFAULT_I1 = 1000


# ------------------------------------------------------------------ basics
def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (8-bit significand), to nearest, ties to even,
    through float32; returned as float64.  Defines the reduced-precision
    product recipe below, not part of the paper."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(
        np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gradient(A: np.ndarray, X: np.ndarray, B: np.ndarray,
             K: Optional[np.ndarray], lam: float,
             products: str = "fp64") -> np.ndarray:
    """Sec. 4.1: grad f(X) = A X A' + lambda K (A, A' symmetric).

    products="bf16" evaluates A X A' with bfloat16 operands: A, A' and X
    rounded to bfloat16, T = A X formed exactly and rounded to bfloat16,
    then T A' formed exactly (the reduced-precision form of the products)."""
    if products == "bf16":
        T = bf16_round(bf16_round(A) @ bf16_round(X))
        G = T @ bf16_round(B)
    else:
        G = (A @ X) @ B
    if lam != 0.0:
        G = G + lam * K
    return G


def p1(Y: np.ndarray) -> np.ndarray:
    """Eq. (P1) for a square N x N matrix.

    D = Y + (1/N) 1 1^T + (1^T Y 1 / N^2) 1 1^T - (1/N) Y 1 1^T
          - (1/N) 1 1^T Y,
    i.e. D_ij = Y_ij + 1/N + s/N^2 - r_i/N - c_j/N with r = Y 1, c = Y^T 1,
    s = 1^T Y 1.
    """
    N = Y.shape[0]
    assert Y.shape == (N, N)
    r = Y.sum(axis=1)
    c = Y.sum(axis=0)
    s = r.sum()
    return Y + 1.0 / N + s / N ** 2 - r[:, None] / N - c[None, :] / N


def p2(Y: np.ndarray) -> np.ndarray:
    """Eq. (P2): (Y + |Y|) / 2."""
    return (Y + np.abs(Y)) / 2.0


@dataclass
class InnerResult:
    Y: np.ndarray
    iters: int
    last_delta: float
    converged: bool


def inner_projection(Y: np.ndarray, eps2: float = DEFAULT_EPS2,
                     max_inner: int = DEFAULT_I1) -> InnerResult:
    """Algorithm 1's inner repeat: Y <- P2(P1(Y)) until it stops moving.

    Stops when max|Y_after - Y_before| < eps2 (Sec. 5, convergence criteria)
    or after ``max_inner`` passes.
    """
    d = np.inf
    for u in range(1, max_inner + 1):
        Yp = Y
        Y = p2(p1(Y))
        d = float(np.max(np.abs(Y - Yp)))
        if d < eps2:
            return InnerResult(Y, u, d, True)
    return InnerResult(Y, max_inner, d, False)


def dykstra_inner(Y: np.ndarray, eps2: float = DEFAULT_EPS2,
                  max_inner: int = DEFAULT_I1) -> InnerResult:
    """P_D(Y) of eq. (DSP) by Dykstra's algorithm (Boyle & Dykstra, 1986).

    Each pass projects onto the affine set of eq. (PP1) with P1 and onto the
    cone of eq. (PP2) with P2.  The affine step needs no correction term; the
    cone step carries q, the part of its input that the last clamp removed:
    z = P1(x); x' = P2(z + q); q' = z + q - x'.  Stops when
    max|x' - x| < eps2 or after ``max_inner`` passes, as the plain inner
    repeat does.
    """
    x = np.array(Y, dtype=np.float64)
    q = np.zeros_like(x)
    d = np.inf
    for u in range(1, max_inner + 1):
        z = p1(x)
        xn = p2(z + q)
        q = z + q - xn
        d = float(np.max(np.abs(xn - x)))
        x = xn
        if d < eps2:
            return InnerResult(x, u, d, True)
    return InnerResult(x, max_inner, d, False)


def dykstra_projection(Y: np.ndarray, tol: float = 1e-13,
                       max_iter: int = 200000) -> np.ndarray:
    """The exact projection to tight tolerance (tests of Lemma 1 and
    Theorem 1, which are statements about P_D itself)."""
    return dykstra_inner(Y, tol, max_iter).Y


# --------------------------------------------------------------- the solve
@dataclass
class SolveResult:
    X: np.ndarray
    slack: np.ndarray          # the full N x N Y at exit (slack part persists)
    outer_iters: int
    inner_iters: list[int]
    eps1_trace: list[float]
    converged: bool
    eps2_last: list[float] = field(default_factory=list)


def uniform_x0(n: int, np_: int, init_scale: float = 0.0) -> np.ndarray:
    c = init_scale if init_scale > 0 else 1.0 / max(n, np_)
    return np.full((n, np_), c)


def fastpfp(A: np.ndarray, B: np.ndarray, K: Optional[np.ndarray],
            lam: float, alpha: float = 0.5, eps1: float = DEFAULT_EPS1,
            eps2: float = DEFAULT_EPS2, max_outer: int = DEFAULT_I0,
            max_inner: int = DEFAULT_I1, X0: Optional[np.ndarray] = None,
            Y0: Optional[np.ndarray] = None, normalize_max: bool = True,
            projector: Optional[Callable[[np.ndarray], np.ndarray]] = None,
            products: str = "fp64",
            projection: str = "alternating") -> SolveResult:
    """Algorithm 1 in float64.

    ``projection``: "alternating" is the inner repeat of Algorithm 1;
    "dykstra" computes eq. (DSP)'s projection with ``dykstra_inner`` under
    the same eps2 / I1.  ``projector`` replaces the inner repeat by any
    function (tests of Lemma 1 / Theorem 1); ``Y0`` resumes with a given
    N x N state.
    """
    inner = {"alternating": inner_projection,
             "dykstra": dykstra_inner}[projection]
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    n, np_ = A.shape[0], B.shape[0]
    N = max(n, np_)
    X = uniform_x0(n, np_) if X0 is None else np.array(X0, dtype=np.float64)
    Y = np.zeros((N, N)) if Y0 is None else np.array(Y0, dtype=np.float64)
    inner_counts, trace, e2s = [], [], []
    converged = False
    t = 0
    for t in range(1, max_outer + 1):
        Y = Y.copy()
        Y[:n, :np_] = gradient(A, X, B, K, lam, products)  # step 3
        if projector is None:
            res = inner(Y, eps2, max_inner)              # steps 4-7
            Y = res.Y
            inner_counts.append(res.iters)
            e2s.append(res.last_delta)
        else:
            Y = projector(Y)
            inner_counts.append(0)
        Xn = (1.0 - alpha) * X + alpha * Y[:n, :np_]     # step 8
        if normalize_max:
            Xn = Xn / Xn.max()                           # step 9
        e1 = float(np.max(np.abs(Xn - X)))
        trace.append(e1)
        X = Xn
        if e1 < eps1:
            converged = True
            break
    return SolveResult(X, Y, t, inner_counts, trace, converged, e2s)


def projected_gradient(A: np.ndarray, B: np.ndarray, K: Optional[np.ndarray],
                       lam: float, alpha: float, eps1: float = DEFAULT_EPS1,
                       eps2: float = DEFAULT_EPS2,
                       max_outer: int = DEFAULT_I0,
                       max_inner: int = DEFAULT_I1,
                       X0: Optional[np.ndarray] = None,
                       normalize_max: bool = False,
                       projection: str = "alternating",
                       products: str = "fp64") -> SolveResult:
    """The Projected Gradient iteration of eq. (pg), Sec. 4.2:
    X <- P_d(X + alpha grad f(X)), with the same gradient (Sec. 4.1), the same
    slack embedding and inner projection as ``fastpfp`` (the slack block
    carries over between steps, as in Algorithm 1) and the same stopping
    rule.  There is no damping term and, by default, no max-normalisation
    (eq. (pg) has neither); alpha is the step size and may exceed 1.
    """
    inner = {"alternating": inner_projection,
             "dykstra": dykstra_inner}[projection]
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    n, np_ = A.shape[0], B.shape[0]
    N = max(n, np_)
    X = uniform_x0(n, np_) if X0 is None else np.array(X0, dtype=np.float64)
    Y = np.zeros((N, N))
    inner_counts, trace, e2s = [], [], []
    converged = False
    t = 0
    for t in range(1, max_outer + 1):
        Y = Y.copy()
        Y[:n, :np_] = X + alpha * gradient(A, X, B, K, lam, products)
        res = inner(Y, eps2, max_inner)
        Y = res.Y
        inner_counts.append(res.iters)
        e2s.append(res.last_delta)
        Xn = Y[:n, :np_].copy()
        if normalize_max:
            Xn = Xn / Xn.max()
        e1 = float(np.max(np.abs(Xn - X)))
        trace.append(e1)
        X = Xn
        if e1 < eps1:
            converged = True
            break
    return SolveResult(X, Y, t, inner_counts, trace, converged, e2s)


# ------------------------------------------------------- discretisation
def greedy_discretize(X: np.ndarray) -> np.ndarray:
    """Sec. 4.5: pick the largest remaining entry, drop its row and column.

    Ties go to the smallest row-major index.  Returns match[i] (column or -1).
    """
    n, m = X.shape
    W = np.array(X, dtype=np.float64)
    match = np.full(n, -1, dtype=np.int64)
    alive = np.ones((n, m), dtype=bool)
    for _ in range(min(n, m)):
        Wm = np.where(alive, W, -np.inf)
        k = int(np.argmax(Wm))
        i, j = divmod(k, m)
        match[i] = j
        alive[i, :] = False
        alive[:, j] = False
    return match


def hungarian_discretize(X: np.ndarray) -> np.ndarray:
    """Maximum-weight assignment of min(n, n') pairs (library routine)."""
    from scipy.optimize import linear_sum_assignment
    r, c = linear_sum_assignment(np.asarray(X, dtype=np.float64),
                                 maximize=True)
    match = np.full(X.shape[0], -1, dtype=np.int64)
    match[r] = c
    return match


def assignment_score(X: np.ndarray, match: np.ndarray) -> float:
    i = np.nonzero(match >= 0)[0]
    return float(np.sum(X[i, match[i]]))


def match_to_matrix(match: np.ndarray, np_: int) -> np.ndarray:
    P = np.zeros((len(match), np_))
    i = np.nonzero(match >= 0)[0]
    P[i, match[i]] = 1.0
    return P


def objective(A, B, K, lam, match) -> float:
    """Eq. (3): 1/2 tr(P^T A P A') + lambda tr(P^T K) for a partial
    permutation given as match[i]."""
    P = match_to_matrix(match, B.shape[0])
    f = 0.5 * np.trace(P.T @ A @ P @ B)
    if lam != 0.0 and K is not None:
        f += lam * np.trace(P.T @ K)
    return float(f)


def relaxed_objective(A, B, K, lam, X) -> float:
    f = 0.5 * float(np.sum((A @ X @ B) * X))
    if lam != 0.0 and K is not None:
        f += lam * float(np.sum(X * K))
    return f


def matching_error(A, B, match, F=None, G=None, lam: float = 0.0) -> float:
    """Eq. (1) evaluated at a partial permutation."""
    P = match_to_matrix(match, B.shape[0])
    e = 0.5 * float(np.sum((A - P @ B @ P.T) ** 2))
    if lam != 0.0 and F is not None:
        e += lam * float(np.sum((F - P @ G) ** 2))
    return e


def accuracy(match: np.ndarray, perm: np.ndarray) -> float:
    """Fraction of nodes with a planted partner that got exactly it."""
    has = perm >= 0
    return float(np.mean(match[has] == perm[has]))


def brute_force_best(A, B, K, lam) -> tuple[float, np.ndarray]:
    """max over all injective maps of the smaller side into the larger one
    of the eq. (3) objective.  For n, n' <= 8 only."""
    n, m = A.shape[0], B.shape[0]
    best, arg = -np.inf, None
    if n <= m:
        for cols in itertools.permutations(range(m), n):
            match = np.array(cols)
            f = objective(A, B, K, lam, match)
            if f > best:
                best, arg = f, match
    else:
        for rows in itertools.permutations(range(n), m):
            match = np.full(n, -1)
            match[list(rows)] = np.arange(m)
            f = objective(A, B, K, lam, match)
            if f > best:
                best, arg = f, match
    return best, arg


def brute_force_assignment(X: np.ndarray) -> float:
    """max over injective assignments of sum X[i, pi(i)] (n, n' <= 8)."""
    n, m = X.shape
    best = -np.inf
    if n <= m:
        for cols in itertools.permutations(range(m), n):
            best = max(best, float(np.sum(X[np.arange(n), list(cols)])))
    else:
        for rows in itertools.permutations(range(n), m):
            best = max(best, float(np.sum(X[list(rows), np.arange(m)])))
    return best
