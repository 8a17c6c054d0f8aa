"""Scores of a discrete matching, used to report and to gate results.

Host-side bookkeeping on a matching returned by the library's discretisation
(``match[i]`` = column of row i, or -1), not part of the solve:

* ``matching_objective``: eq. (3) at the partial permutation P of ``match``,
  1/2 tr(P^T A P A') + lambda tr(P^T K) = 1/2 sum_{i,k matched}
  A[i,k] A'[m(i), m(k)] + lambda sum_i K[i, m(i)] (A' symmetric).
* ``accuracy``: the fraction of nodes with a planted partner that were
  matched to exactly that partner.
* ``frobenius_error``: eq. (1) without the attribute term, the matching
  error the paper reports for its unweighted benchmark (Sec. 5.1),
  ||A - P A' P^T||_F^2 with (P A' P^T)[i,k] = A'[m(i), m(k)] for matched
  rows and 0 otherwise.
"""
from __future__ import annotations

import numpy as np


def matching_objective(A, B, K, lam: float, match) -> float:
    match = np.asarray(match)
    i = np.nonzero(match >= 0)[0]
    j = match[i]
    f = 0.5 * float(np.sum(np.asarray(A, np.float64)[np.ix_(i, i)]
                           * np.asarray(B, np.float64)[np.ix_(j, j)]))
    if lam != 0.0 and K is not None:
        f += lam * float(np.sum(np.asarray(K, np.float64)[i, j]))
    return f


def accuracy(match, perm) -> float:
    match, perm = np.asarray(match), np.asarray(perm)
    has = perm >= 0
    return float(np.mean(match[has] == perm[has]))


def frobenius_error(A, B, match) -> float:
    A = np.asarray(A, np.float64)
    match = np.asarray(match)
    PBP = np.zeros_like(A)
    i = np.nonzero(match >= 0)[0]
    PBP[np.ix_(i, i)] = np.asarray(B, np.float64)[np.ix_(match[i], match[i])]
    return float(np.sum((A - PBP) ** 2))
