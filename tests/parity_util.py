"""Comparison of a GPU iterate with a stored FP64 oracle iterate, on every
entry (the stored form is written by tests/golden/make_golden.py: entries
above tau stored exactly, the rest known to lie within [-tau, tau])."""
import numpy as np


def full_error(X, g):
    """Compares every entry of X with a stored oracle iterate (sparse form:
    entries above g["tau"] stored exactly, the rest known to lie within
    [-tau, tau]).  Returns (max error over the stored entries, max |X| over
    the others, an upper bound of max|X - X_ref| over all entries)."""
    assert X.shape == tuple(int(v) for v in g["shape"])
    flat = X.ravel()
    idx, tau = g["idx"], float(g["tau"])
    err = float(np.abs(flat[idx] - g["val"]).max()) if idx.size else 0.0
    rest = np.ones(flat.size, dtype=bool)
    rest[idx] = False
    rmax = float(np.abs(flat[rest]).max()) if rest.any() else 0.0
    return err, rmax, max(err, rmax + tau)


def assert_full_parity(X, g, rel=1e-4):
    """|X - X_ref| <= rel * max X_ref on every entry: a stored entry is
    compared directly, an unstored one (|X_ref| <= tau) passes when
    |X| <= tol - tau."""
    tol = rel * float(g["xmax"])
    err, rmax, bound = full_error(X, g)
    print(f"every entry: stored max err {err:.3e}, other entries max "
          f"{rmax:.3e}, bound {bound:.3e} (tol {tol:.1e}, {g['idx'].size} "
          f"stored of {X.size})")
    assert err <= tol
    assert rmax <= tol - float(g["tau"])
    return bound


# Error of a BF16 run against the FP64 oracle, every entry, relative to
# max X: at most one bfloat16 ulp of the largest entry, 2^-8.  A BF16 run
# rounds X and T to bfloat16 and stops at eps1 = 5e-4 (its eps1 wanders on a
# plateau below ~3e-4 instead of reaching 1e-6), so its iterate is not the
# FP64 fixed point; measured: 4.7e-4 (configuration 1), 6.2e-4
# (configuration 2), 9.1e-4 (n = 2000, from the learned start).
BF16_X_ERR = 2.0 ** -8
