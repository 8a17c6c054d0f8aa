"""CPU-side checks of the C ABI: the library loads, exports every entry point
the header declares, and its host-only parts (discretisation, argument
validation, status strings) behave as documented.  No GPU call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import fastpfp_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastpfp.h")


@pytest.fixture(scope="module")
def F():
    from paper_1207_1114_amd import fastpfp
    return fastpfp


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fastpfp_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(F):
    lib = F.lib()
    names = declared_functions()
    assert "fastpfp_solve" in names and "fastpfp_discretize" in names
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(F.EXPORTS) <= set(names)
    assert lib.fastpfp_abi_version() == F.ABI_VERSION == 6


def test_status_strings_and_defaults(F):
    lib = F.lib()
    for s in range(8):
        assert lib.fastpfp_status_string(s).decode()
    p = F.default_params()
    assert (p.alpha, p.tol_outer, p.tol_inner) == (0.5, 1e-6, 1e-8)
    assert (p.max_outer, p.max_inner, p.normalize_max) == (1000, 1000, 1)
    assert p.projection == F.ALTERNATING and p.method == F.METHOD_FASTPFP


def test_null_handle_is_rejected_before_any_device_call(F):
    lib = F.lib()
    p = F.default_params()
    info = F.Info()
    st = lib.fastpfp_solve(None, 4, 4, None, 4, None, 4, None, 4,
                           ctypes.byref(p), None, 4, None, ctypes.byref(info))
    assert st == 1
    assert lib.fastpfp_project(None, 4, None, 1e-6, 10, 0, 0,
                               ctypes.byref(info)) == 1
    assert lib.fastpfp_destroy(None) == 1
    assert lib.fastpfp_project_stream(None, 4, None, 1e-6, 10, 0,
                                      ctypes.byref(info)) == 1
    assert lib.fastpfp_discretize_greedy_batched(None, 1, None, None, None,
                                                 None, None, None,
                                                 None) == 1
    assert lib.fastpfp_autotune(None, 100, 1, 8, None, None, None, 0,
                                None) == 1
    assert lib.fastpfp_warmstart_load(None, None, 0) == 1
    assert lib.fastpfp_warmstart_get(None, None, None, 0) == 1
    assert lib.fastpfp_warmstart_zero_grad(None) == 1
    assert lib.fastpfp_warmstart_adam(None, 1e-3, 0.9, 0.999, 1e-8, 1.0) == 1
    assert lib.fastpfp_warmstart(None, 4, 4, None, 4, None, 4, None, 0, None,
                                 0, 0, 0, None, 4) == 1


def test_warmstart_parameter_count_matches_oracle(F):
    from oracle import warmstart_oracle as W
    txt = open(HEADER).read()
    m = re.search(r"#define FASTPFP_WS_NPARAMS (\d+)", txt)
    assert int(m.group(1)) == W.NPARAMS == F.WS_NPARAMS


@pytest.mark.parametrize("shape", [(1, 1), (6, 6), (5, 9), (9, 5), (40, 55),
                                   (120, 100)])
def test_hungarian_matches_library_assignment(F, shape):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1])
    X = rng.random(shape).astype(np.float32)
    m, score = F.discretize(X, F.HUNGARIAN)
    ref = O.hungarian_discretize(X.astype(np.float64))
    # the optimum can be non-unique: compare scores, then validity
    assert abs(score - O.assignment_score(X.astype(np.float64), ref)) < 1e-9 * max(1, score)
    cols = m[m >= 0]
    assert len(cols) == min(shape) and len(set(cols.tolist())) == len(cols)


def test_hungarian_brute_force_small(F):
    rng = np.random.default_rng(5)
    for _ in range(20):
        X = rng.integers(0, 5, size=(5, 6)).astype(np.float32)
        m, score = F.discretize(X, F.HUNGARIAN)
        assert score == pytest.approx(O.brute_force_assignment(X), abs=1e-9)


@pytest.mark.parametrize("shape", [(7, 7), (5, 11), (11, 5), (64, 80)])
def test_greedy_matches_oracle_including_ties(F, shape):
    rng = np.random.default_rng(shape[0] + 17 * shape[1])
    for ints in (False, True):
        X = (rng.integers(0, 3, size=shape) if ints
             else rng.random(shape)).astype(np.float32)
        m, _ = F.discretize(X, F.GREEDY)
        np.testing.assert_array_equal(m, O.greedy_discretize(X))


def test_discretize_rejects_bad_input(F):
    lib = F.lib()
    X = np.full((3, 3), np.nan, dtype=np.float32)
    match = np.zeros(3, dtype=np.int32)
    st = lib.fastpfp_discretize(3, 3, X.ctypes.data_as(ctypes.c_void_p), 3, 0,
                                match.ctypes.data_as(ctypes.c_void_p), None)
    assert st == 5
    st = lib.fastpfp_discretize(0, 3, X.ctypes.data_as(ctypes.c_void_p), 3, 0,
                                match.ctypes.data_as(ctypes.c_void_p), None)
    assert st == 1
    st = lib.fastpfp_discretize(3, 3, X.ctypes.data_as(ctypes.c_void_p), 3, 7,
                                match.ctypes.data_as(ctypes.c_void_p), None)
    assert st == 1
