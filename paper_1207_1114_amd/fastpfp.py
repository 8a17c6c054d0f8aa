"""Python binding of libfastpfp.so (the C ABI declared in include/fastpfp.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and the HIP stream.  The
library must be built first (``python -m paper_1207_1114_amd.build``); if it
is missing, importing this module raises, so nothing silently falls back to a
CPU path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "libfastpfp.so")

FP32, BF16 = 0, 1
INIT_UNIFORM, INIT_USER = 0, 1
HUNGARIAN, GREEDY = 0, 1
ALTERNATING, DYKSTRA = 0, 1
METHOD_FASTPFP, METHOD_PG = 0, 1
ABI_VERSION = 6

STATUS = {0: "ok", 1: "invalid argument", 2: "shape out of range",
          3: "HIP runtime error", 4: "out of device memory",
          5: "non-finite values", 6: "device wait timed out",
          7: "unsupported request"}

EXPORTS = ("fastpfp_params_default", "fastpfp_create", "fastpfp_destroy",
           "fastpfp_solve", "fastpfp_solve_noalloc", "fastpfp_solve_batched",
           "fastpfp_project",
           "fastpfp_discretize_greedy_batched", "fastpfp_project_stream",
           "fastpfp_discretize", "fastpfp_get_trace", "fastpfp_status_string",
           "fastpfp_last_error", "fastpfp_abi_version",
           "fastpfp_warmstart_load", "fastpfp_warmstart_get",
           "fastpfp_warmstart_features", "fastpfp_warmstart",
           "fastpfp_warmstart_grad", "fastpfp_warmstart_zero_grad",
           "fastpfp_warmstart_adam", "fastpfp_warmstart_batched",
           "fastpfp_autotune")

WS_NPARAMS = 31041
WS_BF16_WEIGHTS = 1


class Params(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("alpha", ctypes.c_double),
                ("tol_outer", ctypes.c_double), ("tol_inner", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("max_inner", ctypes.c_int),
                ("precision", ctypes.c_int), ("init", ctypes.c_int),
                ("init_scale", ctypes.c_double),
                ("normalize_max", ctypes.c_int), ("team_size", ctypes.c_int),
                ("projection", ctypes.c_int), ("method", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int),
                ("inner_iters_total", ctypes.c_int),
                ("inner_iters_max", ctypes.c_int),
                ("inner_capped", ctypes.c_int), ("converged", ctypes.c_int),
                ("status", ctypes.c_int), ("eps1_last", ctypes.c_double),
                ("eps2_last", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("gemm_ms", ctypes.c_double), ("proj_ms", ctypes.c_double),
                ("pair_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class FastPFPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing; build it with "
            "`python -m paper_1207_1114_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, I, L = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER
    lib.fastpfp_params_default.argtypes = [L(Params)]
    lib.fastpfp_create.argtypes = [L(P), I, I, I, P]
    lib.fastpfp_destroy.argtypes = [P]
    lib.fastpfp_solve.argtypes = [P, I, I, P, I, P, I, P, I, L(Params), P, I,
                                  P, L(Info)]
    lib.fastpfp_solve_noalloc.argtypes = lib.fastpfp_solve.argtypes
    lib.fastpfp_solve_batched.argtypes = [P, I, P, P, P, P, P, P, P, P,
                                          L(Params), P, P, P]
    lib.fastpfp_project.argtypes = [P, I, P, ctypes.c_double, I, I, I,
                                    L(Info)]
    lib.fastpfp_discretize.argtypes = [I, I, P, I, I, P, L(ctypes.c_double)]
    lib.fastpfp_get_trace.argtypes = [P, P, I, L(I)]
    D = ctypes.c_double
    lib.fastpfp_warmstart_load.argtypes = [P, P, ctypes.c_size_t]
    lib.fastpfp_warmstart_get.argtypes = [P, P, P, ctypes.c_size_t]
    lib.fastpfp_warmstart_features.argtypes = [P, I, P, I, P, I, I, P, I]
    lib.fastpfp_warmstart.argtypes = [P, I, I, P, I, P, I, P, I, P, I, I, I,
                                      P, I]
    lib.fastpfp_warmstart_batched.argtypes = [P, I, P, P, P, P, P, P, P, P,
                                              P, P, I, I, P, P, P]
    lib.fastpfp_warmstart_grad.argtypes = [P, I, I, P, I, P, I, P, I, P, I,
                                           I, P, I, L(D)]
    lib.fastpfp_warmstart_zero_grad.argtypes = [P]
    lib.fastpfp_warmstart_adam.argtypes = [P, D, D, D, D, D]
    lib.fastpfp_autotune.argtypes = [P, I, I, I, L(I), P, P, I, L(I)]
    lib.fastpfp_discretize_greedy_batched.argtypes = [P, I, P, P, P, P, P, P,
                                                      P]
    lib.fastpfp_project_stream.argtypes = [P, I, P, ctypes.c_double, I, I,
                                           L(Info)]
    lib.fastpfp_status_string.argtypes = [I]
    lib.fastpfp_status_string.restype = ctypes.c_char_p
    lib.fastpfp_last_error.argtypes = [P]
    lib.fastpfp_last_error.restype = ctypes.c_char_p
    for name in ("fastpfp_params_default", "fastpfp_create",
                 "fastpfp_destroy", "fastpfp_solve", "fastpfp_solve_noalloc",
                 "fastpfp_solve_batched",
                 "fastpfp_project", "fastpfp_discretize",
                 "fastpfp_get_trace", "fastpfp_abi_version",
                 "fastpfp_warmstart_load", "fastpfp_warmstart_get",
                 "fastpfp_warmstart_features", "fastpfp_warmstart",
                 "fastpfp_warmstart_grad", "fastpfp_warmstart_zero_grad",
                 "fastpfp_warmstart_adam", "fastpfp_warmstart_batched",
                 "fastpfp_autotune", "fastpfp_discretize_greedy_batched",
                 "fastpfp_project_stream"):
        getattr(lib, name).restype = ctypes.c_int
    if lib.fastpfp_abi_version() != ABI_VERSION:
        raise ImportError(
            f"{path} has ABI {lib.fastpfp_abi_version()}, this binding needs "
            f"{ABI_VERSION}; rebuild with `python -m paper_1207_1114_amd.build`")
    return lib


_LIB: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def default_params(**kw) -> Params:
    p = Params()
    lib().fastpfp_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, "lambda_" if k in ("lam", "lambda") else k, v)
    return p


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _check_dev(t, name):
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device torch.Tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D row-major matrix")


class Solver:
    """A library handle bound to one device and one stream."""

    def __init__(self, max_n: int, max_np: int, device: int = 0,
                 stream=None):
        import torch
        self._lib = lib()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = self._lib.fastpfp_create(ctypes.byref(h), device, max_n, max_np,
                                      ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise FastPFPError(st, "fastpfp_create failed")
        self._h = h
        self.max_n, self.max_np, self.device = max_n, max_np, device

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fastpfp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        raise FastPFPError(st, self._lib.fastpfp_last_error(self._h)
                           .decode(errors="replace"))

    def solve(self, A, B, K, X, params: Params, Y_state=None) -> dict:
        """In-place solve of one pair; X holds X0 (INIT_USER) and the result."""
        return self._solve(self._lib.fastpfp_solve, A, B, K, X, params,
                           Y_state)

    def solve_noalloc(self, A, B, K, X, params: Params, Y_state=None) -> dict:
        """solve() through fastpfp_solve_noalloc: no device allocation, the
        library's fixed per-device scratch instead (max(n, n') <= 1024)."""
        return self._solve(self._lib.fastpfp_solve_noalloc, A, B, K, X,
                           params, Y_state)

    def _solve(self, fn, A, B, K, X, params, Y_state) -> dict:
        for t, nm in ((A, "A"), (B, "B"), (K, "K"), (X, "X"),
                      (Y_state, "Y_state")):
            _check_dev(t, nm)
        n, np_ = A.shape[0], B.shape[0]
        info = Info()
        st = fn(self._h, n, np_, _ptr(A), A.stride(0), _ptr(B), B.stride(0),
                _ptr(K), K.stride(0) if K is not None else 0,
                ctypes.byref(params), _ptr(X), X.stride(0), _ptr(Y_state),
                ctypes.byref(info))
        if st != 0:
            self._raise(st)
        return info.as_dict()

    def solve_batched(self, n: Sequence[int], np_: Sequence[int], A, offA,
                      B, offB, K, offK, X, offX, params: Params) -> list:
        """Packed ragged batch: A, B, K, X are flat float32 device tensors;
        off* are element offsets (host sequences)."""
        b = len(n)
        ni = np.asarray(n, dtype=np.int32)
        npi = np.asarray(np_, dtype=np.int32)
        oa, ob, ox = (np.asarray(o, dtype=np.int64) for o in (offA, offB, offX))
        ok = np.asarray(offK if offK is not None else np.zeros(b),
                        dtype=np.int64)
        infos = (Info * b)()
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        st = self._lib.fastpfp_solve_batched(
            self._h, b, c(ni), c(npi), _ptr(A), c(oa), _ptr(B), c(ob),
            _ptr(K), c(ok), ctypes.byref(params), _ptr(X), c(ox), infos)
        out = [i.as_dict() for i in infos]
        if st != 0:
            err = FastPFPError(st, self._lib.fastpfp_last_error(self._h)
                               .decode(errors="replace"))
            err.infos = out
            raise err
        return out

    def project(self, Y, tol: float, max_inner: int, team_size: int = 0,
                projection: int = ALTERNATING) -> dict:
        _check_dev(Y, "Y")
        if Y.shape[0] != Y.shape[1] or not Y.is_contiguous():
            raise ValueError("Y must be a contiguous square matrix")
        info = Info()
        st = self._lib.fastpfp_project(self._h, Y.shape[0], _ptr(Y), tol,
                                       max_inner, team_size, projection,
                                       ctypes.byref(info))
        if st != 0:
            self._raise(st)
        return info.as_dict()

    def project_stream(self, Y, tol: float, max_inner: int,
                       projection: int = ALTERNATING) -> dict:
        """Steps 4-7 with Y kept in device memory (any N; HBM-bound)."""
        _check_dev(Y, "Y")
        if Y.shape[0] != Y.shape[1] or not Y.is_contiguous():
            raise ValueError("Y must be a contiguous square matrix")
        info = Info()
        st = self._lib.fastpfp_project_stream(self._h, Y.shape[0], _ptr(Y),
                                              tol, max_inner, projection,
                                              ctypes.byref(info))
        if st != 0:
            self._raise(st)
        return info.as_dict()

    def autotune(self, N: int, batch: int, passes: int = 256) -> tuple:
        """(best team size, [(team size, pair-passes per second), ...])."""
        cap = 16
        Ws = np.zeros(cap, dtype=np.int32)
        rates = np.zeros(cap, dtype=np.float64)
        best, cnt = ctypes.c_int(), ctypes.c_int()
        st = self._lib.fastpfp_autotune(
            self._h, N, batch, passes, ctypes.byref(best),
            Ws.ctypes.data_as(ctypes.c_void_p),
            rates.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(cnt))
        if st != 0:
            self._raise(st)
        return best.value, list(zip(Ws[:cnt.value].tolist(),
                                     rates[:cnt.value].tolist()))

    def discretize_greedy_batched(self, n: Sequence[int], np_: Sequence[int],
                                  X, offX, match, offM) -> list:
        """Device greedy discretisation of a packed batch (X flat float32,
        match flat int32, both device tensors; offsets in elements).
        Returns the per-pair statuses; raises on a non-OK call status."""
        import torch
        b = len(n)
        if not (isinstance(match, torch.Tensor) and match.is_cuda
                and match.dtype == torch.int32):
            raise TypeError("match must be a device int32 tensor")
        if not (isinstance(X, torch.Tensor) and X.is_cuda
                and X.dtype == torch.float32):
            raise TypeError("X must be a device float32 tensor")
        ni = np.asarray(n, dtype=np.int32)
        npi = np.asarray(np_, dtype=np.int32)
        ox = np.asarray(offX, dtype=np.int64)
        om = np.asarray(offM, dtype=np.int64)
        stat = np.zeros(b, dtype=np.int32)
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        st = self._lib.fastpfp_discretize_greedy_batched(
            self._h, b, c(ni), c(npi), _ptr(X), c(ox), _ptr(match), c(om),
            c(stat))
        if st != 0:
            err = FastPFPError(st, self._lib.fastpfp_last_error(self._h)
                               .decode(errors="replace"))
            err.statuses = stat.tolist()
            raise err
        return stat.tolist()

    def discretize_greedy(self, X):
        """Device greedy discretisation of one n x n' device matrix;
        returns a device int32 tensor of n columns (-1 = unmatched)."""
        import torch
        _check_dev(X, "X")
        Xc = X.contiguous()
        match = torch.empty(Xc.shape[0], dtype=torch.int32, device=Xc.device)
        self.discretize_greedy_batched([Xc.shape[0]], [Xc.shape[1]],
                                       Xc.view(-1), [0], match, [0])
        return match

    # -- learned warm start ------------------------------------------------

    def warmstart_load(self, params: np.ndarray) -> None:
        """Loads the FASTPFP_WS_NPARAMS network parameters (host array)."""
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        if p.size != WS_NPARAMS:
            raise ValueError(f"need {WS_NPARAMS} parameters, got {p.size}")
        st = self._lib.fastpfp_warmstart_load(
            self._h, p.ctypes.data_as(ctypes.c_void_p), p.nbytes)
        if st != 0:
            self._raise(st)

    def warmstart_get(self) -> tuple:
        """(parameters, accumulated gradient) as host float32 arrays."""
        p = np.zeros(WS_NPARAMS, dtype=np.float32)
        g = np.zeros(WS_NPARAMS, dtype=np.float32)
        st = self._lib.fastpfp_warmstart_get(
            self._h, p.ctypes.data_as(ctypes.c_void_p),
            g.ctypes.data_as(ctypes.c_void_p), WS_NPARAMS)
        if st != 0:
            self._raise(st)
        return p, g

    @staticmethod
    def _attr(F):
        if F is None:
            return None, 0, 0
        _check_dev(F, "F")
        return _ptr(F), F.stride(0), F.shape[1]

    def warmstart_features(self, A, F=None):
        import torch
        _check_dev(A, "A")
        n = A.shape[0]
        fp, ldf, fdim = self._attr(F)
        x = torch.empty((n, 48), dtype=torch.float32, device=A.device)
        st = self._lib.fastpfp_warmstart_features(
            self._h, n, _ptr(A), A.stride(0), fp, ldf, fdim, _ptr(x), 48)
        if st != 0:
            self._raise(st)
        return x

    def warmstart(self, A, B, F, G, X0, bf16_weights: bool = False) -> None:
        """Writes the learned X0 into X0 (n x n' device tensor)."""
        for t, nm in ((A, "A"), (B, "B"), (X0, "X0")):
            _check_dev(t, nm)
        fp, ldf, fdim = self._attr(F)
        gp, ldg, gdim = self._attr(G)
        if fdim != gdim:
            raise ValueError("F and G need the same attribute count")
        st = self._lib.fastpfp_warmstart(
            self._h, A.shape[0], B.shape[0], _ptr(A), A.stride(0), _ptr(B),
            B.stride(0), fp, ldf, gp, ldg, fdim,
            WS_BF16_WEIGHTS if bf16_weights else 0, _ptr(X0), X0.stride(0))
        if st != 0:
            self._raise(st)

    def warmstart_batched(self, n, np_, A, offA, B, offB, F, offF, G, offG,
                          fdim: int, X, offX, bf16_weights: bool = False
                          ) -> list:
        """Packed batch (flat float32 device tensors, host element offsets);
        returns the per-pair status list (0 = OK, 5 = non-finite X0)."""
        b = len(n)
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        ni = np.asarray(n, dtype=np.int32)
        npi = np.asarray(np_, dtype=np.int32)
        oa, ob, ox = (np.asarray(o, dtype=np.int64) for o in (offA, offB, offX))
        of = np.asarray(offF if offF is not None else np.zeros(b), np.int64)
        og = np.asarray(offG if offG is not None else np.zeros(b), np.int64)
        status = np.zeros(b, dtype=np.int32)
        st = self._lib.fastpfp_warmstart_batched(
            self._h, b, c(ni), c(npi), _ptr(A), c(oa), _ptr(B), c(ob),
            _ptr(F) if fdim else None, c(of) if fdim else None,
            _ptr(G) if fdim else None, c(og) if fdim else None, fdim,
            WS_BF16_WEIGHTS if bf16_weights else 0, _ptr(X), c(ox),
            c(status))
        if st not in (0, 5):
            self._raise(st)
        return status.tolist()

    def warmstart_grad(self, A, B, F, G, T) -> float:
        """Accumulates the gradient of the loss against target T; returns
        the loss."""
        for t, nm in ((A, "A"), (B, "B"), (T, "T")):
            _check_dev(t, nm)
        fp, ldf, fdim = self._attr(F)
        gp, ldg, gdim = self._attr(G)
        if fdim != gdim:
            raise ValueError("F and G need the same attribute count")
        loss = ctypes.c_double()
        st = self._lib.fastpfp_warmstart_grad(
            self._h, A.shape[0], B.shape[0], _ptr(A), A.stride(0), _ptr(B),
            B.stride(0), fp, ldf, gp, ldg, fdim, _ptr(T), T.stride(0),
            ctypes.byref(loss))
        if st != 0:
            self._raise(st)
        return loss.value

    def warmstart_zero_grad(self) -> None:
        st = self._lib.fastpfp_warmstart_zero_grad(self._h)
        if st != 0:
            self._raise(st)

    def warmstart_adam(self, lr: float, beta1: float = 0.9,
                       beta2: float = 0.999, eps: float = 1e-8,
                       grad_scale: float = 1.0) -> None:
        st = self._lib.fastpfp_warmstart_adam(self._h, lr, beta1, beta2, eps,
                                              grad_scale)
        if st != 0:
            self._raise(st)

    def trace(self, cap: int = 100000) -> np.ndarray:
        out = np.zeros(cap, dtype=np.float64)
        cnt = ctypes.c_int()
        self._lib.fastpfp_get_trace(self._h,
                                    out.ctypes.data_as(ctypes.c_void_p), cap,
                                    ctypes.byref(cnt))
        return out[:cnt.value].copy()


def discretize(X: np.ndarray, method: int = HUNGARIAN) -> tuple:
    """Host discretisation (Sec. 4.5).  Returns (match int32[n], score)."""
    Xc = np.ascontiguousarray(X, dtype=np.float32)
    n, m = Xc.shape
    match = np.zeros(n, dtype=np.int32)
    score = ctypes.c_double()
    st = lib().fastpfp_discretize(n, m, Xc.ctypes.data_as(ctypes.c_void_p),
                                  m, method,
                                  match.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(score))
    if st != 0:
        raise FastPFPError(st, "fastpfp_discretize failed")
    return match, score.value
