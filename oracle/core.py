"""CPU ORACLE (test infrastructure only): ctypes access to thomas_oracle.c.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library.

Functions take NumPy arrays in the RHS-interleaved layout (F[i, n] = row i of
right-hand side n), widen them exactly to FP64, and return FP64 results.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "thomas_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile thomas_oracle.c with gcc (host only, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                        _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64 = ctypes.c_int64
        lib.oracle_thomas.argtypes = [i64, i64, _D, _D, _D, _D]
        lib.oracle_thomas.restype = ctypes.c_int
        lib.oracle_tridiag_general.argtypes = [i64, _D, _D, _D, _D, _D]
        lib.oracle_tridiag_general.restype = ctypes.c_int
        lib.oracle_grad.argtypes = [i64, i64, _D, _D, _D, _D, _D, _D, _D]
        lib.oracle_grad.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _p(x):
    return x.ctypes.data_as(_D)


class OracleError(RuntimeError):
    pass


def thomas(a, b, F):
    """X = A^{-1} F for every column of F (FP64 sequential sweep per RHS)."""
    lib = _load()
    b = _f64(b)
    M = b.shape[0]
    a = _f64(a) if M > 1 else np.zeros(1)
    F = _f64(F)
    squeeze = F.ndim == 1
    if squeeze:
        F = F[:, None]
    N = F.shape[1]
    X = np.empty((M, N))
    rc = lib.oracle_thomas(M, N, _p(a), _p(b), _p(F), _p(X))
    if rc != 0:
        raise OracleError(f"oracle_thomas failed ({rc})")
    return X[:, 0] if squeeze else X


def tridiag_general(lower, diag, upper, rhs):
    """Solve one general tridiagonal system (row i: lower[i] x[i-1] +
    diag[i] x[i] + upper[i] x[i+1] = rhs[i])."""
    lib = _load()
    diag = _f64(diag)
    n = diag.shape[0]
    lower, upper, rhs = _f64(lower), _f64(upper), _f64(rhs)
    assert lower.shape == upper.shape == rhs.shape == (n,)
    x = np.empty(n)
    rc = lib.oracle_tridiag_general(n, _p(lower), _p(diag), _p(upper), _p(rhs), _p(x))
    if rc != 0:
        raise OracleError(f"oracle_tridiag_general failed ({rc})")
    return x


def grad(a, b, X, gX):
    """Adjoint of X = A^{-1} F: returns (gF, ga, gb) in FP64."""
    lib = _load()
    b = _f64(b)
    M = b.shape[0]
    a = _f64(a) if M > 1 else np.zeros(1)
    X, gX = _f64(X), _f64(gX)
    N = X.shape[1]
    gF = np.empty((M, N))
    ga = np.empty(max(M - 1, 1))
    gb = np.empty(M)
    rc = lib.oracle_grad(M, N, _p(a), _p(b), _p(X), _p(gX), _p(gF), _p(ga), _p(gb))
    if rc != 0:
        raise OracleError(f"oracle_grad failed ({rc})")
    return gF, ga[: M - 1], gb


def num_threads() -> int:
    return int(_load().oracle_num_threads())
