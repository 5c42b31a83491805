"""ctypes wrapper of the plain Gaussian elimination in ge.c (oracle; test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ge.c")
_LIB = os.path.join(_HERE, "_build", "liboracle_ge.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ge.c with gcc (OpenMP) into oracle/_build/liboracle_ge.so."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        c_long, c_void_p = ctypes.c_long, ctypes.c_void_p
        lib.oracle_ge_eliminate.restype = c_long
        lib.oracle_ge_eliminate.argtypes = [c_long, c_long, c_void_p, c_long, c_void_p,
                                            c_void_p, c_long, c_long]
        lib.oracle_back_substitute.restype = None
        lib.oracle_back_substitute.argtypes = [c_long, c_long, c_void_p, c_long, c_void_p, c_long]
        lib.oracle_zgesv.restype = c_long
        lib.oracle_zgesv.argtypes = [c_long, c_long, c_void_p, c_long, c_void_p, c_void_p, c_long]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oracle_threads())


def solve(M: np.ndarray, B: np.ndarray) -> tuple[np.ndarray, np.ndarray, int]:
    """Solve M X = B.  Returns (X, LU, ipiv) with LU the packed L\\U factors.

    Raises ZeroDivisionError when an exactly zero pivot column appears.
    """
    lib = _load()
    A = np.array(M, dtype=np.complex128, order="C", copy=True)
    X = np.array(B, dtype=np.complex128, order="C", copy=True)
    if X.ndim == 1:
        X = X[:, None]
    n = A.shape[0]
    ipiv = np.zeros(n, dtype=np.int32)
    info = lib.oracle_zgesv(n, X.shape[1], A.ctypes.data, n, ipiv.ctypes.data,
                            X.ctypes.data, X.shape[1])
    if info != 0:
        raise ZeroDivisionError(f"exactly zero pivot in column {info - 1}")
    return X, A, ipiv


def eliminate_steps(M: np.ndarray, B: np.ndarray, steps: int) -> int:
    """Run the first `steps` elimination steps in place (bounded timing sample)."""
    lib = _load()
    assert M.flags.c_contiguous and B.flags.c_contiguous
    assert M.dtype == np.complex128 and B.dtype == np.complex128
    n = M.shape[0]
    ipiv = np.zeros(n, dtype=np.int32)
    return int(lib.oracle_ge_eliminate(n, B.shape[1], M.ctypes.data, n, ipiv.ctypes.data,
                                       B.ctypes.data, B.shape[1], steps))
