"""Oracle: loader and build step for oracle/liboracle.so (plain C loops).

TEST INFRASTRUCTURE ONLY.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "csrc", "oracle_kernels.c")
LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        # numpy's BLAS threads and OpenMP's threads share the cores; spinning
        # waiters of either starve the other.
        os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        L.oracle_csr_spmm.argtypes = [I, I, P, P, P, P, P]
        L.oracle_csr_spmm.restype = None
        L.oracle_csr_shifted_spmm.argtypes = [I, I, P, P, P, P, P, P, P]
        L.oracle_csr_shifted_spmm.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def spmm(row_ptr, col, val, X):
    """Y = A X, A in CSR (rows = len(row_ptr)-1), X row-major."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n = row_ptr.shape[0] - 1
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    p = X.shape[1]
    Y = np.empty((n, p))
    lib().oracle_csr_spmm(n, p, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(X), _ptr(Y))
    return Y[:, 0] if squeeze else Y


def shifted_spmm(row_ptr, col, lh, b, lam, X):
    """Y[:, l] = (Lh - lam[l] B) X[:, l]."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    n = row_ptr.shape[0] - 1
    p = X.shape[1]
    Y = np.empty((n, p))
    lib().oracle_csr_shifted_spmm(n, p, _ptr(row_ptr), _ptr(col), _ptr(lh), _ptr(b), _ptr(lam),
                                  _ptr(X), _ptr(Y))
    return Y
