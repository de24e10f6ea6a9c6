"""Builds and loads ``liboracle.so`` from ``csr_core.c`` (test infrastructure)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "csr_core.c")
LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_csr_spmv.argtypes = [i64, p, p, p, p, p]
        L.oracle_csr_spmv.restype = None
        L.oracle_csr_spmv_t.argtypes = [i64, i64, p, p, p, p, p]
        L.oracle_csr_spmv_t.restype = None
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def csr_spmv(rowptr, col, val, x) -> np.ndarray:
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = rowptr.size - 1
    y = np.empty(n, dtype=np.float64)
    lib().oracle_csr_spmv(n, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y))
    return y


def csr_spmv_t(rowptr, col, val, g, m: int) -> np.ndarray:
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    n = rowptr.size - 1
    y = np.empty(m, dtype=np.float64)
    lib().oracle_csr_spmv_t(n, m, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(g), _ptr(y))
    return y


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(t: int) -> None:
    """Threads of the following parallel loops (the CPU baseline times one
    thread and all of them)."""
    lib().oracle_set_num_threads(int(t))
