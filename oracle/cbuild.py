"""Build and load the C oracle (``csum.c``) with gcc (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csum.c")
LIB = os.path.join(HERE, "libcsum.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def load():
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    f = lib.oracle_triple_sum
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    return lib


def triple_sum(field, X, family: int, I: int, m: int = 0, gradient: bool = False):
    """C oracle triple sum; field float32 or float64 [N,N,N,3]; returns (u, grad|None, threads)."""
    import numpy as np
    from . import kernels
    lib = load()
    field = np.ascontiguousarray(field)
    is32 = field.dtype == np.float32
    if not is32:
        field = np.ascontiguousarray(field, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
    coef = np.ascontiguousarray(kernels.coeff_table_f64(family, I, m))
    dcoef = np.zeros((I, I))
    dcoef[:, : I - 1] = kernels.coeff_table_f64(family, I, m, deriv=True)[:, : I - 1]
    u = np.empty((X.shape[0], 3))
    g = np.empty((X.shape[0], 3, 3)) if gradient else None
    nt = lib.oracle_triple_sum(field.ctypes.data, int(is32), field.shape[0], X.ctypes.data,
                               X.shape[0], coef.ctypes.data, dcoef.ctypes.data, I,
                               u.ctypes.data, g.ctypes.data if gradient else None)
    return u, g, nt
