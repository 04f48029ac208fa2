"""ctypes wrapper for sectors128.c (oracle, test only): the sector weights of
one cluster in binary128, from the definition (Schur complement, its
eigenvalues, the power series; no contour).  build() compiles it with gcc."""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sectors128.c")
_LIB = os.path.join(_HERE, "libsectors128.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", _LIB, _SRC, "-lquadmath", "-lm"])
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        _lib.oracle128_sector_weights.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ctypes.c_int, dp, dp]
    return _lib


def sector_weights(W: np.ndarray, T: Sequence[int], L: int) -> Tuple[np.ndarray, np.ndarray]:
    """g_T[kappa], kappa < L, of the sub-ensemble with Q-covariance W (2n x 2n,
    taken as exact) and the cluster T (positions in the clicked set) empty:
    (hi, lo) doubles whose sum carries the binary128 value."""
    lib = _load()
    n = W.shape[0] // 2
    w = np.ascontiguousarray(W, dtype=np.float64)
    t = np.ascontiguousarray(list(T), dtype=np.int32)
    hi, lo = np.zeros(L), np.zeros(L)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.oracle128_sector_weights(n, w.ctypes.data_as(dp), len(t),
                                      t.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if len(t) else None,
                                      L, hi.ctypes.data_as(dp), lo.ctypes.data_as(dp))
    if rc != 0:
        raise ValueError("sectors128: W or W_TT not positive definite")
    return hi, lo
