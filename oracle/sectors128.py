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


def _cluster_job(args):
    W, T, L = args
    hi, lo = sector_weights(W, T, L)
    return hi, lo


def cluster_moments(W: np.ndarray, jmax: int, L: int, workers: int = 1) -> np.ndarray:
    """S_t[kappa] = sum over the clusters T of t positions of g_T[kappa], t = 0..jmax,
    kappa < L (Methods, Moments calculation), every g_T in binary128: [jmax+1, L].
    The sum runs in fp64 over the (hi + lo) values; every g_T[kappa] is >= 0 (a
    sub-ensemble weight), so it adds no cancellation."""
    import itertools
    n = W.shape[0] // 2
    S = np.zeros((jmax + 1, L))
    for t in range(jmax + 1):
        jobs = [(W, T, L) for T in itertools.combinations(range(n), t)]
        if workers > 1 and len(jobs) > 1:
            from multiprocessing import Pool
            with Pool(workers) as pool:
                res = pool.map(_cluster_job, jobs, chunksize=max(1, len(jobs) // (4 * workers)))
        else:
            res = [_cluster_job(j) for j in jobs]
        for hi, lo in res:
            S[t] += hi + lo
    return S
