"""ctypes wrapper for exact128.c (oracle, test only).  build() compiles it with gcc."""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exact128.c")
_LIB = os.path.join(_HERE, "libexact128.so")
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
        _lib.oracle128_exact.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int, ip, ip,
                                         dp, dp, dp, dp]
        _lib.oracle128_q_matrix.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, dp, dp]
    return _lib


def _d(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def exact(M: int, U: Optional[np.ndarray], r, eta, offsets, modes, sigma=None):
    """binary128 exact click probabilities.  Returns dict(p_hi, p_lo, logp, kappa)."""
    lib = _load()
    P = len(offsets) - 1
    ure = _d(U.real) if U is not None else None
    uim = _d(U.imag) if U is not None else None
    r = _d(r); eta = _d(eta); sg = _d(sigma)
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    mod = np.ascontiguousarray(modes, dtype=np.int32)
    out = {k: np.zeros(P) for k in ("p_hi", "p_lo", "logp", "kappa")}
    rc = lib.oracle128_exact(M, _ptr(ure), _ptr(uim), _ptr(r), _ptr(eta), _ptr(sg), P,
                             off.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                             mod.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                             _ptr(out["p_hi"]), _ptr(out["p_lo"]), _ptr(out["logp"]),
                             _ptr(out["kappa"]))
    if rc != 0:
        raise ValueError(f"oracle128_exact: block not positive definite (row {-rc - 1})")
    return out


def q_matrix(M: int, U, r, eta, sigma=None):
    lib = _load()
    ure = _d(U.real) if U is not None else None
    uim = _d(U.imag) if U is not None else None
    hi = np.zeros((2 * M, 2 * M)); lo = np.zeros((2 * M, 2 * M))
    lib.oracle128_q_matrix(M, _ptr(ure), _ptr(uim), _ptr(_d(r)), _ptr(_d(eta)), _ptr(_d(sigma)),
                           _ptr(hi), _ptr(lo))
    return hi, lo
