"""Finite-difference gradients of the oracle's log-probabilities (oracle, test only).

The paper does not differentiate; a gradient of sum_p w_p log p_hat_p with
respect to the squeezing parameters r_j and the transmissions eta_i is what a
fit of a device model to observed clicks needs.  The reference here is the
central difference (f(x+h) - f(x-h)) / 2h in fp64, taken on the oracle itself,
with the oracle's own choices (order, series length) held fixed.
"""
from __future__ import annotations

from typing import Callable, Sequence

import numpy as np


def central_fd(f: Callable[[np.ndarray], float], x: np.ndarray, idx: Sequence[int],
               h: float = 1e-6) -> np.ndarray:
    g = np.zeros(len(idx))
    for k, i in enumerate(idx):
        xp = x.copy(); xp[i] += h
        xm = x.copy(); xm[i] -= h
        g[k] = (f(xp) - f(xm)) / (2.0 * h)
    return g


def directional_fd(f: Callable[[np.ndarray], float], x: np.ndarray, v: np.ndarray,
                   h: float = 1e-6) -> float:
    return (f(x + h * v) - f(x - h * v)) / (2.0 * h)
