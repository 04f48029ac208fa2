"""Truncated Fock-basis brute force for tiny devices (oracle, test only), fp64.

Methods, Model gives the output state as exp(-sum_{ii'} X_ii' a+_i a+_i')|0> with
X = (1/2) U diag(tanh r) U^T (convention a_out = U a_in) and the single-mode
expansion of exp(-x a+ a+)|0> in the Fock basis.  Here the M-mode state is
expanded the same way: the amplitude of |n_1..n_M> is the coefficient of
z^n in the polynomial exp(-z^T X z), times sqrt(prod n_i!), truncated at D
photons per mode.  The polynomial is built by multiplying in the series of
exp(-X_ii z_i^2) and exp(-2 X_ij z_i z_j) one at a time (direct convolution).

Output loss (outside the paper, which is lossless) acts on photon numbers as
independent binomial thinning with probability eta_i per photon; that is exact
for photon-number statistics because the loss channel commutes with phase
rotations.  From the resulting photon-number distribution every click-pattern
probability and every sector weight follows by summation.
"""
from __future__ import annotations

from math import comb, factorial, lgamma
from typing import Sequence, Tuple

import numpy as np


def _mul_series_axis(F: np.ndarray, axis: int, coef: np.ndarray, step: int) -> np.ndarray:
    """F * sum_k coef[k] z_axis^(step*k), truncated to F's shape."""
    D = F.shape[axis]
    out = np.zeros_like(F)
    for k, ck in enumerate(coef):
        s = step * k
        if s >= D:
            break
        src = [slice(None)] * F.ndim
        dst = [slice(None)] * F.ndim
        src[axis] = slice(0, D - s)
        dst[axis] = slice(s, D)
        out[tuple(dst)] += ck * F[tuple(src)]
    return out


def _mul_series_pair(F: np.ndarray, a: int, b: int, coef: np.ndarray) -> np.ndarray:
    """F * sum_k coef[k] (z_a z_b)^k, truncated."""
    D = F.shape[a]
    out = np.zeros_like(F)
    for k, ck in enumerate(coef):
        if k >= D:
            break
        src = [slice(None)] * F.ndim
        dst = [slice(None)] * F.ndim
        src[a] = slice(0, D - k)
        src[b] = slice(0, D - k)
        dst[a] = slice(k, D)
        dst[b] = slice(k, D)
        out[tuple(dst)] += ck * F[tuple(src)]
    return out


def fock_amplitudes(X: np.ndarray, D: int) -> np.ndarray:
    """Unnormalised amplitudes <n|exp(-a+ X a+)|0>, n_i < D: complex [D]*M."""
    M = X.shape[0]
    F = np.zeros([D] * M, dtype=complex)
    F[(0,) * M] = 1.0
    kk = np.arange(D)
    inv_fact = np.array([1.0 / factorial(int(k)) for k in kk])
    for i in range(M):
        F = _mul_series_axis(F, i, (-X[i, i]) ** kk * inv_fact, 2)
    for i in range(M):
        for j in range(i + 1, M):
            F = _mul_series_pair(F, i, j, (-2.0 * X[i, j]) ** kk * inv_fact)
    sq = np.exp(0.5 * np.array([lgamma(k + 1.0) for k in kk]))
    for i in range(M):
        shape = [1] * M
        shape[i] = D
        F = F * sq.reshape(shape)
    return F


def photon_distribution(U: np.ndarray, r: np.ndarray, eta: np.ndarray, D: int) -> Tuple[np.ndarray, float]:
    """Output photon-number distribution after loss, P[n_1..n_M], and the
    truncation defect 1 - (captured norm) / Z_X."""
    X = 0.5 * (U * np.tanh(r)[None, :]) @ U.T
    amp = fock_amplitudes(X, D)
    P = np.abs(amp) ** 2
    norm_exact = 1.0 / np.sqrt(np.linalg.det(np.eye(len(r)) - 4.0 * np.conj(X) @ X).real)
    defect = 1.0 - P.sum() / norm_exact
    P = P / norm_exact
    M = len(r)
    for i in range(M):
        e = float(eta[i])
        B = np.array([[comb(nn, mm) * e ** mm * (1 - e) ** (nn - mm) if mm <= nn else 0.0
                       for nn in range(D)] for mm in range(D)])
        P = np.moveaxis(np.tensordot(B, P, axes=([1], [i])), 0, i)
    return P, float(defect)


def click_prob(P: np.ndarray, C: Sequence[int]) -> float:
    M = P.ndim
    idx = []
    for i in range(M):
        idx.append(slice(1, None) if i in set(C) else 0)
    return float(P[tuple(idx)].sum())


def sector_weights(P: np.ndarray, C: Sequence[int], T: Sequence[int], L: int) -> np.ndarray:
    """g_T[kappa] = P(N_C = kappa, N_T = 0 | N_Cbar = 0), kappa < L, with T
    given as positions within the sorted clicked set C."""
    M = P.ndim
    C = list(C)
    Tm = {C[a] for a in T}
    idx = []
    for i in range(M):
        if i not in set(C) or i in Tm:
            idx.append(0)
        else:
            idx.append(slice(None))
    sub = P[tuple(idx)]
    pv = float(P[tuple(0 if i not in set(C) else slice(None) for i in range(M))].sum())
    out = np.zeros(L)
    if sub.ndim == 0:
        out[0] = float(sub) / pv
        return out
    grids = np.indices(sub.shape).sum(axis=0)
    for kap in range(min(L, grids.max() + 1)):
        out[kap] = sub[grids == kap].sum() / pv
    return out


def allclick_sectors(P: np.ndarray, C: Sequence[int], L: int) -> np.ndarray:
    """P(N_C = kappa, every mode of C fires | N_Cbar = 0), kappa < L."""
    M = P.ndim
    C = list(C)
    idx = [slice(1, None) if i in set(C) else 0 for i in range(M)]
    sub = P[tuple(idx)]
    pv = float(P[tuple(0 if i not in set(C) else slice(None) for i in range(M))].sum())
    out = np.zeros(L)
    grids = np.indices(sub.shape).sum(axis=0) + len(C)
    for kap in range(min(L, grids.max() + 1)):
        out[kap] = sub[grids == kap].sum() / pv
    return out
