"""Photon-number sectors of the sub-ensemble and their cluster moments
(oracle, test only).  fp64, plus an mpmath variant for pins.

Methods, Partition function: the sector weight of k photons is the Fourier
coefficient of the generating function Z^nu = <X| e^{i nu N} |X>.  Methods,
Probability of any sample: the sub-ensemble of a click pattern C is the state
with every unclicked mode projected on vacuum (eq. 3).  Methods, Moments
calculation: moments of the click count inside a sector come from the same
generating functions taken on minors, i.e. with further modes forced empty.

Plain definition used here.  Let W be the Q-covariance (covariance + I/2) of the
sub-ensemble, 2n x 2n in xxpp order.  For a cluster T of clicked modes forced
empty and Z = C \\ T, the generating function

    G_T(w) = E[ w^{N_C} 1{N_T = 0} | Cbar empty ]

is the vacuum probability of the modes of T together with a loss channel of
transmission 1 - w on the modes of Z (E[w^N] is the vacuum probability after
such a loss), hence G_T(w) = det(W - D_w (W - I))^{-1/2}, D_w = w on Z, 0 on T.
Taking the Schur complement S = W_ZZ - W_ZT W_TT^{-1} W_TZ with eigenvalues mu,

    G_T(w) = det(W)^{-1/2} * prod_mu (1 - w lambda_mu)^{-1/2},  lambda = 1 - 1/mu,

and log G_T(w) = log det(W)^{-1/2} + sum_{k>=1} w^k P_k / (2k), P_k = sum lambda^k.
The sector weights g_T[kappa] are the power-series coefficients, obtained by
exponentiating that series term by term: no contour and no Fourier grid.

Cluster moments: S_t[kappa] = sum_{|T| = t} g_T[kappa] = E[1{N_C = kappa} C(V, t)]
with V the number of clicked-set modes that stay empty.  S_0 is the sector
weight itself.
"""
from __future__ import annotations

import itertools
from math import comb
from typing import List

import numpy as np


def _exp_series(l: np.ndarray) -> np.ndarray:
    """Coefficients of exp(sum_{k>=1} l_k w^k) for each row of l [B, L]
    (l[:, 0] ignored): f_0 = 1, k f_k = sum_{i=1..k} i l_i f_{k-i}."""
    B, L = l.shape
    f = np.zeros((B, L))
    f[:, 0] = 1.0
    il = l * np.arange(L)[None, :]
    for k in range(1, L):
        f[:, k] = np.einsum("bi,bi->b", il[:, 1:k + 1], f[:, k - 1::-1][:, :k]) / k
    return f


def _cluster_lambdas(W: np.ndarray, clusters: List[tuple]) -> np.ndarray:
    """lambda = 1 - 1/mu for the Schur complement of each cluster (all clusters of
    one size t): [len(clusters), 2(n-t)]."""
    n = W.shape[0] // 2
    t = len(clusters[0])
    zs = n - t
    if zs == 0:
        return np.zeros((len(clusters), 0))
    T = np.array(clusters, dtype=np.int64).reshape(len(clusters), t)
    Z = np.array([[a for a in range(n) if a not in set(c)] for c in clusters], dtype=np.int64)
    it = np.concatenate([T, T + n], axis=1)
    iz = np.concatenate([Z, Z + n], axis=1)
    Wzz = W[iz[:, :, None], iz[:, None, :]]
    if t > 0:
        Wzt = W[iz[:, :, None], it[:, None, :]]
        Wtt = W[it[:, :, None], it[:, None, :]]
        S = Wzz - Wzt @ np.linalg.solve(Wtt, np.swapaxes(Wzt, 1, 2))
    else:
        S = Wzz
    mu = np.linalg.eigvalsh(S)
    return 1.0 - 1.0 / mu


def cluster_sector_weights(W: np.ndarray, clusters: List[tuple], L: int,
                           absolute: bool = False) -> np.ndarray:
    """g_T[kappa], kappa = 0..L-1, for each cluster T (tuple of positions 0..n-1
    within the clicked set).  Returns [len(clusters), L].  With absolute=True the
    series is taken with |lambda| in place of lambda: a bound on the sum of
    |terms| behind each coefficient, i.e. on its rounding error / 1e-16."""
    sign, logdet_w = np.linalg.slogdet(W)
    pref = np.exp(-0.5 * logdet_w)
    by_size = {}
    for i, T in enumerate(clusters):
        by_size.setdefault(len(T), []).append(i)
    out = np.zeros((len(clusters), L))
    for t, ids in by_size.items():
        lam = _cluster_lambdas(W, [clusters[i] for i in ids])
        if absolute:
            lam = np.abs(lam)
        # l_k = P_k / (2k), P_k = sum lambda^k
        l = np.zeros((len(ids), L))
        if lam.shape[1] > 0:
            pw = lam.copy()
            for kk in range(1, L):
                l[:, kk] = pw.sum(axis=1) / (2.0 * kk)
                pw *= lam
        out[ids] = pref * _exp_series(l)
    return out


def clusters_of_size(n: int, t: int):
    return list(itertools.combinations(range(n), t))


def cluster_moments(W: np.ndarray, jmax: int, L: int) -> np.ndarray:
    """S_t[kappa] for t = 0..jmax, kappa = 0..L-1: [jmax+1, L]."""
    n = W.shape[0] // 2
    S = np.zeros((jmax + 1, L))
    for t in range(jmax + 1):
        cl = clusters_of_size(n, t)
        # chunk to bound memory
        for s in range(0, len(cl), 2048):
            S[t] += cluster_sector_weights(W, cl[s:s + 2048], L).sum(axis=0)
    return S


def sector_allclick_exact(W: np.ndarray, L: int) -> np.ndarray:
    """Exact all-click weight of each sector of the sub-ensemble,
    sum_T (-1)^{|T|} g_T[kappa] over all 2^n clusters (tiny n only)."""
    n = W.shape[0] // 2
    tot = np.zeros(L)
    for t in range(n + 1):
        g = cluster_sector_weights(W, clusters_of_size(n, t), L).sum(axis=0)
        tot += (-1) ** t * g
    return tot


# ---------------------------------------------------------------- mpmath variant
def cluster_sector_weights_mp(W, T, L: int, dps: int = 40):
    """Same as cluster_sector_weights for one cluster, in mpmath at `dps` digits
    (W given as an fp64 array; taken as exact)."""
    import mpmath as mp
    with mp.workdps(dps):
        n = W.shape[0] // 2
        Wm = mp.matrix(W.tolist())
        T = list(T)
        Z = [a for a in range(n) if a not in set(T)]
        it = T + [a + n for a in T]
        iz = Z + [a + n for a in Z]

        def sub(rows, cols):
            return mp.matrix([[Wm[i, j] for j in cols] for i in rows])

        if len(iz) == 0:
            lam = []
        else:
            S = sub(iz, iz)
            if T:
                Wzt = sub(iz, it)
                S = S - Wzt * mp.inverse(sub(it, it)) * Wzt.T
            mu, _ = mp.eigsy(S)
            lam = [1 - 1 / m for m in mu]
        pref = 1 / mp.sqrt(mp.det(Wm))
        l = [mp.mpf(0)] + [sum(x ** k for x in lam) / (2 * k) for k in range(1, L)]
        f = [mp.mpf(1)] + [mp.mpf(0)] * (L - 1)
        for k in range(1, L):
            f[k] = sum(i * l[i] * f[k - i] for i in range(1, k + 1)) / k
        return [pref * x for x in f]


def binom_table(n: int, jmax: int) -> np.ndarray:
    return np.array([[comb(a, t) for t in range(jmax + 1)] for a in range(n + 1)], dtype=float)
