"""Order-j estimate of a click-pattern probability (oracle, test only), fp64.

Results, Approximation scheme and Probability of any specific sample; Methods,
Approximation method.  Three steps, in the paper's order:
  1. partition functions: the weight of the sub-ensemble, P_vac(Cbar) =
     Z_X'/Z_X (eq. 3, second factor), and the sector weights S_0[kappa];
  2. moments of the click count in every sector from clusters of at most j
     modes (S_t[kappa], t <= j; sectors.py);
  3. per sector, the exp-polynomial fit and its value at the last point
     (all n clicked; fit.py); the estimate is the sum over sectors times the
     sub-ensemble weight.

    log p_hat(C) = log P_vac(Cbar) + log sum_{kappa >= n} S_0[kappa] q_kappa(n)

Sectors with fewer photons than clicks contribute nothing.  The sum runs over
every kappa >= n until the remaining tail (bounded by sum S_0, since q <= 1) is
below 1e-15 of the partial sum; the series length doubles until it is.
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np

from .exact import conditional_W
from .fit import maxent_curve, maxent_last_point, moment_targets
from .model import vacuum_prob
from .sectors import cluster_moments, cluster_sector_weights


def prob_approx(Q: np.ndarray, C: Sequence[int], order: int, L0: int = 0,
                return_detail: bool = False, moments=None, floor: float = 1e-10):
    """moments(W, jp, L) -> S[jp+1, L] replaces the fp64 cluster moments (the
    binary128 ones of sectors128.cluster_moments, for rows whose fp64 series
    cancels); floor is then the matching noise level (sectors below
    floor x the absolute series are dropped)."""
    M = Q.shape[0] // 2
    C = list(C)
    n = len(C)
    Cbar = [m for m in range(M) if m not in set(C)]
    log_pv = float(np.log(vacuum_prob(Q, Cbar)))
    if n == 0:
        return (log_pv, {}) if return_detail else log_pv
    W = conditional_W(Q, C)
    jp = min(order, n - 1)
    L = max(L0, 4 * n + 64)
    while True:
        S = cluster_moments(W, jp, L) if moments is None else moments(W, jp, L)
        # rounding floor of each S_0 coefficient: 1e-16 x the |lambda| series;
        # sectors within 1e6 of it (pure states: every odd sector) are noise
        S0abs = cluster_sector_weights(W, [()], L, absolute=True)[0]
        terms = {}
        nfail = 0
        failed = []
        for kap in range(n, L):
            if not S[0, kap] > floor * S0abs[kap]:
                continue
            m = moment_targets(S[:, kap], n, jp)
            lq, ok, _ = maxent_last_point(m, n)
            if not ok:
                nfail += 1
                failed.append(kap)
                continue
            terms[kap] = np.log(S[0, kap]) + lq
        vals = np.array(list(terms.values()))
        vmax = vals.max()
        part = vmax + np.log(np.exp(vals - vmax).sum())
        # tail bound: sum_{kappa >= L} S_0, geometric with the rate of the last
        # two pairs of sectors (pairs, because pure states have no odd sectors)
        a = max(S[0, L - 2], 0.0) + max(S[0, L - 1], 0.0)
        b = max(S[0, L - 4], 0.0) + max(S[0, L - 3], 0.0)
        r = a / b if b > 0 else 1.0
        tail = a * r / (1.0 - r) if r < 1 else np.inf
        if tail <= 1e-15 * np.exp(part) or L >= 8192:
            break
        L *= 2
    out = log_pv + part
    if return_detail:
        fail_weight = float(sum(S[0, k] for k in failed)) / float(np.exp(part))
        return out, dict(S=S, S0abs=S0abs, terms=terms, nfail=nfail, fail_weight=fail_weight, L=L,
                         log_pv=log_pv, jp=jp)
    return out


def sector_estimates(Q: np.ndarray, C: Sequence[int], order: int, L: int) -> Dict[int, float]:
    """log p_hat_kappa for each sector kappa >= n (diagnostics)."""
    _, det = prob_approx(Q, C, order, L0=L, return_detail=True)
    return det["terms"]


def click_distribution(Q: np.ndarray, order: int, ks=(), L0: int = 0):
    """Order-j estimate of the whole device's click distribution (Results,
    Calculation of p(n) and of sectors p_k(n); Approximation scheme): with
    C = every mode (no conditioning, P_vac of the empty set is 1), the cluster
    moments S_t[k] (t <= j) give each photon-number sector k its moments;
    the exp-polynomial fitted to them on the sector's support n' = 1..min(k, M)
    is its curve p_k(n') / S_0[k]; p(n') = sum_k p_k(n'), p(0) = S_0[0].
    Returns (p[0..M], {k: p_k[0..M]} for k in ks, detail)."""
    M = Q.shape[0] // 2
    W = Q
    jp = min(order, M - 1)
    L = max(L0, 4 * M + 64)
    while True:
        S = cluster_moments(W, jp, L)
        S0abs = cluster_sector_weights(W, [()], L, absolute=True)[0]
        a = max(S[0, L - 2], 0.0) + max(S[0, L - 1], 0.0)
        b = max(S[0, L - 4], 0.0) + max(S[0, L - 3], 0.0)
        r = a / b if b > 0 else 1.0
        tail = a * r / (1.0 - r) if r < 1 else np.inf
        if tail <= 1e-15 * S[0].sum() or L >= 8192:
            break
        L *= 2
    p = np.zeros(M + 1)
    p[0] = S[0, 0]
    curves = {k: np.zeros(M + 1) for k in ks}
    if 0 in curves:
        curves[0][0] = S[0, 0]
    nfail = 0
    for k in range(1, L):
        if not S[0, k] > 1e-10 * S0abs[k]:
            continue
        s = min(k, M)
        j = min(jp, s - 1)
        m = moment_targets(S[:, k], M, j)
        lq, ok = maxent_curve(m, M, s)
        if not ok:
            nfail += 1
            continue
        pk = S[0, k] * np.exp(lq)
        p[1:s + 1] += pk
        if k in curves:
            curves[k][1:s + 1] = pk
    return p, curves, dict(L=L, nfail=nfail, S0_sum=float(S[0].sum()))
