"""Metropolis-Hastings over click patterns with a fixed number of clicks
(oracle, test only).

Discussion: the approximate probabilities as the target of a Markov chain
Monte Carlo sampler.  The chain moves by swapping one clicked mode for one
unclicked mode; every one of the n (M - n) swaps is equally likely and the
reverse swap is equally likely from the new pattern, so the Metropolis rule
(Metropolis et al. 1953; Hastings 1970) accepts with min(1, p(new) / p(old)),
and the chain's stationary distribution is p restricted to patterns of n
clicks, normalised.

The swap is drawn from two uniforms: position i = floor(u0 n) of the ascending
row, and the k-th (from 0) unclicked mode in increasing order,
k = floor(u1 (M - n)); acceptance when log p(new) >= log p(old) or
u2 < exp(log p(new) - log p(old)).  A proposal whose log p is NaN is rejected.
"""
from __future__ import annotations

import math
from typing import Callable, List, Sequence, Tuple


def propose(row: Sequence[int], M: int, u0: float, u1: float) -> List[int]:
    n = len(row)
    if n == 0 or n == M:
        return list(row)
    i = min(n - 1, int(u0 * n))
    k = min(M - n - 1, int(u1 * (M - n)))
    free = [m for m in range(M) if m not in set(row)]
    new = [m for r, m in enumerate(row) if r != i] + [free[k]]
    return sorted(new)


def mh_step(rows: Sequence[Sequence[int]], M: int, u: Sequence[float], logp: Sequence[float],
            logp_fn: Callable[[List[int]], float]) -> Tuple[List[List[int]], List[float], List[int], List[List[int]]]:
    """One step for every chain: (new rows, new log p, accepted flags, proposals)."""
    out_rows, out_lp, acc, props = [], [], [], []
    for p, row in enumerate(rows):
        prop = propose(row, M, u[3 * p], u[3 * p + 1])
        lq = logp_fn(prop)
        ok = not math.isnan(lq)
        d = lq - logp[p]
        a = ok and (math.isnan(logp[p]) or d >= 0.0 or u[3 * p + 2] < math.exp(d))
        props.append(prop)
        acc.append(1 if a else 0)
        out_rows.append(prop if a else list(row))
        out_lp.append(lq if a else logp[p])
    return out_rows, out_lp, acc, props
