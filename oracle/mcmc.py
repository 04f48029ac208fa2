"""Metropolis-Hastings over click patterns with a fixed number of clicks
(oracle, test only): the plain step with a given target, and the two-stage
(delayed-acceptance) step with an estimate as the screen and the exact p as
the target.

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


def da_step(rows: Sequence[Sequence[int]], M: int, u: Sequence[float], logp_hat: Sequence[float],
            logp_exact: Sequence[float], hat_fn: Callable[[List[int]], float],
            exact_fn: Callable[[List[int]], float]):
    """One two-stage (delayed-acceptance) step for every chain (Christen & Fox
    2005): the approximation screens each symmetric swap proposal, the exact
    probability corrects the survivors, so the chain's stationary distribution
    is the exact p restricted to n clicks, normalised (Discussion: the
    approximation as the proposal distribution of a Markov chain Monte Carlo
    sampler).  Four uniforms per chain: u0, u1 the swap (as in `propose`), u2
    the first stage (accept when log p_hat(new) >= log p_hat(old) or
    u2 < exp(difference)), u3 the second (accept when
    r = [log p(new) - log p(old)] - [log p_hat(new) - log p_hat(old)] >= 0 or
    u3 < exp(r)).  A chain whose current values are not both finite takes any
    proposal whose two values are.  Returns (rows, log p_hat, log p, codes,
    proposals); code 1 = moved, 0 = rejected by the approximation, 2 =
    rejected by the exact correction."""
    out_rows, out_h, out_e, codes, props = [], [], [], [], []
    for p, row in enumerate(rows):
        prop = propose(row, M, u[4 * p], u[4 * p + 1])
        props.append(prop)
        h0, e0 = logp_hat[p], logp_exact[p]
        h1 = hat_fn(prop)
        bad_cur = not (math.isfinite(h0) and math.isfinite(e0))
        code = 0
        if not math.isnan(h1):
            dh = h1 - h0
            if bad_cur or dh >= 0.0 or u[4 * p + 2] < math.exp(dh):
                e1 = exact_fn(prop)
                code = 2
                if not math.isnan(e1):
                    if bad_cur:
                        code = 1 if math.isfinite(h1) and math.isfinite(e1) else 2
                    else:
                        r = (e1 - e0) - dh
                        code = 1 if (r >= 0.0 or u[4 * p + 3] < math.exp(r)) else 2
        if code == 1:
            out_rows.append(prop); out_h.append(h1); out_e.append(e1)
        else:
            out_rows.append(list(row)); out_h.append(h0); out_e.append(e0)
        codes.append(code)
    return out_rows, out_h, out_e, codes, props
