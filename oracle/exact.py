"""Exact click probability (oracle, test only), fp64.

Methods, Model: a click of detector j is the projector I - |0_j><0_j|.  Expanding
the product of click projectors over the clicked set C and the vacuum
projectors over the rest gives the plain definition used here,

    p(C) = sum_{T subset of C} (-1)^{|T|} P_vac(Cbar u T),

a signed sum of 2^n vacuum probabilities, which is the "2^n determinants" of
Methods, Probability of any sample.  Three algebraically equal forms are
provided; they differ only in which determinants are taken:

  direct        det(Q_{Cbar u T})^{-1/2} straight from Q
  conditional   P_vac(Cbar) * sum_T (-1)^{|T|} det(W_T)^{-1/2}, with W the
                covariance of the sub-ensemble (eq. 3: the state conditioned on
                the unclicked modes being empty) -- W = Schur complement of Q_Cbar
  torontonian   det(Q)^{-1/2} sum_{Z subset C} (-1)^{n-|Z|} det(A_Z)^{-1/2},
                A = (Q^{-1})_CC

The cancellation factor kappa = sum|terms| / |p| is returned alongside; fp64
results carry a relative error of order kappa * 1e-16.  exact128.c repeats the
conditional form in binary128 for the parity references.
"""
from __future__ import annotations

import itertools
from typing import Sequence, Tuple

import numpy as np

from .model import quad_index, vacuum_prob


def _subsets(items: Sequence[int]):
    for k in range(len(items) + 1):
        for T in itertools.combinations(items, k):
            yield T


def prob_exact_direct(Q: np.ndarray, C: Sequence[int]) -> Tuple[float, float]:
    M = Q.shape[0] // 2
    C = list(C)
    Cbar = [m for m in range(M) if m not in set(C)]
    total, absum = 0.0, 0.0
    for T in _subsets(C):
        term = vacuum_prob(Q, sorted(Cbar + list(T)))
        total += (-1) ** len(T) * term
        absum += term
    return total, (absum / abs(total) if total != 0 else np.inf)


def conditional_W(Q: np.ndarray, C: Sequence[int]) -> np.ndarray:
    """Q-covariance of the clicked modes given that every unclicked mode is
    empty: W = Q_CC - Q_{C,Cbar} Q_Cbar^{-1} Q_{Cbar,C} (order: x of C, p of C)."""
    M = Q.shape[0] // 2
    C = list(C)
    Cbar = [m for m in range(M) if m not in set(C)]
    ic, ib = quad_index(M, C), quad_index(M, Cbar)
    Qcc = Q[np.ix_(ic, ic)]
    if len(Cbar) == 0:
        return Qcc
    Qcb = Q[np.ix_(ic, ib)]
    Qbb = Q[np.ix_(ib, ib)]
    return Qcc - Qcb @ np.linalg.solve(Qbb, Qcb.T)


def prob_exact_conditional(Q: np.ndarray, C: Sequence[int]) -> Tuple[float, float]:
    M = Q.shape[0] // 2
    C = list(C)
    n = len(C)
    Cbar = [m for m in range(M) if m not in set(C)]
    pv = vacuum_prob(Q, Cbar)
    W = conditional_W(Q, C)
    total, absum = 0.0, 0.0
    for T in _subsets(range(n)):
        if len(T) == 0:
            term = 1.0
        else:
            it = np.concatenate([np.array(T), np.array(T) + n])
            term = 1.0 / np.sqrt(np.linalg.det(W[np.ix_(it, it)]))
        total += (-1) ** len(T) * term
        absum += term
    return pv * total, (absum / abs(total) if total != 0 else np.inf)


def prob_exact_torontonian(Q: np.ndarray, C: Sequence[int]) -> Tuple[float, float]:
    M = Q.shape[0] // 2
    C = list(C)
    n = len(C)
    ic = quad_index(M, C)
    A = np.linalg.inv(Q)[np.ix_(ic, ic)]
    total, absum = 0.0, 0.0
    for Z in _subsets(range(n)):
        if len(Z) == 0:
            term = 1.0
        else:
            iz = np.concatenate([np.array(Z), np.array(Z) + n])
            term = 1.0 / np.sqrt(np.linalg.det(A[np.ix_(iz, iz)]))
        total += (-1) ** (n - len(Z)) * term
        absum += term
    det_q = np.linalg.det(Q)
    return total / np.sqrt(det_q), (absum / abs(total) if total != 0 else np.inf)


def all_pattern_probs(Q: np.ndarray) -> dict:
    """p(C) for all 2^M click patterns (direct form), keyed by the tuple C."""
    M = Q.shape[0] // 2
    return {C: prob_exact_direct(Q, C)[0] for C in _subsets(list(range(M)))}
