"""Per-sector exp-polynomial fit (oracle, test only), fp64.

Results, Approximation scheme and Methods, Approximation method: inside a
photon-number sector the click-count distribution is modelled as the
exponential of a degree-j polynomial, and its parameters are found iteratively
so that the model's low moments equal the true ones; the estimate is the
model's value at the last point (every clicked detector fires).

Reading used here.  The support is n' = 1..n clicks (a sector with photons has
at least one click; n' = 0 is impossible, so leaving it in would make the fit
infeasible).  The j' = min(j, n-1) constraints are written in the basis
phi_t(n') = C(n-n', t) / C(n-1, t), t = 1..j', which spans the same polynomials
of degree <= j' as the paper's powers n'^t, so the fitted family is the same;
it is matched to m_t = S_t / (S_0 C(n-1, t)) (cluster moments, sectors.py).
Among distributions exp(-c . phi(n')) / Z(c) the moment-matching one is the
unique minimiser of the convex dual L(c) = log Z(c) + c . m, found by Newton's
method from c = 0 with Armijo backtracking.  Since phi(n) = 0, the estimate at
the last point is q(n) = 1 / Z(c).
"""
from __future__ import annotations

from math import comb
from typing import Tuple

import numpy as np

FIT_MAXIT = 200


def basis(n: int, jp: int) -> np.ndarray:
    """phi_t(n') for t = 1..jp and n' = 1..n: [jp, n]."""
    npr = np.arange(1, n + 1)
    return np.array([[comb(n - a, t) / comb(n - 1, t) for a in npr] for t in range(1, jp + 1)],
                    dtype=float).reshape(jp, n)


def _lse(z: np.ndarray) -> float:
    zm = z.max()
    return float(zm + np.log(np.exp(z - zm).sum()))


def maxent_last_point(m: np.ndarray, n: int, maxit: int = FIT_MAXIT) -> Tuple[float, bool, int]:
    """Fit and return (log q(n), converged, iterations) for targets m [jp]."""
    lq, ok, it, _ = maxent_fit(m, n, maxit)
    return lq, ok, it


def maxent_fit(m: np.ndarray, n: int, maxit: int = FIT_MAXIT):
    """The fit of maxent_last_point, also returning the fitted parameters c:
    (log q(n), converged, iterations, c)."""
    jp = len(m)
    if jp == 0:          # n = 1: a single support point, q(1) = 1
        return 0.0, True, 0, np.zeros(0)
    phi = basis(n, jp)
    c = np.zeros(jp)

    def dual(cc):
        return _lse(-cc @ phi) + cc @ m

    for it in range(maxit + 1):
        z = -c @ phi
        lse = _lse(z)
        prob = np.exp(z - lse)
        E = phi @ prob
        g = m - E
        if np.all(np.abs(g) <= 1e-15 + 1e-12 * np.abs(m)):
            # one polishing Newton step, then report
            H = (phi * prob) @ phi.T - np.outer(E, E)
            try:
                c = c + np.linalg.solve(H + 1e-14 * np.trace(H) * np.eye(jp), -g)
            except np.linalg.LinAlgError:
                pass
            return -_lse(-c @ phi), True, it, c
        if it == maxit:
            break
        H = (phi * prob) @ phi.T - np.outer(E, E)
        H = H + 1e-14 * np.trace(H) * np.eye(jp)
        try:
            step = np.linalg.solve(H, -g)
        except np.linalg.LinAlgError:
            step = np.linalg.lstsq(H, -g, rcond=None)[0]
        L0 = lse + c @ m
        slope = g @ step
        t = 1.0
        # Backtrack only while the predicted decrease is resolvable in fp64;
        # below that the full Newton step is taken (quadratic-convergence region).
        if -slope > 1e-13 * max(1.0, abs(L0)):
            while t > 1e-12:
                if dual(c + t * step) <= L0 + 1e-4 * t * slope:
                    break
                t *= 0.5
        c = c + t * step
    return float("nan"), False, maxit, c


def maxent_curve(m: np.ndarray, n: int, s: int, maxit: int = FIT_MAXIT) -> Tuple[np.ndarray, bool]:
    """The same fit on the support n' = 1..s (s <= n; a sector of k photons
    clicks at most k detectors, so s = min(k, n)), with the basis phi_t of the
    full n (the moments m_t are the same S_t / (S_0 C(n-1, t))); returns
    (log q(n') for n' = 1..s, converged).  jp = len(m) <= s - 1."""
    jp = len(m)
    if s == 1 or jp == 0:
        out = np.full(s, -np.inf)
        out[0 if s == 1 else s - 1] = 0.0
        if s > 1:              # no moment: the uniform curve on the support
            out[:] = -np.log(s)
        return out, True
    phi = basis(n, jp)[:, :s]
    c = np.zeros(jp)

    def dual(cc):
        return _lse(-cc @ phi) + cc @ m

    for it in range(maxit + 1):
        z = -c @ phi
        lse = _lse(z)
        prob = np.exp(z - lse)
        E = phi @ prob
        g = m - E
        H = (phi * prob) @ phi.T - np.outer(E, E)
        H = H + 1e-14 * np.trace(H) * np.eye(jp)
        if np.all(np.abs(g) <= 1e-15 + 1e-12 * np.abs(m)):
            try:
                c = c + np.linalg.solve(H, -g)
            except np.linalg.LinAlgError:
                pass
            z = -c @ phi
            return z - _lse(z), True
        if it == maxit:
            break
        try:
            step = np.linalg.solve(H, -g)
        except np.linalg.LinAlgError:
            step = np.linalg.lstsq(H, -g, rcond=None)[0]
        L0 = lse + c @ m
        slope = g @ step
        t = 1.0
        if -slope > 1e-13 * max(1.0, abs(L0)):
            while t > 1e-12:
                if dual(c + t * step) <= L0 + 1e-4 * t * slope:
                    break
                t *= 0.5
        c = c + t * step
    return np.full(s, np.nan), False


def moment_targets(S_col: np.ndarray, n: int, jp: int) -> np.ndarray:
    """m_t = S_t / (S_0 C(n-1, t)), t = 1..jp, for one sector column S_col [>= jp+1]."""
    return np.array([S_col[t] / (S_col[0] * comb(n - 1, t)) for t in range(1, jp + 1)])
