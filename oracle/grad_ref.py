"""Reference gradient of L = sum_p w_p log p_hat_p with respect to the
squeezing parameters r and the transmissions eta (oracle, test only).

torch-CPU fp64 automatic differentiation through the oracle's own steps, in the
paper's order (Methods, Model; Partition function; Moments calculation;
Approximation method), sharing nothing with the hand-written GPU adjoint:

  sigma(r, eta) and Q = sigma + I/2                      (model.covariance)
  log P_vac(Cbar) = -(1/2) sum log eigvalsh(Q_Cbar)
  W = Q_CC - Q_{C,Cbar} Q_Cbar^{-1} Q_{Cbar,C}           (exact.conditional_W)
  g_T[kappa] = det(W)^{-1/2} [w^kappa] prod_mu (1 - w lambda_mu)^{-1/2},
      lambda = 1 - 1/mu, mu = eigvalsh of the Schur complement of T's rows
  S_t[kappa] = sum_{|T| = t} g_T[kappa]                  (sectors.cluster_moments)
  per sector: the max-entropy fit to m_t = S_t / (S_0 C(n-1, t)) (fit.py)
  log p_hat = log P_vac(Cbar) + log sum_kappa S_0[kappa] q_kappa(n)

The discrete choices (series length, which sectors are fitted, how many
moments) are the numpy oracle's at the given point (approx.prob_approx), held
fixed, as a frozen plan holds them on the GPU.  The fit enters through one
Newton step taken from the converged parameters c* (numpy) with the moments m
as differentiable inputs: c1 = c* + H^{-1} (E_{c*}[phi] - m), whose value is c*
and whose derivative is dc*/dm = -H^{-1} (H the covariance of the basis).

Memory stays bounded by differentiating in stages: the fits and the log-sum
against the sector sums S as leaves; then the cluster series, in chunks of
clusters, against those cotangents (each chunk's graph freed after its
backward pass); then W and log P_vac(Cbar) against Q; then Q against r, eta.
"""
from __future__ import annotations

import itertools
from math import comb
from typing import Sequence

import numpy as np
import torch

from . import approx, fit, model

F64 = torch.float64


def covariance_t(U: np.ndarray, r: torch.Tensor, eta: torch.Tensor) -> torch.Tensor:
    """sigma = D sigma0 D + (I - D^2)/2, sigma0 = O diag(e^{-2r}, e^{2r}) O^T / 2."""
    O = torch.tensor(model.symplectic_O(U), dtype=F64)
    d = torch.cat([torch.exp(-2.0 * r), torch.exp(2.0 * r)])
    sigma0 = (O * d[None, :]) @ O.T / 2.0
    s = torch.sqrt(torch.cat([eta, eta]))
    return s[:, None] * sigma0 * s[None, :] + torch.diag(1.0 - s * s) / 2.0


def _cluster_series(W: torch.Tensor, clusters, L: int) -> torch.Tensor:
    """sum over the given clusters (all of one size t) of g_T[kappa], kappa < L."""
    n = W.shape[0] // 2
    t = len(clusters[0])
    logdet_w = torch.log(torch.linalg.eigvalsh(W)).sum()
    T = torch.tensor(clusters, dtype=torch.long).reshape(len(clusters), t)
    Z = torch.tensor([[a for a in range(n) if a not in set(c)] for c in clusters], dtype=torch.long)
    it = torch.cat([T, T + n], dim=1)
    iz = torch.cat([Z, Z + n], dim=1)
    Wzz = W[iz[:, :, None], iz[:, None, :]]
    if t > 0:
        Wzt = W[iz[:, :, None], it[:, None, :]]
        Wtt = W[it[:, :, None], it[:, None, :]]
        S = Wzz - Wzt @ torch.linalg.solve(Wtt, Wzt.transpose(1, 2))
    else:
        S = Wzz
    S = 0.5 * (S + S.transpose(1, 2))
    lam = 1.0 - 1.0 / torch.linalg.eigvalsh(S)               # [B, 2(n-t)]
    # l_k = sum lambda^k / (2k), k = 1..L-1
    k = torch.arange(1, L, dtype=F64)
    pk = (lam[:, :, None] ** k[None, None, :]).sum(1)      # [B, L-1]
    il = pk / 2.0                                           # k l_k
    f = [torch.ones(len(clusters), dtype=F64)]
    for kk in range(1, L):
        prev = torch.stack(f[::-1], dim=1)                  # f_{kk-1}, ..., f_0
        f.append((il[:, :kk] * prev).sum(1) / kk)
    g = torch.stack(f, dim=1) * torch.exp(-0.5 * logdet_w)
    return g.sum(0)


def _row_value(S: torch.Tensor, n: int, jp: int, kept, log_pv: torch.Tensor):
    """log P_vac(Cbar) + log sum over the kept sectors of S_0 q(n), with the
    fits entering through one Newton step from the numpy fit."""
    terms = []
    for kap in kept:
        S0 = S[0, kap]
        m = torch.stack([S[t, kap] / (S0 * comb(n - 1, t)) for t in range(1, jp + 1)]) if jp else None
        if jp == 0:
            terms.append(torch.log(S0))
            continue
        mnp = m.detach().numpy()
        lq, ok, _, c = fit.maxent_fit(mnp, n)
        assert ok
        phi = fit.basis(n, jp)
        z = -c @ phi
        prob = np.exp(z - z.max())
        prob /= prob.sum()
        E = phi @ prob
        H = (phi * prob) @ phi.T - np.outer(E, E)
        Hinv = torch.tensor(np.linalg.inv(H), dtype=F64)
        c1 = torch.tensor(c, dtype=F64) + Hinv @ (torch.tensor(E, dtype=F64) - m)
        zz = -(c1[:, None] * torch.tensor(phi, dtype=F64)).sum(0)
        terms.append(torch.log(S0) - torch.logsumexp(zz, 0))
    return log_pv + torch.logsumexp(torch.stack(terms), 0)


def loss_and_grad(U: np.ndarray, r: np.ndarray, eta: np.ndarray, rows: Sequence[Sequence[int]], order: int,
                  w: Sequence[float], chunk: int = 256):
    """(L, dL/dr, dL/deta) with L = sum_p w_p log p_hat_p (order-j estimate)."""
    M = U.shape[0]
    r_t = torch.tensor(r, dtype=F64, requires_grad=True)
    e_t = torch.tensor(eta, dtype=F64, requires_grad=True)
    Q = covariance_t(U, r_t, e_t) + torch.eye(2 * M, dtype=F64) / 2.0
    Qd = Q.detach().clone().requires_grad_(True)
    Qnp = Qd.detach().numpy()
    total = 0.0
    for C, wp in zip(rows, w):
        C = list(C)
        n = len(C)
        Cbar = [m for m in range(M) if m not in set(C)]
        ic = torch.tensor(model.quad_index(M, C), dtype=torch.long)
        ib = torch.tensor(model.quad_index(M, Cbar), dtype=torch.long)
        if len(Cbar):
            Qbb = Qd[ib][:, ib]
            log_pv = -0.5 * torch.log(torch.linalg.eigvalsh(Qbb)).sum()
        else:
            log_pv = torch.zeros((), dtype=F64)
        if n == 0:
            (wp * log_pv).backward()
            total += wp * log_pv.item()
            continue
        Qcc = Qd[ic][:, ic]
        if len(Cbar):
            Qcb = Qd[ic][:, ib]
            W = Qcc - Qcb @ torch.linalg.solve(Qbb, Qcb.T)
        else:
            W = Qcc
        W = 0.5 * (W + W.T)
        lp, det = approx.prob_approx(Qnp, C, order, return_detail=True)
        jp, kept = det["jp"], sorted(det["terms"])
        L = max(kept) + 1
        # stage 1: the fits and the log-sum against S as a leaf
        S_leaf = torch.tensor(det["S"][:jp + 1, :L], dtype=F64, requires_grad=True)
        val = _row_value(S_leaf, n, jp, kept, log_pv.detach())
        (gS,) = torch.autograd.grad(val, S_leaf)
        total += wp * val.item()
        # stage 2: the cluster series against gS, chunk by chunk, into W
        Wl = W.detach().clone().requires_grad_(True)
        for t in range(jp + 1):
            cl = list(itertools.combinations(range(n), t))
            for s0 in range(0, len(cl), chunk):
                st = _cluster_series(Wl, cl[s0:s0 + chunk], L)
                (wp * (gS[t] * st).sum()).backward()
        # stage 3: W and log P_vac(Cbar) into Q
        (wp * log_pv + (W * Wl.grad).sum()).backward()
    # stage 4: Q into r and eta
    Q.backward(Qd.grad)
    return total, r_t.grad.numpy().copy(), e_t.grad.numpy().copy()
