"""Model: the Gaussian output state of a lossy boson sampler (oracle, test only).

Methods, Model: inputs are single-mode squeezed vacua with parameters r_j, mixed
by an interferometer U and read by threshold detectors.  The paper writes the
pure output state as exp(-sum X_ii' a+_i a+_i')|0> with X = (1/2) sum_j U U
tanh(r_j); loss is outside the paper (it treats the lossless device), so the
state is carried here as its covariance matrix, which reduces to the paper's X
at eta = 1 (checked by the tests).

Conventions: hbar = 1, vacuum covariance I/2, quadratures ordered xxpp (mode i
has rows i and M+i), a = (x + ip)/sqrt(2), a_out = U a_in, squeezing along x.
"""
from __future__ import annotations

import numpy as np


def symplectic_O(U: np.ndarray) -> np.ndarray:
    """Real orthogonal-symplectic form of the interferometer in xxpp order:
    x_out + i p_out = U (x_in + i p_in)."""
    return np.block([[U.real, -U.imag], [U.imag, U.real]])


def covariance(U: np.ndarray, r: np.ndarray, eta: np.ndarray) -> np.ndarray:
    """sigma = D sigma0 D + (I - D^2)/2 with sigma0 = O diag(e^{-2r}, e^{2r}) O^T / 2
    and D = diag(sqrt(eta), sqrt(eta)): squeezed inputs, interferometer, then a
    pure-loss channel of transmission eta_i on each output mode."""
    M = U.shape[0]
    O = symplectic_O(U)
    d = np.concatenate([np.exp(-2.0 * r), np.exp(2.0 * r)])
    sigma0 = (O * d[None, :]) @ O.T / 2.0
    s = np.sqrt(np.concatenate([eta, eta]))
    return s[:, None] * sigma0 * s[None, :] + np.diag(1.0 - s * s) / 2.0


def q_matrix(sigma: np.ndarray) -> np.ndarray:
    """Q = sigma + I/2, the covariance of the state's Husimi function."""
    return sigma + np.eye(sigma.shape[0]) / 2.0


def quad_index(M: int, modes) -> np.ndarray:
    """Rows of the given modes in xxpp order: x rows first, then p rows."""
    modes = np.asarray(modes, dtype=np.int64)
    return np.concatenate([modes, modes + M])


def vacuum_prob(Q: np.ndarray, modes) -> float:
    """Probability that every mode in `modes` holds no photon:
    det(Q_S)^{-1/2} with Q_S the 2|S| x 2|S| block of Q (1 for the empty set)."""
    M = Q.shape[0] // 2
    if len(modes) == 0:
        return 1.0
    idx = quad_index(M, modes)
    return 1.0 / np.sqrt(np.linalg.det(Q[np.ix_(idx, idx)]))


def takagi_X(U: np.ndarray, r: np.ndarray) -> np.ndarray:
    """The paper's X (Methods, Model) in this module's convention a_out = U a_in:
    X = (1/2) U diag(tanh r) U^T.  (The paper indexes U_{ji}U_{ji'}, i.e. its U
    is the transpose of this one.)"""
    return 0.5 * (U * np.tanh(r)[None, :]) @ U.T


def partition_function(X: np.ndarray) -> float:
    """Z_X = <X|X> of the unnormalised state exp(-a+ X a+)|0> (Methods, Partition
    function).  The normalisation of the single-mode series in Methods, Model,
    sum_l |x|^{2l}(2l)!/(l!)^2 = (1-4|x|^2)^{-1/2}, fixes the factor 4 that the
    printed matrix formula leaves out: Z_X = det(I - 4 conj(X) X)^{-1/2}."""
    n = X.shape[0]
    if n == 0:
        return 1.0
    val = np.linalg.det(np.eye(n) - 4.0 * np.conj(X) @ X)
    return 1.0 / np.sqrt(val.real)
