"""Seeded synthetic inputs for the click-probability workloads.

This module only draws random numbers and arranges them; it holds none of the
method's arithmetic (no covariance, no determinants, no sectors).  Both the CPU
oracle (tests only) and the GPU path take their inputs from here.

Shapes follow the paper's setups: a Haar-random interferometer U (the paper
draws a "random unitary", Results, Fig. 2 caption), a block of squeezed inputs
with the rest in vacuum (about half of the inputs filled, Results, Numerical
accuracy), output transmissions eta, and random measurement outcomes given as
the sorted list of clicked detectors (Methods, Probability of any sample).
The two large configurations take the sizes of the 100- and 144-mode
experiments the paper cites (Introduction); their data are not available, so a
Haar U stands in.

Conventions: a_out = U a_in; mode ids are 0-based; a click pattern is the sorted
list of clicked output modes.  Every stream is numpy's PCG64 seeded with
[210601445, config, stream] where stream 0 = U, 1 = r, 2 = eta, 3 = patterns.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_ROOT = 210601445
S_U, S_R, S_ETA, S_PAT = 0, 1, 2, 3


def rng_for(config: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, int(config), int(stream)])


def haar_unitary(M: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed M x M unitary: QR of a complex Ginibre matrix with the
    phases of R's diagonal moved into Q (Mezzadri, Notices AMS 54, 2007)."""
    z = (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def random_patterns(M: int, P: int, n_lo: int, n_hi: int,
                    rng: np.random.Generator) -> Tuple[np.ndarray, np.ndarray]:
    """P click patterns in CSR form: n ~ U{n_lo..n_hi}, then a uniform n-subset
    of the M modes, sorted ascending.  Returns (offsets[P+1], modes) as int32."""
    ns = rng.integers(n_lo, n_hi + 1, size=P)
    offsets = np.zeros(P + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(ns)
    modes = np.empty(int(offsets[-1]), dtype=np.int32)
    for p in range(P):
        sel = rng.choice(M, size=int(ns[p]), replace=False)
        modes[offsets[p]:offsets[p + 1]] = np.sort(sel)
    return offsets, modes


def csr_from_lists(patterns: Sequence[Sequence[int]]) -> Tuple[np.ndarray, np.ndarray]:
    offsets = np.zeros(len(patterns) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum([len(c) for c in patterns])
    modes = np.array([m for c in patterns for m in c], dtype=np.int32)
    return offsets, modes


def csr_rows(offsets: np.ndarray, modes: np.ndarray) -> List[np.ndarray]:
    return [modes[offsets[p]:offsets[p + 1]] for p in range(len(offsets) - 1)]


@dataclasses.dataclass
class Workload:
    name: str
    config: int
    M: int
    U: np.ndarray          # complex128 [M, M]
    r: np.ndarray          # float64 [M]; 0 = vacuum input
    eta: np.ndarray        # float64 [M]; output transmissions
    offsets: np.ndarray    # int32 [P+1]
    modes: np.ndarray      # int32 [offsets[-1]]
    order: int             # approximation order j of the paper's scheme
    exact: bool            # whether the exact (2^n) path is part of the workload
    description: str

    @property
    def P(self) -> int:
        return len(self.offsets) - 1

    def subset(self, idx: Sequence[int]) -> "Workload":
        rows = csr_rows(self.offsets, self.modes)
        off, mod = csr_from_lists([rows[i] for i in idx])
        return dataclasses.replace(self, offsets=off, modes=mod)


# name, M, n_squeezed, r range (lo, hi) or scalar, eta (scalar or per-mode range),
# P, click range, order, exact
_SPECS = {
    1: dict(name="m8_exact_order2", M=8, nsq=8, r=(1.0, 1.0), eta=1.0, eta_range=None,
            P=16, n=(2, 6), order=2, exact=True,
            desc="8 modes, r=1.0 on all 8 inputs, eta=1, 16 patterns with 2-6 clicks; "
                 "exact and order-2"),
    2: dict(name="m20_exact", M=20, nsq=10, r=(0.5, 1.5), eta=0.5, eta_range=None,
            P=4096, n=(6, 14), order=3, exact=True,
            desc="20 modes, 10 inputs r~U[0.5,1.5], eta=0.5, 4096 patterns with 6-14 "
                 "clicks; exact and order-2/3"),
    3: dict(name="m70_order3", M=70, nsq=35, r=(1.0, 1.6), eta=0.4, eta_range=None,
            P=10000, n=(15, 40), order=3, exact=False,
            desc="70 modes, 35 inputs r~U[1.0,1.6], eta=0.4, 10^4 patterns with 15-40 "
                 "clicks; order-3"),
    4: dict(name="m100_order3", M=100, nsq=50, r=(1.1, 1.6), eta=0.3, eta_range=None,
            P=10000, n=(25, 60), order=3, exact=False,
            desc="100 modes, 50 inputs r~U[1.1,1.6], eta=0.3, 10^4 patterns with 25-60 "
                 "clicks; order-3"),
    5: dict(name="m144_order2_grad", M=144, nsq=50, r=(1.1, 1.6), eta=None,
            eta_range=(0.2, 0.5), P=4096, n=(40, 110), order=2, exact=False,
            desc="144 modes, 50 inputs r~U[1.1,1.6], per-mode eta~U[0.2,0.5], 4096 "
                 "patterns with 40-110 clicks; order-2 forward and gradient"),
}


def make_workload(config: int, P: Optional[int] = None) -> Workload:
    """Build configuration `config` (1..5).  `P` truncates the pattern list to
    its first P rows (the same seeded stream, so a prefix of the full batch)."""
    s = _SPECS[config]
    M = s["M"]
    U = haar_unitary(M, rng_for(config, S_U))
    lo, hi = s["r"]
    r = np.zeros(M)
    if lo == hi:
        r[: s["nsq"]] = lo
    else:
        r[: s["nsq"]] = rng_for(config, S_R).uniform(lo, hi, size=s["nsq"])
    if s["eta_range"] is None:
        eta = np.full(M, float(s["eta"]))
    else:
        eta = rng_for(config, S_ETA).uniform(*s["eta_range"], size=M)
    offsets, modes = random_patterns(M, s["P"], s["n"][0], s["n"][1], rng_for(config, S_PAT))
    wl = Workload(name=s["name"], config=config, M=M, U=U, r=r, eta=eta,
                  offsets=offsets, modes=modes, order=s["order"], exact=s["exact"],
                  description=s["desc"])
    if P is not None and P < wl.P:
        wl = wl.subset(range(P))
    return wl


def accuracy_workload(M: int, r: float, n: int, P: int = 100) -> Workload:
    """Accuracy-study setup of the paper's Numerical accuracy paragraph (Fig. 4):
    a lossless M-mode Haar interferometer with every second input squeezed at
    r, and P random outcomes with n clicked detectors (stream [SEED_ROOT, 97,
    M, round(100 r), n, s])."""
    tag = [97, M, int(round(100 * r)), n]
    U = haar_unitary(M, np.random.default_rng([SEED_ROOT, *tag, S_U]))
    rr = np.zeros(M)
    rr[::2] = r
    offsets, modes = random_patterns(M, P, n, n, np.random.default_rng([SEED_ROOT, *tag, S_PAT]))
    return Workload(name=f"acc_m{M}_r{r:g}_n{n}", config=0, M=M, U=U, r=rr, eta=np.ones(M),
                    offsets=offsets, modes=modes, order=4, exact=True,
                    description=f"{M} modes, r = {r:g} on every second input, eta = 1, "
                                f"{P} outcomes with {n} clicks; exact and orders 2-4")


def device30_model():
    """The device of the paper's Fig. 2: a 30-mode Haar interferometer, 15
    inputs squeezed at r = 1.4, the others in vacuum, lossless (stream
    [SEED_ROOT, 96, s])."""
    M = 30
    U = haar_unitary(M, np.random.default_rng([SEED_ROOT, 96, S_U]))
    r = np.zeros(M)
    r[:15] = 1.4
    return U, r, np.ones(M)


def small_model(M: int, seed: int, n_squeezed: Optional[int] = None,
                r_range=(0.5, 1.5), eta_range=(0.3, 1.0)):
    """A small random lossy model for pins and edge cases."""
    rng = np.random.default_rng([SEED_ROOT, 99, seed])
    U = haar_unitary(M, rng)
    nsq = M if n_squeezed is None else n_squeezed
    r = np.zeros(M)
    r[:nsq] = rng.uniform(*r_range, size=nsq)
    eta = rng.uniform(*eta_range, size=M)
    return U, r, eta
