"""The exact path at 25-30 clicks (2^25 .. 2^30 terms per row), where no
binary128 reference finishes in reasonable time, against references the
problem fixes:

  - product of independent blocks: with U block-diagonal (ten Haar 3 x 3
    blocks) the state is a product over the blocks, so p(C) is the product of
    the blocks' probabilities (each from the binary128 oracle on 3 modes);
  - U = I: the product of single-mode closed forms (Methods, Model: the
    single squeezed mode, here with loss);
  - relabelling the modes (rows of U and eta permuted with the pattern)
    leaves p unchanged, while the kernel then conditions and expands the modes
    in another order.
Tolerance: relative 1e-10 (the exact path's target).
"""
import numpy as np
import pytest

from oracle import exact128
from workloads import SEED_ROOT, csr_from_lists, haar_unitary

from paper_2106_01445_amd import gbs

pytestmark = pytest.mark.gpu
TOL = 1e-10


def block_model(nb=10, bs=3, seed=7):
    rng = np.random.default_rng([SEED_ROOT, 131, seed])
    M = nb * bs
    U = np.zeros((M, M), complex)
    blocks = []
    for b in range(nb):
        Ub = haar_unitary(bs, rng)
        U[b * bs:(b + 1) * bs, b * bs:(b + 1) * bs] = Ub
        blocks.append(Ub)
    r = rng.uniform(0.6, 1.2, M)
    eta = rng.uniform(0.5, 1.0, M)
    return U, r, eta, blocks


def test_block_product_30_clicks(gpu_ctx):
    nb, bs = 10, 3
    U, r, eta, blocks = block_model(nb, bs)
    M = nb * bs
    drop = {4, 13, 29}
    rows = [list(range(M)), [m for m in range(M) if m not in drop]]
    off, mod = csr_from_lists(rows)
    gpu_ctx.gbs_set_model(U, r, eta)
    out = gpu_ctx.gbs_prob_exact(off, mod)
    assert np.all(out["status"] == 0), out["status"]
    for i, C in enumerate(rows):
        ref = 1.0
        for b in range(nb):
            sl = slice(b * bs, (b + 1) * bs)
            Cb = [m - b * bs for m in C if b * bs <= m < (b + 1) * bs]
            o, mo = csr_from_lists([Cb])
            rb = exact128.exact(bs, blocks[b], r[sl], eta[sl], o, mo)
            ref *= rb["p_hi"][0] + rb["p_lo"][0]
        assert abs(out["p"][i] / ref - 1) < TOL, (len(C), out["p"][i], ref)
    assert out["kappa"].min() > 1e6


def test_product_state_30_clicks(gpu_ctx):
    M = 30
    rng = np.random.default_rng([SEED_ROOT, 132, 0])
    # (strongly enough squeezed that the sum's cancellation, the product of
    # the modes' (1 + P0)/(1 - P0), stays below the 1e20 that double-double
    # resolves)
    r = rng.uniform(1.0, 1.6, M)
    eta = rng.uniform(0.7, 1.0, M)
    gpu_ctx.gbs_set_model(np.eye(M, dtype=complex), r, eta)
    C = list(range(M))
    out = gpu_ctx.gbs_prob_exact(*csr_from_lists([C]))
    assert out["status"][0] == 0
    P0 = (1 + eta * (2 - eta) * np.sinh(r) ** 2) ** -0.5
    assert abs(out["kappa"][0] / np.prod((1 + P0) / (1 - P0)) - 1) < 1e-10
    ref = np.prod(1 - P0)
    assert abs(out["p"][0] / ref - 1) < TOL


def test_cancellation_beyond_double_double_is_flagged(gpu_ctx):
    """A weakly squeezed product state: the signed sum over the 2^n subsets
    cancels by prod (1 + P0)/(1 - P0) ~ 4e36 at 24 clicks, beyond the 1e20
    that double-double resolves, so the row is NaN with GBS_PS_CANCEL (the
    other row, 10 clicks of the same state, cancels by ~2e15 and is exact)."""
    M = 24
    r = np.full(M, 0.35)
    eta = np.full(M, 0.9)
    gpu_ctx.gbs_set_model(np.eye(M, dtype=complex), r, eta)
    P0 = (1 + eta * (2 - eta) * np.sinh(r) ** 2) ** -0.5
    k24 = np.prod((1 + P0) / (1 - P0))
    k10 = np.prod(((1 + P0) / (1 - P0))[:10])
    assert k24 > 1e22 and k10 < 1e16
    out = gpu_ctx.gbs_prob_exact(*csr_from_lists([list(range(M)), list(range(10))]))
    assert out["status"][0] == gbs.GBS_PS_CANCEL and np.isnan(out["p"][0])
    assert out["status"][1] == 0
    ref = np.prod(1 - P0[:10]) * np.prod(P0[10:])
    assert abs(out["p"][1] / ref - 1) < TOL


def test_relabelled_modes_26_clicks(gpu_ctx):
    M = 30
    rng = np.random.default_rng([SEED_ROOT, 133, 0])
    U = haar_unitary(M, rng)
    r = np.zeros(M)
    r[:15] = rng.uniform(0.8, 1.2, 15)
    eta = rng.uniform(0.5, 0.9, M)
    C = sorted(rng.choice(M, 26, replace=False).tolist())
    gpu_ctx.gbs_set_model(U, r, eta)
    a = gpu_ctx.gbs_prob_exact(*csr_from_lists([C]))
    perm = rng.permutation(M)            # output mode i becomes perm[i]
    Up = np.zeros_like(U)
    Up[perm, :] = U
    ep = np.zeros_like(eta)
    ep[perm] = eta
    gpu_ctx.gbs_set_model(Up, r, ep)
    b = gpu_ctx.gbs_prob_exact(*csr_from_lists([sorted(perm[C].tolist())]))
    assert a["status"][0] == 0 and b["status"][0] == 0
    assert abs(a["p"][0] / b["p"][0] - 1) < TOL
