"""GPU parity of the exact click probability (double-double kernel, through the
C ABI) against the binary128 oracle.

Tolerance: relative error <= 1e-10 (the target for the exact path); the kernel
works in double-double throughout, so the measured error is ~1e-16 even where
the signed 2^n-term sum cancels by 1e10.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import exact, exact128, model
from workloads import SEED_ROOT, csr_from_lists, csr_rows, make_workload, small_model

pytestmark = pytest.mark.gpu
TOL = 1e-10


def ref128(M, U, r, eta, off, mod, sigma=None):
    o = exact128.exact(M, U, r, eta, off, mod, sigma=sigma)
    return o["p_hi"] + o["p_lo"], o["kappa"]


def test_m8_all_rows(gpu_ctx):
    wl = make_workload(1)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    out = gpu_ctx.gbs_prob_exact(wl.offsets, wl.modes)
    assert np.all(out["status"] == 0)
    ref, kap = ref128(wl.M, wl.U, wl.r, wl.eta, wl.offsets, wl.modes)
    assert np.max(np.abs(out["p"] / ref - 1)) < TOL
    assert np.allclose(out["kappa"], kap, rtol=1e-8)
    assert np.allclose(out["logp"], np.log(ref), atol=1e-12)


def test_m20_full_batch_sampled(gpu_ctx):
    """20 modes, 4096 rows of 6-14 clicks in one launch; 14 rows (the largest
    click counts included) against binary128; every row resolved."""
    wl = make_workload(2)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    out = gpu_ctx.gbs_prob_exact(wl.offsets, wl.modes)
    assert np.all(out["status"] == 0)
    assert np.all(out["p"] > 0)
    n = np.diff(wl.offsets)
    idx = sorted({*np.flatnonzero(n == 14)[:3].tolist(), *np.flatnonzero(n == 6)[:2].tolist(),
                  *range(0, 4096, 455)})
    sub = wl.subset(idx)
    ref, kap = ref128(wl.M, wl.U, wl.r, wl.eta, sub.offsets, sub.modes)
    assert np.max(np.abs(out["p"][idx] / ref - 1)) < TOL
    assert np.allclose(out["kappa"][idx], kap, rtol=1e-6)
    assert kap.max() > 1e7   # these sums do cancel


@pytest.mark.parametrize("rows", [
    [[], [3], [0, 5], [1, 2, 4]],                       # leaf-only work items
    [list(range(9)), list(range(10)), [0, 2, 3, 5, 6, 8, 9, 10, 11, 12, 13]],  # 9/10/11 clicks
])
def test_edge_rows(gpu_ctx, rows):
    U, r, eta = small_model(14, 20)
    gpu_ctx.gbs_set_model(U, r, eta)
    off, mod = csr_from_lists(rows)
    out = gpu_ctx.gbs_prob_exact(off, mod)
    ref, _ = ref128(14, U, r, eta, off, mod)
    assert np.max(np.abs(out["p"] / ref - 1)) < TOL


def test_all_patterns_sum_to_one(gpu_ctx):
    U, r, eta = small_model(7, 21)
    gpu_ctx.gbs_set_model(U, r, eta)
    import itertools
    rows = [list(c) for k in range(8) for c in itertools.combinations(range(7), k)]
    off, mod = csr_from_lists(rows)
    out = gpu_ctx.gbs_prob_exact(off, mod)
    assert abs(out["p"].sum() - 1.0) < 1e-14


def test_product_state_closed_form(gpu_ctx):
    """U = I: p(C) = prod_C (1 - P0_i) prod_Cbar P0_i; at 14 clicks the signed sum
    cancels by ~3^14, which only an extended-precision sum survives."""
    M = 20
    rng = np.random.default_rng([SEED_ROOT, 97, 1])
    r = rng.uniform(0.5, 1.5, M)
    eta = rng.uniform(0.3, 0.9, M)
    U = np.eye(M, dtype=complex)
    gpu_ctx.gbs_set_model(U, r, eta)
    C = sorted(rng.choice(M, 14, replace=False).tolist())
    off, mod = csr_from_lists([C])
    out = gpu_ctx.gbs_prob_exact(off, mod)
    with mp.workdps(40):
        p0 = [1 / mp.sqrt(1 + mp.mpf(e) * (2 - mp.mpf(e)) * mp.sinh(mp.mpf(x)) ** 2)
              for x, e in zip(r, eta)]
        ref = mp.mpf(1)
        for i in range(M):
            ref *= (1 - p0[i]) if i in C else p0[i]
        rel = float(abs(mp.mpf(out["p"][0]) / ref - 1))
    assert rel < 1e-14
    assert out["kappa"][0] > 1e5


def test_covariance_route(gpu_ctx):
    U, r, eta = small_model(10, 22)
    sig = model.covariance(U, r, eta)
    sig = (sig + sig.T) / 2
    rows = [[0, 1, 4, 7], [2, 3, 5, 6, 8, 9]]
    off, mod = csr_from_lists(rows)
    gpu_ctx.gbs_set_covariance(sig)
    out = gpu_ctx.gbs_prob_exact(off, mod)
    ref, _ = ref128(10, None, r, eta, off, mod, sigma=sig)
    assert np.max(np.abs(out["p"] / ref - 1)) < TOL


def test_errors(gpu_ctx):
    import paper_2106_01445_amd as g
    U, r, eta = small_model(32, 23)
    gpu_ctx.gbs_set_model(U, r, eta)
    off, mod = csr_from_lists([list(range(31))])
    with pytest.raises(g.GBSError) as e:
        gpu_ctx.gbs_prob_exact(off, mod)
    assert e.value.code == -1
    bad = -np.eye(4)
    with pytest.raises(g.GBSError) as e:
        gpu_ctx.gbs_set_covariance(bad)
    assert e.value.code == -2
