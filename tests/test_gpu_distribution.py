"""The whole device's click distribution p(n) and its sector curves p_k(n) on
the GPU (gbs_click_distribution) against the CPU oracle (power-series sector
weights, each sector fitted on its own support), and the exact identities
sum_n p(n) = 1 and sum_n n p(n) = sum_l (1 - P_vac(l)) at the paper's Fig. 2
device.  The GPU takes the sector weights from a contour transform whose
rounding is ~1e-16 of the largest tilted weight, so the bar is absolute:
|p_gpu(n) - p_oracle(n)| <= 1e-10 (measured up to 1.5e-11, at order 4, from
the few-photon sectors, whose moments carry that rounding relative to their
own small weight into four-moment fits)."""
import numpy as np
import pytest

from oracle import approx, model
from workloads import device30_model, small_model

pytestmark = pytest.mark.gpu
ABS = 1e-10


@pytest.mark.parametrize("M,seed", [(12, 41), (16, 42)])
@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_distribution_matches_oracle(gpu_ctx, M, seed, order):
    U, r, eta = small_model(M, seed, n_squeezed=M // 2, r_range=(0.6, 1.0), eta_range=(0.5, 0.9))
    gpu_ctx.gbs_set_model(U, r, eta)
    ks = (0, 1, 3, 7, 12)
    out = gpu_ctx.gbs_click_distribution(order, ks)
    assert out["status"] == 0
    Q = model.q_matrix(model.covariance(U, r, eta))
    p, curves, det = approx.click_distribution(Q, order, ks=ks)
    assert det["nfail"] == 0
    assert np.max(np.abs(out["p_n"] - p)) < ABS
    for i, k in enumerate(ks):
        assert np.max(np.abs(out["p_k"][i] - curves[k])) < ABS


@pytest.mark.parametrize("order", [2, 4])
def test_fig2_device_norm_and_mean(gpu_ctx, order):
    """30 modes, 15 inputs at r = 1.4, lossless (the device of Fig. 2): the
    distribution sums to 1 and its mean is the exact mean click number."""
    U, r, eta = device30_model()
    gpu_ctx.gbs_set_model(U, r, eta)
    out = gpu_ctx.gbs_click_distribution(order, (20, 110))
    assert out["status"] == 0
    p = out["p_n"]
    assert np.all(p >= -1e-14)
    assert p.sum() == pytest.approx(1.0, abs=1e-10)
    Q = model.q_matrix(model.covariance(U, r, eta))
    mean = sum(1.0 - model.vacuum_prob(Q, [l]) for l in range(30))
    assert float(np.arange(31) @ p) == pytest.approx(mean, abs=1e-9)
    # every sector's curve lies on its support and is part of p(n)
    assert np.all(out["p_k"][0][21:] == 0.0)
    assert np.all(out["p_k"] <= p + 1e-15)


def test_distribution_argument_errors(gpu_ctx):
    from paper_2106_01445_amd import gbs as g
    U, r, eta = small_model(41, 5)
    gpu_ctx.gbs_set_model(U, r, eta)
    with pytest.raises(g.GBSError):
        gpu_ctx.gbs_click_distribution(2)
    U, r, eta = small_model(8, 5)
    gpu_ctx.gbs_set_model(U, r, eta)
    with pytest.raises(g.GBSError):
        gpu_ctx.gbs_click_distribution(5)
