"""The paper's fourth-order scheme on the GPU (forward): quadruple clusters,
four-moment fits.  Parity against the CPU oracle (power-series sector weights,
generic in the order) at |log p_gpu - log p_oracle| <= 1e-9 (rows above 40
clicks: their own rounding estimate where larger), against the exact
probability where four moments fix the click distribution (n <= 5), and against
the plain comparison kernel."""
import numpy as np
import pytest

from oracle import approx, exact, model
from workloads import csr_from_lists, csr_rows, make_workload, small_model

from paper_2106_01445_amd import gbs as g

pytestmark = pytest.mark.gpu
TOL = 1e-9


def test_order4_equals_exact_up_to_five_clicks(gpu_ctx):
    """With j = 4 >= n - 1 the fitted click distribution is the true one
    (Results, Approximation scheme), so order 4 returns the exact probability."""
    U, r, eta = small_model(10, 21)
    gpu_ctx.gbs_set_model(U, r, eta)
    Q = model.q_matrix(model.covariance(U, r, eta))
    rows = [[3], [0, 7], [1, 4, 9], [0, 2, 5, 8], [1, 2, 3, 6, 9], [0, 4, 5, 7, 8]]
    off, mod = csr_from_lists(rows)
    out = gpu_ctx.gbs_prob_approx(off, mod, 4)
    assert np.all(out["status"] == 0)
    ref = np.array([np.log(exact.prob_exact_direct(Q, c)[0]) for c in rows])
    assert np.max(np.abs(out["logp"] - ref)) < TOL


def test_order4_m20_sample(gpu_ctx):
    """20 modes, the full 4096-row batch (6-14 clicks) at order 4 in one launch;
    10 rows (smallest and largest click counts included) against the oracle."""
    wl = make_workload(2)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    out = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, 4)
    assert np.all(out["status"] == 0)
    assert np.all(np.isfinite(out["logp"]))
    n = np.diff(wl.offsets)
    idx = sorted({int(np.argmin(n)), int(np.argmax(n)), *range(0, 4096, 512)})
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    rows = csr_rows(wl.offsets, wl.modes)
    ref = np.array([approx.prob_approx(Q, list(rows[i]), 4) for i in idx])
    assert np.max(np.abs(out["logp"][idx] - ref)) < TOL


def test_order4_m70_rows(gpu_ctx):
    """70 modes: 512 rows of the benchmark batch (15-40 clicks) at order 4, all
    finite with status 0; the rows with the fewest clicks against the oracle."""
    wl = make_workload(3, P=512)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    out = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, 4)
    assert np.all(out["status"] == 0)
    assert np.all(np.isfinite(out["logp"]))
    n = np.diff(wl.offsets)
    idx = [int(i) for i in np.argsort(n, kind="stable")[:3]]
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    rows = csr_rows(wl.offsets, wl.modes)
    ref = np.array([approx.prob_approx(Q, list(rows[i]), 4) for i in idx])
    assert np.max(np.abs(out["logp"][idx] - ref)) < TOL


def test_order4_plain_agrees(gpu_ctx):
    """The plain kernel (own LDL^T of every 8x8 cluster block) and the tuned one
    (quadruple units on the eliminated pair and third mode) agree to the parity
    bar: both take the same contour sums through different elimination orders
    (measured spread 2e-10 over these rows)."""
    wl = make_workload(3, P=96)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    a = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, 4)
    b = gpu_ctx.gbs_prob_approx_plain(wl.offsets, wl.modes, 4)
    assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
    assert np.max(np.abs(a["logp"] - b["logp"])) < TOL


def test_order4_segment_lengths_agree(gpu_ctx):
    """Every tunable quadruple-unit length gives the same estimate, up to the
    order of the floating-point sums (about 10^3 quadruple terms per contour
    point here, so a few units in the last place of log p)."""
    import torch
    wl = make_workload(2, P=256)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    plan = gpu_ctx.gbs_plan_create(wl.offsets, wl.modes, 4)
    out = torch.empty(wl.P, dtype=torch.float64, device="cuda")
    res = []
    for seg in (1, 3, 7, 15):
        plan.set_params([seg, 3, 8, 8])
        gpu_ctx.gbs_prob_approx_dev(plan, out)
        torch.cuda.synchronize()
        res.append(out.cpu().numpy().copy())
    for x in res[1:]:
        assert np.max(np.abs(x - res[0])) < 1e-11


def test_order4_argument_errors(gpu_ctx):
    """Order 4 takes rows of at most 64 clicks (the mixed tier runs it in fp64,
    flagged GBS_PS_ESCALATED); order 5 does not exist."""
    U, r, eta = small_model(70, 3)
    gpu_ctx.gbs_set_model(U, r, eta)
    off, mod = csr_from_lists([list(range(65))])
    with pytest.raises(g.GBSError):
        gpu_ctx.gbs_prob_approx(off, mod, 4)
    off, mod = csr_from_lists([list(range(10))])
    out = gpu_ctx.gbs_prob_approx(off, mod, 4, g.GBS_PREC_MIXED)
    assert out["status"][0] == g.GBS_PS_ESCALATED
    with pytest.raises(g.GBSError):
        gpu_ctx.gbs_prob_approx(off, mod, 5)
    out = gpu_ctx.gbs_grad(off, mod, 4, np.ones(1), g.GBS_PREC_MIXED)
    assert out["status"][0] == g.GBS_PS_ESCALATED and np.all(np.isfinite(out["grad_r"]))


def test_order4_rows_above_40_clicks(gpu_ctx):
    """The fourth-order scheme (Results, Approximation scheme; Discussion) on
    rows above 40 clicks (V read from L2, M(w) in LDS): rows of 46 and 49
    clicks of the 100-mode batch, with the rest of a 300-row slice of that
    batch in the same call, against the oracle (tests/golden/order4_rows.json,
    written by tests/golden/make_order4_rows.py).  Tolerance: the row's own
    rounding estimate (gbs_plan_info), floor 1e-9 in log p -- four fitted
    moments amplify the transform's rounding by the fit's sensitivity, which
    the estimate carries."""
    import json
    import os
    import torch
    rec = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "order4_rows.json")))
    wl = make_workload(rec["config"])
    idx = sorted(set(range(300)) | {c["row"] for c in rec["cases"]})
    sub = wl.subset(idx)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    plan = gpu_ctx.gbs_plan_create(sub.offsets, sub.modes, 4)
    lp = torch.empty(sub.P, dtype=torch.float64, device="cuda")
    st = torch.empty(sub.P, dtype=torch.int32, device="cuda")
    gpu_ctx.gbs_prob_approx_dev(plan, lp, st)
    torch.cuda.synchronize()
    logp, status = lp.cpu().numpy(), st.cpu().numpy()
    err = plan.info()["err"]
    plan.close()
    assert np.all((status & g.GBS_PS_FAILED) == 0), status
    assert np.max(np.diff(sub.offsets)) > 40
    for c in rec["cases"]:
        assert c["n"] >= 45
        i = idx.index(c["row"])
        assert err[i] < 1e-7, (c, err[i])
        assert abs(logp[i] - c["logp"]) <= max(1e-9, err[i]), (c, logp[i], err[i])
