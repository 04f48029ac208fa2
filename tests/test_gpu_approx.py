"""GPU parity of the order-j estimate (libgbs.so, through the C ABI) against the
CPU oracle (power-series sector weights, no contour).

Tolerance: |log p_gpu - log p_oracle| <= 1e-9, i.e. relative error of p_hat
<= 1e-9.  The GPU extracts the sector moments by a DFT on a contour of K points
at radius rho, with aliasing (rho/R)^K <= 1e-16 and rounding of order 1e-16 of
the tilted sum; the fits add ~1e-12; measured spread is <= 1e-10.
"""
import json
import os

import numpy as np
import pytest

from oracle import approx, exact, model
from workloads import csr_from_lists, csr_rows, make_workload, small_model

pytestmark = pytest.mark.gpu
TOL = 1e-9


def oracle_logp(wl, idx, order=None):
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    rows = csr_rows(wl.offsets, wl.modes)
    return np.array([approx.prob_approx(Q, list(rows[i]), order or wl.order) for i in idx])


def test_model_build(gpu_ctx):
    wl = make_workload(3, P=1)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    qi, ld = gpu_ctx.gbs_get_model()
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    assert np.max(np.abs(qi - np.linalg.inv(Q))) < 1e-12
    assert ld == pytest.approx(np.linalg.slogdet(Q)[1], abs=1e-11)


def test_m8_all_rows(gpu_ctx):
    """8 modes, r = 1 on all inputs, eta = 1: every row, order 2."""
    wl = make_workload(1)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    out = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, 2)
    assert np.all(out["status"] == 0)
    ref = oracle_logp(wl, range(wl.P), 2)
    assert np.max(np.abs(out["logp"] - ref)) < TOL


@pytest.mark.parametrize("order", [1, 2, 3])
def test_m20_sample(gpu_ctx, order):
    """20 modes: the full 4096-row batch in one launch; 35 rows against the
    oracle: three of every click count 6..14 (seeded draw) and every 512th."""
    wl = make_workload(2)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    out = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, order)
    assert np.all(out["status"] == 0)
    assert np.all(np.isfinite(out["logp"]))
    n = np.diff(wl.offsets)
    rng = np.random.default_rng(2003)
    per = [rng.choice(np.flatnonzero(n == k), 3, replace=False) for k in range(int(n.min()), int(n.max()) + 1)]
    idx = sorted({*(int(i) for i in np.concatenate(per)), *range(0, 4096, 512)})
    ref = oracle_logp(wl, idx, order)
    assert np.max(np.abs(out["logp"][idx] - ref)) < TOL


def test_m70_full_batch_sampled(gpu_ctx):
    """70 modes, 10^4 rows of 15-40 clicks, order 3, in the launch configuration
    the benchmark times; every row finite with status 0; against the oracle:
    three rows computed here (the largest click count among them) and the 104
    rows of tests/golden/m70_rows.json (four of every click count 15..40,
    written by make_m70_rows.py from the oracle alone)."""
    wl = make_workload(3)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    out = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, 3)
    assert np.all(out["status"] == 0)
    assert np.all(np.isfinite(out["logp"]))
    n = np.diff(wl.offsets)
    idx = [int(np.argmax(n)), 7, 4242]
    ref = oracle_logp(wl, idx, 3)
    assert np.max(np.abs(out["logp"][idx] - ref)) < TOL
    rec = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "m70_rows.json")))
    assert len(rec["cases"]) == 104 and {c["n"] for c in rec["cases"]} == set(range(15, 41))
    rows = np.array([c["row"] for c in rec["cases"]])
    gold = np.array([c["logp"] for c in rec["cases"]])
    assert np.all(n[rows] == [c["n"] for c in rec["cases"]])
    err = np.abs(out["logp"][rows] - gold)
    assert np.max(err) < TOL, (np.max(err), int(rows[np.argmax(err)]))


def test_edge_rows(gpu_ctx):
    """Ragged batch with an empty row (probability that nothing clicks), single
    clicks (exact at any order) and a row at order >= n-1 (exact)."""
    U, r, eta = small_model(9, 11)
    gpu_ctx.gbs_set_model(U, r, eta)
    rows = [[], [4], [0, 8], [1, 2, 3], [], [0, 1, 2, 3, 4, 5, 6, 7, 8]]
    off, mod = csr_from_lists(rows)
    out = gpu_ctx.gbs_prob_approx(off, mod, 2)
    assert np.all(out["status"] == 0)
    Q = model.q_matrix(model.covariance(U, r, eta))
    for i, C in enumerate(rows):
        ref = approx.prob_approx(Q, C, 2)
        assert abs(out["logp"][i] - ref) < TOL, (i, out["logp"][i], ref)
        if len(C) <= 3:
            ex = np.log(exact.prob_exact_direct(Q, C)[0])
            assert abs(out["logp"][i] - ex) < TOL


def test_empty_batch(gpu_ctx):
    U, r, eta = small_model(4, 12)
    gpu_ctx.gbs_set_model(U, r, eta)
    out = gpu_ctx.gbs_prob_approx(np.zeros(1, np.int32), np.zeros(0, np.int32), 2)
    assert out["logp"].shape == (0,)


def test_deterministic(gpu_ctx):
    wl = make_workload(2, P=256)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    a = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, 3)["logp"]
    b = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, 3)["logp"]
    assert np.array_equal(a, b)


def test_frozen_plan_reuse(gpu_ctx):
    import torch
    wl = make_workload(2, P=64)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    plan = gpu_ctx.gbs_plan_create(wl.offsets, wl.modes, 2)
    out = torch.empty(64, dtype=torch.float64, device="cuda")
    gpu_ctx.gbs_prob_approx_dev(plan, out)
    torch.cuda.synchronize()
    first = out.cpu().numpy().copy()
    info = plan.info()
    plan.freeze(True)
    gpu_ctx.gbs_prob_approx_dev(plan, out)
    torch.cuda.synchronize()
    assert np.array_equal(first, out.cpu().numpy())
    assert np.array_equal(info["K"], plan.info()["K"])
    assert np.all(info["rho"] < info["rconv"])
    plan.close()


@pytest.mark.parametrize("rows,order", [
    ([[1, 0]], 2),            # not ascending
    ([[2, 2]], 2),            # duplicate
    ([[0, 199]], 2),          # out of range
    ([[0, 1]], 5),            # order outside 1..4
    ([[0, 1]], 0),
    ([list(range(65))], 3),   # more clicks than order 3 supports
    ([list(range(65))], 4),   # more clicks than order 4 supports
    ([list(range(129))], 2),  # more clicks than supported
])
def test_argument_errors(gpu_ctx, rows, order):
    import paper_2106_01445_amd as g
    U, r, eta = small_model(140, 13)
    gpu_ctx.gbs_set_model(U, r, eta)
    off, mod = csr_from_lists(rows)
    with pytest.raises(g.GBSError) as e:
        gpu_ctx.gbs_prob_approx(off, mod, order)
    assert e.value.code == -1


@pytest.mark.parametrize("cfg,order,P", [(1, 2, None), (2, 3, 512), (3, 3, 64)])
def test_plain_kernel_agrees(gpu_ctx, cfg, order, P):
    """The plain comparison kernel (own LDL^T per cluster, no reuse) and the tuned
    contour kernel agree: they share only the eigen-decomposition, the plan and
    the fits, so this cross-checks the M(w) tiles on the matrix cores, the
    2x2-block eliminations and the work units."""
    wl = make_workload(cfg, P=P)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    a = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, order)
    b = gpu_ctx.gbs_prob_approx_plain(wl.offsets, wl.modes, order)
    assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
    assert np.max(np.abs(a["logp"] - b["logp"])) < 1e-10


def test_plan_params_and_tuner(gpu_ctx):
    """Launch choices change the speed, not the results: every setting the tuner
    may pick gives the same log p (to the order of the sums), and the tuner
    returns values from its candidate sets; bad values are rejected."""
    import paper_2106_01445_amd as g
    import torch
    wl = make_workload(2, P=300)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    plan = gpu_ctx.gbs_plan_create(wl.offsets, wl.modes, 3)
    assert list(plan.get_params()) == [3, 3, 8, 8]
    out = torch.empty(wl.P, dtype=torch.float64, device="cuda")
    gpu_ctx.gbs_prob_approx_dev(plan, out)
    torch.cuda.synchronize()
    ref = out.cpu().numpy().copy()
    for prm in ([2, 3, 4, 2], [6, 2, 16, 4], [1, 6, 64, 1]):
        plan.set_params(prm)
        gpu_ctx.gbs_prob_approx_dev(plan, out)
        torch.cuda.synchronize()
        assert np.max(np.abs(out.cpu().numpy() - ref)) < 1e-12, prm
    for bad in ([0, 3, 8, 8], [3, 3, 12, 8], [3, 3, 8, 3]):
        with pytest.raises(g.GBSError):
            plan.set_params(bad)
    prm = plan.tune(3)
    assert prm[0] in (2, 3, 4, 6, 8, 12) and prm[1] in (2, 3, 4, 6)
    assert prm[2] in (4, 8, 16) and prm[3] in (2, 4, 8)
    assert list(plan.get_params()) == list(prm)
    gpu_ctx.gbs_prob_approx_dev(plan, out)
    torch.cuda.synchronize()
    assert np.max(np.abs(out.cpu().numpy() - ref)) < 1e-12
    plan.close()


@pytest.mark.parametrize("cfg,order,P", [(2, 3, None), (3, 3, 1000), (4, 3, 300), (5, 2, 100)])
def test_mixed_precision(gpu_ctx, cfg, order, P):
    """GBS_PREC_MIXED (fp32 cluster eliminations, fp64 everything else) against
    the fp64 path on the same batch: every row within the tier's target,
    |d log p| <= 1e-5, where rows whose rounding bound exceeds 1e-5 have been
    run again in fp64 (GBS_PS_ESCALATED, and then equal to the fp64 value); no
    other status bit.  The bound of every row that was not escalated holds."""
    import torch
    import paper_2106_01445_amd as g
    wl = make_workload(cfg, P=P)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    a = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, order)
    assert np.all(a["status"] == 0)
    plan = gpu_ctx.gbs_plan_create(wl.offsets, wl.modes, order, prec=g.GBS_PREC_MIXED)
    lp = torch.empty(wl.P, dtype=torch.float64, device="cuda")
    st = torch.empty(wl.P, dtype=torch.int32, device="cuda")
    gpu_ctx.gbs_prob_approx_dev(plan, lp, st)
    torch.cuda.synchronize()
    b, bs = lp.cpu().numpy(), st.cpu().numpy()
    err = plan.info()["err"]
    plan.close()
    assert np.all((bs & ~g.gbs.GBS_PS_ESCALATED) == 0), np.unique(bs)
    esc = (bs & g.gbs.GBS_PS_ESCALATED) != 0
    d = np.abs(a["logp"] - b)
    assert np.max(d) <= 1e-5, (np.max(d), np.median(d), esc.mean())
    assert np.max(d[esc], initial=0.0) < 1e-9
    assert np.all(d[~esc] <= np.maximum(err[~esc], 1e-9)), np.max(d[~esc] / err[~esc])
    assert np.all(err[~esc] <= 1e-5)


def test_mixed_precision_where_no_fp32_kernel_exists(gpu_ctx):
    """The exact path, order 4 and the gradient have no fp32 kernels: asked for
    the mixed tier they run at the higher precision and flag every row
    GBS_PS_ESCALATED, with results equal to the fp64 call's; the plain
    comparison kernel rejects the tier."""
    import paper_2106_01445_amd as g
    wl = make_workload(1)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    esc = g.gbs.GBS_PS_ESCALATED
    a = gpu_ctx.gbs_prob_exact(wl.offsets, wl.modes)
    b = gpu_ctx.gbs_prob_exact(wl.offsets, wl.modes, prec=g.GBS_PREC_MIXED)
    assert np.all(a["status"] == 0) and np.all(b["status"] == esc)
    assert np.array_equal(a["p"], b["p"])
    a = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, 4)
    b = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, 4, prec=g.GBS_PREC_MIXED)
    assert np.all(a["status"] == 0) and np.all(b["status"] == esc)
    assert np.array_equal(a["logp"], b["logp"])
    w = np.linspace(0.5, 1.5, wl.P)
    a = gpu_ctx.gbs_grad(wl.offsets, wl.modes, 2, w)
    b = gpu_ctx.gbs_grad(wl.offsets, wl.modes, 2, w, prec=g.GBS_PREC_MIXED)
    assert np.all(a["status"] == 0) and np.all(b["status"] == esc)
    assert np.array_equal(a["logp"], b["logp"])
    # (the adjoint sums over clusters with atomic adds: equal up to their order)
    for k in ("grad_r", "grad_eta"):
        assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-14 * np.max(np.abs(a[k])))
    with pytest.raises(g.GBSError) as e:
        gpu_ctx.gbs_prob_approx_plain(wl.offsets, wl.modes, 2, prec=g.GBS_PREC_MIXED)
    assert e.value.code == -1
