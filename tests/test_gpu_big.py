"""Rows with more than 40 clicks (the 100- and 144-mode workloads): the path
that keeps the eigenvectors and M(w) in HBM, with its own eigen-decomposition
(Householder tridiagonalisation + implicit QL), against the CPU oracle.

Expected values for the full batches come from tests/golden/big_rows.json,
written by tests/golden/make_big_rows.py from oracle/ alone (a 60-click row at
order 3 takes the oracle about 30 s).  Smaller cases call the oracle directly.
Tolerance as for the smaller rows: 1e-9 in log p.
"""
import json
import os

import numpy as np
import pytest

from oracle import approx, model
from workloads import csr_from_lists, make_workload, small_model

pytestmark = pytest.mark.gpu
TOL = 1e-9
HERE = os.path.dirname(os.path.abspath(__file__))


def golden(cfg):
    rec = json.load(open(os.path.join(HERE, "golden", "big_rows.json")))
    return [c for c in rec["cases"] if c["config"] == cfg]


@pytest.mark.parametrize("cfg,order", [(4, 3), (5, 2)])
def test_full_batch_vs_golden(gpu_ctx, cfg, order):
    """100 modes / 10^4 rows of 25-60 clicks at order 3, and 144 modes / 4096
    rows of 40-110 clicks at order 2, each in one call; every row finite with
    status 0, sampled rows (smallest and largest click counts among them)
    against the oracle."""
    wl = make_workload(cfg)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    out = gpu_ctx.gbs_prob_approx(wl.offsets, wl.modes, order)
    assert np.all(out["status"] == 0)
    assert np.all(np.isfinite(out["logp"]))
    cases = golden(cfg)
    assert cases
    for c in cases:
        assert c["order"] == order
        assert abs(out["logp"][c["row"]] - c["logp"]) < TOL, (c, out["logp"][c["row"]])


def test_rows_across_the_lds_limit(gpu_ctx):
    """A 50-mode model, rows of 38-45 clicks in one batch (both paths), order 2
    and 3, against the oracle."""
    U, r, eta = small_model(50, 21, n_squeezed=25, r_range=(1.0, 1.5), eta_range=(0.3, 0.6))
    rng = np.random.default_rng(77)
    rows = [sorted(rng.choice(50, size=k, replace=False).tolist()) for k in (38, 40, 41, 45)]
    off, mod = csr_from_lists(rows)
    gpu_ctx.gbs_set_model(U, r, eta)
    Q = model.q_matrix(model.covariance(U, r, eta))
    for order in (2, 3):
        out = gpu_ctx.gbs_prob_approx(off, mod, order)
        assert np.all(out["status"] == 0)
        for i in ([0, 2] if order == 3 else range(len(rows))):
            ref = approx.prob_approx(Q, rows[i], order)
            assert abs(out["logp"][i] - ref) < TOL, (order, len(rows[i]), out["logp"][i], ref)


def test_big_grad_directional(gpu_ctx):
    """144 modes, 24 rows of the batch (40-110 clicks), order 2: the adjoint
    against central differences of the GPU forward on a frozen plan along two
    random directions in (r, eta)."""
    import torch
    wl = make_workload(5).subset(list(range(24)))
    M = wl.M
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    plan = gpu_ctx.gbs_plan_create(wl.offsets, wl.modes, 2)
    dev = torch.device("cuda")
    ure = torch.tensor(np.ascontiguousarray(wl.U.real), device=dev)
    uim = torch.tensor(np.ascontiguousarray(wl.U.imag), device=dev)
    logp = torch.empty(wl.P, dtype=torch.float64, device=dev)
    st = torch.empty(wl.P, dtype=torch.int32, device=dev)

    def f(r, eta):
        gpu_ctx.gbs_set_model_dev(ure, uim, torch.tensor(r, device=dev), torch.tensor(eta, device=dev))
        gpu_ctx.gbs_prob_approx_dev(plan, logp, st)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0
        return logp.cpu().numpy().copy()

    w = np.random.default_rng(8).uniform(0.5, 1.5, wl.P)
    f(wl.r, wl.eta)
    plan.freeze(True)
    dl = torch.tensor(w, device=dev)
    gr = torch.empty(M, dtype=torch.float64, device=dev)
    ge = torch.empty(M, dtype=torch.float64, device=dev)
    gpu_ctx.gbs_set_model_dev(ure, uim, torch.tensor(wl.r, device=dev), torch.tensor(wl.eta, device=dev))
    gpu_ctx.gbs_grad_dev(plan, dl, logp, gr, ge, st)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    g = np.concatenate([gr.cpu().numpy(), ge.cpu().numpy()])
    assert np.all(np.isfinite(g))
    mask = np.concatenate([wl.r > 0, np.ones(M, bool)])
    rng = np.random.default_rng(9)
    h = 1e-5
    for _ in range(2):
        v = rng.standard_normal(2 * M) * mask
        v /= np.linalg.norm(v)
        x0 = np.concatenate([wl.r, wl.eta])
        xp, xm = x0 + h * v, x0 - h * v
        fd = (w @ f(xp[:M], xp[M:]) - w @ f(xm[:M], xm[M:])) / (2 * h)
        assert abs(g @ v - fd) < 1e-4 * np.linalg.norm(g), (g @ v, fd)
    plan.close()


@pytest.mark.parametrize("order", [2, 3])
def test_grad_few_large_rows(gpu_ctx, order):
    """Two rows above 40 clicks next to two below (so most of the per-XCD
    queues of the larger rows' adjoint are empty and their workgroups take
    items from the others): the adjoint against central differences of the
    GPU forward on the frozen plan along random directions in (r, eta)."""
    import torch
    M = 50
    U, r, eta = small_model(M, 21, n_squeezed=25, r_range=(1.0, 1.5), eta_range=(0.3, 0.6))
    rng = np.random.default_rng(78)
    rows = [sorted(rng.choice(M, size=k, replace=False).tolist()) for k in (38, 41, 40, 45)]
    off, mod = csr_from_lists(rows)
    P = len(rows)
    gpu_ctx.gbs_set_model(U, r, eta)
    plan = gpu_ctx.gbs_plan_create(off, mod, order)
    dev = torch.device("cuda")
    ure = torch.tensor(np.ascontiguousarray(U.real), device=dev)
    uim = torch.tensor(np.ascontiguousarray(U.imag), device=dev)
    logp = torch.empty(P, dtype=torch.float64, device=dev)
    st = torch.empty(P, dtype=torch.int32, device=dev)

    def f(rr, ee):
        gpu_ctx.gbs_set_model_dev(ure, uim, torch.tensor(rr, device=dev), torch.tensor(ee, device=dev))
        gpu_ctx.gbs_prob_approx_dev(plan, logp, st)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0
        return logp.cpu().numpy().copy()

    w = np.array([0.7, 1.3, 0.9, 1.1])
    f(r, eta)
    plan.freeze(True)
    dl = torch.tensor(w, device=dev)
    gr = torch.empty(M, dtype=torch.float64, device=dev)
    ge = torch.empty(M, dtype=torch.float64, device=dev)
    gpu_ctx.gbs_set_model_dev(ure, uim, torch.tensor(r, device=dev), torch.tensor(eta, device=dev))
    gpu_ctx.gbs_grad_dev(plan, dl, logp, gr, ge, st)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    g = np.concatenate([gr.cpu().numpy(), ge.cpu().numpy()])
    assert np.all(np.isfinite(g))
    mask = np.concatenate([r > 0, np.ones(M, bool)])
    rng = np.random.default_rng(79)
    h = 1e-5
    for _ in range(3):
        v = rng.standard_normal(2 * M) * mask
        v /= np.linalg.norm(v)
        xp = np.concatenate([r, eta]) + h * v
        xm = np.concatenate([r, eta]) - h * v
        fd = (w @ f(xp[:M], xp[M:]) - w @ f(xm[:M], xm[M:])) / (2 * h)
        assert abs(g @ v - fd) < 1e-4 * np.linalg.norm(g), (g @ v, fd)
    plan.close()


def test_grad_m144_vs_reference_gradient(gpu_ctx):
    """144 modes, order 2: the hand-written adjoint (gbs_grad: forward, then
    the adjoint with the forward's contour plan) against the reference
    gradient of the oracle (torch fp64 autograd through the power-series
    oracle, tests/golden/grad_rows.json) for five rows of 40-110 clicks, two of
    them with a capped contour radius: every component of d L / d r and
    d L / d eta within 1e-7 of the largest."""
    rec = json.load(open(os.path.join(HERE, "golden", "grad_rows.json")))
    wl = make_workload(5).subset(rec["rows"])
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    out = gpu_ctx.gbs_grad(wl.offsets, wl.modes, 2, np.array(rec["weights"]))
    assert np.all(out["status"] == 0), out["status"]
    g = np.concatenate([out["grad_r"], out["grad_eta"]])
    ref = np.concatenate([rec["grad_r"], rec["grad_eta"]])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(g - ref)) < 1e-7 * scale, (np.max(np.abs(g - ref)) / scale, int(np.argmax(np.abs(g - ref))))
    assert abs(float(np.dot(rec["weights"], out["logp"])) - rec["loss"]) < 1e-8


def test_capped_rows_in_golden_set():
    """The forward golden set holds at least five 144-mode rows whose radius is
    capped (they are checked with the whole batch above)."""
    assert sum(1 for c in golden(5) if c.get("capped_radius")) >= 5


def test_grad_order2_up_to_128_clicks(gpu_ctx):
    """Order 2, the 144-mode model, rows of 49, 97, 121 and 128 clicks (2n
    from 98 to 256: one to two column tiles of R per wavefront of the order-2
    adjoint, up to its 17 register tiles): the adjoint against central
    differences of the GPU forward on the frozen plan along random directions
    in (r, eta)."""
    import torch
    from paper_2106_01445_amd import gbs as gb
    wl = make_workload(5)
    M = wl.M
    rng = np.random.default_rng(88)
    rows = [sorted(rng.choice(M, size=k, replace=False).tolist()) for k in (49, 97, 121, 128)]
    off, mod = csr_from_lists(rows)
    P = len(rows)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    plan = gpu_ctx.gbs_plan_create(off, mod, 2)
    dev = torch.device("cuda")
    ure = torch.tensor(np.ascontiguousarray(wl.U.real), device=dev)
    uim = torch.tensor(np.ascontiguousarray(wl.U.imag), device=dev)
    logp = torch.empty(P, dtype=torch.float64, device=dev)
    st = torch.empty(P, dtype=torch.int32, device=dev)

    def f(rr, ee):
        gpu_ctx.gbs_set_model_dev(ure, uim, torch.tensor(rr, device=dev), torch.tensor(ee, device=dev))
        gpu_ctx.gbs_prob_approx_dev(plan, logp, st)
        torch.cuda.synchronize()
        assert int((st & gb.GBS_PS_FAILED).sum()) == 0
        return logp.cpu().numpy().copy()

    w = np.array([0.8, 1.2, 0.9, 1.1])
    f0 = f(wl.r, wl.eta)
    assert np.all(np.isfinite(f0))
    plan.freeze(True)
    dl = torch.tensor(w, device=dev)
    gr = torch.empty(M, dtype=torch.float64, device=dev)
    ge = torch.empty(M, dtype=torch.float64, device=dev)
    gpu_ctx.gbs_set_model_dev(ure, uim, torch.tensor(wl.r, device=dev), torch.tensor(wl.eta, device=dev))
    gpu_ctx.gbs_grad_dev(plan, dl, logp, gr, ge, st)
    torch.cuda.synchronize()
    g = np.concatenate([gr.cpu().numpy(), ge.cpu().numpy()])
    assert np.all(np.isfinite(g))
    mask = np.concatenate([wl.r > 0, np.ones(M, bool)])
    h = 1e-5
    for _ in range(2):
        v = rng.standard_normal(2 * M) * mask
        v /= np.linalg.norm(v)
        xp = np.concatenate([wl.r, wl.eta]) + h * v
        xm = np.concatenate([wl.r, wl.eta]) - h * v
        fd = (w @ f(xp[:M], xp[M:]) - w @ f(xm[:M], xm[M:])) / (2 * h)
        assert abs(g @ v - fd) < 1e-4 * np.linalg.norm(g), (g @ v, fd)
    plan.close()
