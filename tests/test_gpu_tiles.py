"""Rows of every click count from 1 to 40 on the 70-mode model, order 3.

The kernels keep these rows in LDS with V and d_k zero-padded to whole 16-wide
tiles (2n rounded up to 16T) and the adjoint's Z(w) copied into a padded packed
triangle, so the tile edges (2n = 16T and 2n = 16T + 2) are the cases where a
padding or bounds mistake would show.  Checked here:

  - the forward against the plain comparison kernel (own dot products for
    M(w), own LDL^T per cluster, no padding) at every click count, to 1e-10
    in log p;
  - the forward against the CPU oracle (power-series sectors, no contour) at
    the click counts on and next to the tile edges, to 1e-9 in log p;
  - the adjoint against central differences of the GPU forward on the frozen
    plan along random directions in (r, eta), to 1e-4 of |grad|.
"""
import numpy as np
import pytest

from oracle import approx, model
from workloads import csr_from_lists, make_workload

pytestmark = pytest.mark.gpu
EDGE_COUNTS = [1, 2, 7, 8, 9, 15, 16, 17, 23, 24, 25, 31, 32, 33, 39, 40]


def rows_all_counts(M, seed):
    rng = np.random.default_rng([2106, 1445, seed])
    return [sorted(rng.choice(M, size=n, replace=False).tolist()) for n in range(1, 41)]


def test_forward_every_click_count(gpu_ctx):
    wl = make_workload(3, P=1)
    rows = rows_all_counts(wl.M, 1)
    off, mod = csr_from_lists(rows)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    a = gpu_ctx.gbs_prob_approx(off, mod, 3)
    b = gpu_ctx.gbs_prob_approx_plain(off, mod, 3)
    assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
    assert np.all(np.isfinite(a["logp"]))
    assert np.max(np.abs(a["logp"] - b["logp"])) < 1e-10
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    for n in EDGE_COUNTS:
        ref = approx.prob_approx(Q, rows[n - 1], 3)
        assert abs(a["logp"][n - 1] - ref) < 1e-9, (n, a["logp"][n - 1], ref)


def test_adjoint_every_click_count(gpu_ctx):
    import torch
    wl = make_workload(3, P=1)
    rows = rows_all_counts(wl.M, 2)
    off, mod = csr_from_lists(rows)
    P, M = len(rows), wl.M
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    plan = gpu_ctx.gbs_plan_create(off, mod, 3)
    dev = torch.device("cuda")
    ure = torch.tensor(np.ascontiguousarray(wl.U.real), device=dev)
    uim = torch.tensor(np.ascontiguousarray(wl.U.imag), device=dev)
    logp = torch.empty(P, dtype=torch.float64, device=dev)
    st = torch.empty(P, dtype=torch.int32, device=dev)

    def f(r, eta):
        gpu_ctx.gbs_set_model_dev(ure, uim, torch.tensor(r, device=dev), torch.tensor(eta, device=dev))
        gpu_ctx.gbs_prob_approx_dev(plan, logp, st)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0
        return logp.cpu().numpy().copy()

    w = np.random.default_rng(11).uniform(0.5, 1.5, P)
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
    # inputs with r = 0 (vacuum) stay in vacuum: perturb only squeezed r_j
    mask = np.concatenate([wl.r > 0, np.ones(M, bool)])
    rng = np.random.default_rng(12)
    h = 1e-5
    for _ in range(3):
        v = rng.standard_normal(2 * M) * mask
        v /= np.linalg.norm(v)
        xp = np.concatenate([wl.r, wl.eta]) + h * v
        xm = np.concatenate([wl.r, wl.eta]) - h * v
        fd = (w @ f(xp[:M], xp[M:]) - w @ f(xm[:M], xm[M:])) / (2 * h)
        assert abs(g @ v - fd) < 1e-4 * np.linalg.norm(g), (g @ v, fd)
    plan.close()
