"""The paper's headline case on the GPU (Results, Approximation scheme; Fig. 1):
50 clicks of a lossless 70-mode device with every second input squeezed at
r = 1.6 (workloads.accuracy_workload(70, 1.6, 50, P=16)).  For this pure state
the contour that first tilts to max(n, untilted mean) leaves the sectors that
carry the estimate under its rounding floor; the forward then re-tilts those
rows on the device.  Parity: rows 0 and 1 at order 1 and row 0 at order 2
against the oracle with binary128 sector weights (tests/golden/headline_rows.json,
written by tests/golden/make_headline_rows.py), within the row's own rounding
estimate (floor 1e-9)."""
import json
import os

import numpy as np
import pytest

from workloads import accuracy_workload

from paper_2106_01445_amd import gbs as g

pytestmark = pytest.mark.gpu


def _run(ctx, wl, order):
    import torch
    plan = ctx.gbs_plan_create(wl.offsets, wl.modes, order)
    lp = torch.empty(wl.P, dtype=torch.float64, device="cuda")
    st = torch.empty(wl.P, dtype=torch.int32, device="cuda")
    ctx.gbs_prob_approx_dev(plan, lp, st)
    torch.cuda.synchronize()
    info = plan.info()
    plan.close()
    return lp.cpu().numpy(), st.cpu().numpy(), info


def test_headline_rows_against_binary128_oracle(gpu_ctx):
    rec = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                      "headline_rows.json")))
    wl = accuracy_workload(70, 1.6, 50, P=16)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    for order in sorted({c["order"] for c in rec["cases"]}):
        logp, status, info = _run(gpu_ctx, wl, order)
        # every row resolved at orders 1 and 2 (re-tilted where needed)
        assert np.all(status == 0), (order, status)
        for c in rec["cases"]:
            if c["order"] != order:
                continue
            assert c["n"] == 50 and c["amplification"] < 1e16  # >= 17 of binary128's digits left
            i = c["row"]
            tol = max(1e-9, info["err"][i])
            assert abs(logp[i] - c["logp"]) <= tol, (c, logp[i], info["err"][i])


def test_headline_orders_3_and_4_report_their_contour(gpu_ctx):
    """At orders 3 and 4 a few rows keep estimate weight in sectors that even the
    re-tilted contour (radius at its cap) leaves unresolved: those carry
    GBS_PS_CONTOUR and nothing else; every row has a finite result."""
    wl = accuracy_workload(70, 1.6, 50, P=16)
    gpu_ctx.gbs_set_model(wl.U, wl.r, wl.eta)
    for order in (3, 4):
        logp, status, info = _run(gpu_ctx, wl, order)
        assert np.all(np.isfinite(logp)), order
        assert np.all((status & ~g.GBS_PS_CONTOUR) == 0), (order, status)
        ok = status == 0
        assert ok.sum() >= 8, (order, status)
        assert np.all(info["err"][ok] < 1e-6), (order, info["err"][ok])
