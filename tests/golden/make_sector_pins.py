"""Writes sector_pins.json: sector weights g_T[kappa] of the sub-ensemble of
sampled rows of the 70-, 100- and 144-mode batches (workloads.py), for the
empty cluster and one cluster of each size up to the row's order, evaluated in
binary128 from the definition (oracle/sectors128.c: Schur complement,
eigenvalues, power series), on the sectors that carry the order-j estimate
(those holding at least 1e-8 of it in the fp64 oracle).  The rows are the
smallest and the largest of each batch, one more drawn at random, and at 144
modes two rows whose contour radius would be capped below the saddle point.
Calls only oracle/ and workloads.py; run from the repository root (about ten
minutes on eight cores):

    python tests/golden/make_sector_pins.py
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import approx, model, sectors128  # noqa: E402
from oracle.exact import conditional_W  # noqa: E402
from workloads import csr_rows, make_workload  # noqa: E402

# rows of the 144-mode batch whose saddle-point radius lies beyond 0.98 of the
# convergence radius (the cap of the contour plan)
CAPPED_144 = [1146, 3675]


def rows_for(cfg):
    wl = make_workload(cfg)
    ns = np.diff(wl.offsets)
    order = np.argsort(ns, kind="stable")
    idx = [int(order[0]), int(order[-1]), int(np.random.default_rng(2000 + cfg).integers(wl.P))]
    if cfg == 5:
        idx += CAPPED_144
    return wl, idx


def clusters(n, order):
    out = [(), (n // 2,), (1, n - 2)]
    if order >= 3:
        out.append((0, n // 3, n - 1))
    return out


def task(args):
    cfg, row, order = args
    wl = make_workload(cfg)
    C = list(csr_rows(wl.offsets, wl.modes)[row])
    n = len(C)
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    W = conditional_W(Q, C)
    W = 0.5 * (W + W.T)
    lp, det = approx.prob_approx(Q, C, order, return_detail=True)
    terms = det["terms"]
    top = max(terms.values())
    tot = top + np.log(sum(np.exp(v - top) for v in terms.values()))
    kaps = sorted(k for k, v in terms.items() if v - tot >= np.log(1e-8))
    L = max(kaps) + 1
    out = []
    for T in clusters(n, order):
        hi, lo = sectors128.sector_weights(W, T, L)
        out.append({"T": list(T), "kappa": kaps, "g_hi": [hi[k] for k in kaps], "g_lo": [lo[k] for k in kaps]})
    print(cfg, row, n, len(kaps), flush=True)
    return {"config": cfg, "row": row, "n": n, "order": order, "logp_oracle_fp64": lp, "clusters": out}


def main():
    sectors128.build(force=True)
    jobs = []
    for cfg, order in ((3, 3), (4, 3), (5, 2)):
        _, idx = rows_for(cfg)
        jobs += [(cfg, i, order) for i in idx]
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count())) as ex:
        cases = list(ex.map(task, jobs))
    rec = {"generator": "tests/golden/make_sector_pins.py", "cases": cases}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "sector_pins.json"), "w") as f:
        json.dump(rec, f)


if __name__ == "__main__":
    main()
