"""Writes big_rows.json: log p-hat from the CPU oracle (power-series sectors,
max-entropy fits; see oracle/approx.py) for sampled rows of the 100-mode
(order 3) and 144-mode (order 2) batches of workloads.py, and for five rows of
the 144-mode batch whose saddle-point radius lies beyond 0.98 of the
convergence radius (the GPU caps the contour radius there).  Calls only
oracle/ and workloads.py; run from the repository root:

    python tests/golden/make_big_rows.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import approx, model  # noqa: E402
from workloads import csr_rows, make_workload  # noqa: E402


def sample(ns, k, seed):
    order = np.argsort(ns, kind="stable")
    idx = {int(order[0]), int(order[-1])}
    rng = np.random.default_rng(seed)
    idx.update(int(i) for i in rng.choice(len(ns), size=k, replace=False))
    return sorted(idx)


# rows of the 144-mode batch whose saddle-point radius is capped (tilted mean
# at the cap 0.83 .. 0.89 of the click count)
CAPPED_144 = [1146, 1667, 3758, 488, 3675]


def main():
    out = {"generator": "tests/golden/make_big_rows.py", "cases": []}
    for cfg, order, k in ((4, 3, 3), (5, 2, 4)):
        wl = make_workload(cfg)
        rows = csr_rows(wl.offsets, wl.modes)
        ns = np.diff(wl.offsets)
        Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
        idx = sample(ns, k, 1000 + cfg) + (CAPPED_144 if cfg == 5 else [])
        for i in idx:
            lp = approx.prob_approx(Q, list(rows[i]), order)
            out["cases"].append({"config": cfg, "order": order, "row": i, "n": int(ns[i]), "logp": lp,
                                 "capped_radius": cfg == 5 and i in CAPPED_144})
            print(cfg, order, i, int(ns[i]), lp, flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "big_rows.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
