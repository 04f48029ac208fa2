"""Writes big_rows.json: log p-hat from the CPU oracle (power-series sectors,
max-entropy fits; see oracle/approx.py) for 26 sampled rows each (the smallest
and largest click counts and 24 seeded draws) of the 100-mode (order 3) and
144-mode (order 2) batches of workloads.py, and for five rows of
the 144-mode batch whose saddle-point radius lies beyond 0.98 of the
convergence radius (the GPU caps the contour radius there).  Calls only
oracle/ and workloads.py; run from the repository root (8 worker processes):

    python tests/golden/make_big_rows.py
"""
import json
import os
import sys
from multiprocessing import Pool

# one BLAS thread per worker: the oracle's fp64 series then rounds the same way
# on every run (threaded reductions change its last ~1e-10 of log p)
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import numpy as np  # noqa: E402

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


def one(job):
    cfg, order, i = job
    wl = make_workload(cfg)
    row = csr_rows(wl.offsets, wl.modes)[i]
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    return cfg, order, i, len(row), approx.prob_approx(Q, list(row), order)


def main():
    out = {"generator": "tests/golden/make_big_rows.py", "cases": []}
    jobs = []
    for cfg, order, k in ((4, 3, 24), (5, 2, 24)):
        ns = np.diff(make_workload(cfg).offsets)
        jobs += [(cfg, order, i) for i in sample(ns, k, 1000 + cfg) + (CAPPED_144 if cfg == 5 else [])]
    with Pool(8) as pool:
        for cfg, order, i, n, lp in pool.imap(one, jobs):
            out["cases"].append({"config": cfg, "order": order, "row": i, "n": n, "logp": lp,
                                 "capped_radius": cfg == 5 and i in CAPPED_144})
            print(cfg, order, i, n, lp, flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "big_rows.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
