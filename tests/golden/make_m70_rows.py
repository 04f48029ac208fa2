"""Writes m70_rows.json: log p-hat from the CPU oracle (power-series sectors,
max-entropy fits; see oracle/approx.py) at order 3 for 104 rows of the
70-mode batch of workloads.py (10^4 patterns of 15-40 clicks): four rows of
every click count 15..40, chosen by a seeded draw.  Calls only oracle/ and
workloads.py; run from the repository root (8 worker processes):

    python tests/golden/make_m70_rows.py
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

PER_COUNT = 4


def pick():
    wl = make_workload(3)
    ns = np.diff(wl.offsets)
    rng = np.random.default_rng(70003)
    idx = []
    for k in range(int(ns.min()), int(ns.max()) + 1):
        rows_k = np.flatnonzero(ns == k)
        idx += sorted(int(i) for i in rng.choice(rows_k, size=min(PER_COUNT, len(rows_k)), replace=False))
    return wl, idx


def one(i):
    wl, _ = pick()
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    row = csr_rows(wl.offsets, wl.modes)[i]
    return i, len(row), approx.prob_approx(Q, list(row), 3)


def main():
    _, idx = pick()
    with Pool(8) as pool:
        res = pool.map(one, idx)
    out = {"generator": "tests/golden/make_m70_rows.py", "config": 3, "order": 3,
           "cases": [{"row": i, "n": n, "logp": lp} for i, n, lp in res]}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "m70_rows.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(len(res), "rows")


if __name__ == "__main__":
    main()
