"""Writes grad_rows.json: the reference gradient of L = sum_p w_p log p_hat_p
(order 2) with respect to r[144] and eta[144] for five rows of the 144-mode
batch of workloads.py (40 to 110 clicks; rows 1146 and 3675 have their
contour radius capped below the saddle point), by torch-CPU fp64 autograd
through the oracle (oracle/grad_ref.py).  Calls only oracle/ and workloads.py;
run from the repository root (a few minutes):

    python tests/golden/make_grad_rows.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import grad_ref  # noqa: E402
from workloads import csr_rows, make_workload  # noqa: E402

ROWS = [7, 1763, 1146, 3675, 3971]
WEIGHTS = [0.7, 1.3, 0.9, 1.1, 1.0]


def main():
    wl = make_workload(5)
    rows = csr_rows(wl.offsets, wl.modes)
    val, gr, ge = grad_ref.loss_and_grad(wl.U, wl.r, wl.eta, [rows[i] for i in ROWS], 2, WEIGHTS)
    rec = {"generator": "tests/golden/make_grad_rows.py", "config": 5, "order": 2, "rows": ROWS,
           "n": [int(len(rows[i])) for i in ROWS], "weights": WEIGHTS, "loss": val,
           "grad_r": gr.tolist(), "grad_eta": ge.tolist()}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_rows.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(val, np.abs(gr).max(), np.abs(ge).max())


if __name__ == "__main__":
    main()
