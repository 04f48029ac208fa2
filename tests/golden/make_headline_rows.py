"""Writes headline_rows.json: the oracle's order-1 and order-2 log p-hat for
rows of the paper's headline case (Results, Approximation scheme; Fig. 1: 50
clicks of a lossless 70-mode device, every second input squeezed at r = 1.6;
workloads.accuracy_workload(70, 1.6, 50, P=16), rows 0 and 1), with every
cluster's sector weights in binary128 (oracle/sectors128.c).  For this pure
state the power series cancels strongly (measured: the |lambda| series
exceeds the signed one by 8e10 at the sector of largest order-1 weight and by
4e14 at that of order 2; the fp64 S_0 is wrong by O(1) between 50 and 400
photons); binary128 carries 33 digits, so at least 17 are left.  The record
holds, per case, that amplification, so that the digits left can be checked.  Calls only oracle/ and
workloads.py; run from the repository root (about ten minutes on 8 cores):

    python tests/golden/make_headline_rows.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import approx, model, sectors128  # noqa: E402
from workloads import accuracy_workload, csr_rows  # noqa: E402

CASES = [(0, 1), (1, 1), (0, 2)]   # (row, order)
L = 1024                           # S_0 falls below 1e-35 of its sum by kappa = 1000


def main():
    sectors128.build(force=True)
    hw = accuracy_workload(70, 1.6, 50, P=16)
    Q = model.q_matrix(model.covariance(hw.U, hw.r, hw.eta))
    rows = csr_rows(hw.offsets, hw.modes)
    out = []
    for row, order in CASES:
        C = list(rows[row])
        mom = lambda W, jp, LL: sectors128.cluster_moments(W, jp, LL, workers=8)  # noqa: E731
        lp, det = approx.prob_approx(Q, C, order, L0=L, return_detail=True, moments=mom, floor=1e-27)
        terms = det["terms"]
        kmax = max(terms, key=terms.get)
        amp = float(det["S0abs"][kmax] / det["S"][0, kmax])
        print(row, order, len(C), lp, "sector", kmax, "amplification", amp, "nfail", det["nfail"], flush=True)
        out.append({"row": row, "order": order, "n": len(C), "logp": lp, "top_sector": int(kmax),
                    "amplification": amp, "nfail": det["nfail"], "L": det["L"]})
    rec = {"generator": "tests/golden/make_headline_rows.py",
           "workload": "accuracy_workload(70, 1.6, 50, P=16)", "cases": out}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "headline_rows.json"), "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
