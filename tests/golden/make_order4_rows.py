"""Writes order4_rows.json: the oracle's fourth-order log p-hat (power-series
sectors, max-entropy fits with four moments; oracle/approx.py) for two rows of
more than 40 clicks (46 and 49) of the 100-mode batch of workloads.py.  (The
paper's own headline case, 50 clicks of a lossless 70-mode device, is out of
the fp64 power series' reach: for a pure state its terms cancel so strongly at
50 photons that every sector falls under the series' rounding floor.)  Calls
only oracle/ and workloads.py; run from the repository root (about fifteen
minutes):

    python tests/golden/make_order4_rows.py
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import approx, model  # noqa: E402
from workloads import csr_rows, make_workload  # noqa: E402

CONFIG = 4
ROWS = [1196, 7268]


def one(i):
    wl = make_workload(CONFIG)
    Q = model.q_matrix(model.covariance(wl.U, wl.r, wl.eta))
    C = list(csr_rows(wl.offsets, wl.modes)[i])
    lp = approx.prob_approx(Q, C, 4)
    print(i, len(C), lp, flush=True)
    return {"row": i, "n": len(C), "logp": lp}


def main():
    with ProcessPoolExecutor(max_workers=len(ROWS)) as ex:
        cases = list(ex.map(one, ROWS))
    rec = {"generator": "tests/golden/make_order4_rows.py", "config": CONFIG, "order": 4, "cases": cases}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "order4_rows.json"), "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
