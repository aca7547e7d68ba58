"""Writes tests/golden/batch_hard_feasibility.json: for two problems of the
batch workload (inputs.mixed_problem 229 and 55: hexahedral cubes of 52^3
and 49^3 cells at CFL 0.52 and 1.26) whose least-change problem is hard to
solve to the tolerance, whether the paper's box 0 <= 1 + x <= 2 (level 0)
and the relaxed box x >= -1 (level 1) admit a solution, decided by the
oracle's feasibility LP on the oracle's own A^(N) (Sec. 3.2, eq.
opti_masscons; the relaxation levels follow the paper's remark on an empty
box).  Takes several minutes per problem and level on one core.

    python tests/golden/make_batch_hard.py
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import qp as oqp  # noqa: E402
from oracle import transfer as otr  # noqa: E402
from paper_1908_05834_amd import inputs  # noqa: E402


def main():
    out = {}
    for p in (229, 55):
        q = inputs.mixed_problem(p)
        T = otr.build_transfer(q["mesh"], q["vel"], q["dt"], layout=q["layout"],
                               stop_after="sinkhorn")
        rows = otr.csr_rows(T["row_ptr"])
        b = T["b"]
        scale = float(np.max(np.abs(b)))
        rec = {"name": q["name"], "cells": int(b.size), "nnz": int(T["col"].size)}
        for level in (0, 1):
            lo, hi = oqp.BOX_LEVELS[level]
            t0 = time.time()
            feas, slack = oqp.feasible_lp(rows, T["col"], T["AN"] / scale, b / scale, b / scale,
                                          lo, hi)
            rec[f"level{level}_feasible"] = bool(feas)
            rec[f"level{level}_slack"] = float(slack)
            print(p, level, feas, slack, f"{time.time() - t0:.1f} s", flush=True)
            if feas:
                break
        out[str(p)] = rec
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "batch_hard_feasibility.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path)


if __name__ == "__main__":
    main()
