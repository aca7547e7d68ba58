"""Writes tests/golden/batch47_step.npz: one step of problem 47 of the batch
workload (inputs.mixed_problem(47): a cube of 42^3 hexahedra, CFL 2.13, 8
sub-cell balls per cell) computed by the oracle alone, whose least-change
problem is solved on the relaxed box x >= -1 (Sec. 3.2, eq.
opti_masscons; the paper's box is empty here): the updated concentration
at 4,096 cells drawn with seed 47, the box level and the porous mass.  The
oracle takes about 90 s on one core.

    python tests/golden/make_batch47.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import transfer as otr  # noqa: E402
from paper_1908_05834_amd import inputs  # noqa: E402


def main():
    q = inputs.mixed_problem(47)
    T = otr.build_transfer(q["mesh"], q["vel"], q["dt"], layout=q["layout"])
    c1 = otr.apply(T["row_ptr"], T["col"], T["A"], T["b"], q["c0"])
    idx = np.sort(np.random.default_rng(47).choice(c1.size, 4096, replace=False))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch47_step.npz")
    np.savez_compressed(out, idx=idx, c1=c1[idx], qp_level=T["qp"]["level"],
                        nnz=T["col"].size, mass=otr.mass(q["mesh"]["phi"], T["cell_vol"], c1),
                        c1_max=np.max(np.abs(c1)))
    print(out, c1.size, T["qp"]["level"], T["col"].size)


if __name__ == "__main__":
    main()
