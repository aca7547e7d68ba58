"""Writes tests/golden/cswirl32_step.npz: the first step of the
non-solenoidal swirl on 32^3 hexahedra (inputs.compressible_swirl_hex(32,
squeeze=0.1), 8 sub-cell balls per cell, dt = 1/128, the row targets of
eq. volTracked; Sec. 3.2, Remark on non-solenoidal fields) computed by the
oracle alone, whose least-change problem is solved on the relaxed box
x >= -1 (the paper's box is empty): the updated concentration at 4,096
cells drawn with seed 32, the box level and the porous mass.  The oracle
takes about half an hour on one core.

    python tests/golden/make_cswirl32.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import transfer as otr  # noqa: E402
from paper_1908_05834_amd import inputs  # noqa: E402


def main():
    w = inputs.compressible_swirl_hex(32, squeeze=0.1)
    T = otr.build_transfer(w["mesh"], w["vel_fn"](0), w["dt"], layout="subcell",
                           solenoidal=False)
    c0 = np.asarray(w["c0"], dtype=np.float64)
    c1 = otr.apply(T["row_ptr"], T["col"], T["A"], T["b"], c0)
    idx = np.sort(np.random.default_rng(32).choice(c1.size, 4096, replace=False))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cswirl32_step.npz")
    np.savez_compressed(out, idx=idx, c1=c1[idx], qp_level=T["qp"]["level"],
                        nnz=T["col"].size, mass=otr.mass(w["mesh"]["phi"], T["cell_vol"], c1),
                        c1_max=np.max(np.abs(c1)))
    print(out, c1.size, T["qp"]["level"], T["col"].size)


if __name__ == "__main__":
    main()
