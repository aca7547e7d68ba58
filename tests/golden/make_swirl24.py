"""Writes tests/golden/swirl24_step.npz: one step of the 3D swirl on 24^3
hexahedra (8 sub-cell balls per cell, phi = 1, dt = 1/128, the field of the
fourth interval) computed by the oracle alone, applied to c^0 ~ U[0,1]
(seed 11).  The oracle's least-change solve takes about 80 s at this size,
too long to repeat inside a GPU test; at 32^3 it did not finish in 20
minutes.

    python tests/golden/make_swirl24.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import transfer as otr  # noqa: E402
from paper_1908_05834_amd import inputs  # noqa: E402


def main():
    w = inputs.swirl_hex(24)
    T = otr.build_transfer(w["mesh"], w["vel_fn"](3), w["dt"], layout="subcell")
    c0 = inputs.uniform_c(w["mesh"], 11)
    c1 = otr.apply(T["row_ptr"], T["col"], T["A"], T["b"], c0)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "swirl24_step.npz")
    np.savez_compressed(out, c1=c1, qp_level=T["qp"]["level"], nnz=T["col"].size,
                        mass=otr.mass(w["mesh"]["phi"], T["cell_vol"], c1))
    print(out, c1.size, T["qp"]["level"], T["col"].size)


if __name__ == "__main__":
    main()
