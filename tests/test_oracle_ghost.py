"""Pins of the oracle's ghost cells (Sec. 3.2, Remark on inflow and
outflow, option b): the paper's translation test (Sec. 4.1, test case 1),
whose exact solution is the translated block, against the errors the paper
prints for B-char; the interior mass balance of an outflow; and the
identity the closed-box constraints force on a translation without ghost
cells."""

import json
import math
import os

import numpy as np
import pytest

from oracle import transfer as otr
from paper_1908_05834_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _grid(n, g):
    """n x n interior cells of the unit square plus g ghost layers."""
    h = 1.0 / n
    return inputs.cartesian_mesh((n + 2 * g, n + 2 * g), length=h * (n + 2 * g),
                                 origin=(-g * h, -g * h))


def _block(n, g, x0, x1, y0, y1):
    """1 on interior cells whose centroid lies in [x0, x1] x [y0, y1]."""
    mesh = _grid(n, g)
    cen = inputs.cell_centroids(mesh)
    inside = (cen[:, 0] > x0) & (cen[:, 0] < x1) & (cen[:, 1] > y0) & (cen[:, 1] < y1)
    return inside.astype(np.float64)


def _translate(n, dt, g, steps=None):
    mesh = _grid(n, g)
    vel = inputs.sample_velocity(mesh, inputs.constant_field((1.0 / 16.0, 0.0)))
    T = otr.build_transfer(mesh, vel, dt, layout="subcell", n_ghost=g)
    c = _block(n, g, 1 / 16, 5 / 16, 1 / 16, 5 / 16)
    ghost = T["ghost"] if g else np.zeros(c.size, dtype=bool)
    m0 = otr.mass(mesh["phi"], T["cell_vol"], c, ~ghost)
    k = int(round(8.0 / dt)) if steps is None else steps
    for _ in range(k):
        c = otr.apply(T["row_ptr"], T["col"], T["A"], T["b"], c)
        c[ghost] = 0.0                      # inflow data: clean water
    return mesh, T, c, ghost, m0


@pytest.mark.parametrize("row", json.load(open(os.path.join(HERE, "golden",
                                                             "tc1_translation_errors.json")))
                         ["rows"])
def test_translation_with_ghost_cells(row):
    """The block moves to [9/16, 13/16] x [1/16, 5/16], and the relative L1
    / L2 errors of the cell values against the exact block are the ones the
    paper prints for B-char on 16^2, 32^2 and 64^2 (4 balls per square, one
    layer of ghost cells), to within one unit of the last printed digit."""
    n, dt = row["n"], row["dt"]
    mesh, T, c, ghost, m0 = _translate(n, dt, 1)
    exact = _block(n, 1, 9 / 16, 13 / 16, 1 / 16, 5 / 16)
    vol = T["cell_vol"]
    act = ~ghost
    e1 = np.sum(vol[act] * np.abs(c - exact)[act]) / np.sum(vol[act] * exact[act])
    e2 = math.sqrt(np.sum(vol[act] * ((c - exact) ** 2)[act])
                   / np.sum(vol[act] * exact[act] ** 2))
    cen = inputs.cell_centroids(mesh)
    cx = np.sum(vol[act] * c[act] * cen[act, 0]) / np.sum(vol[act] * c[act])
    assert abs(cx - 11 / 16) < 0.02                 # moved by 0.5
    assert abs(e1 - row["E1"]) <= 1.5e-5, e1
    assert abs(e2 - row["E2"]) <= 1.5e-5, e2
    # the block has not reached the outflow: the interior mass is kept
    m1 = otr.mass(mesh["phi"], vol, c, act)
    assert abs(m1 - m0) <= 1e-12 * m0


def test_translation_errors_fall_with_refinement():
    errs = []
    for n, dt in ((16, 0.8), (32, 0.4)):
        mesh, T, c, ghost, _ = _translate(n, dt, 1)
        exact = _block(n, 1, 9 / 16, 13 / 16, 1 / 16, 5 / 16)
        act = ~ghost
        errs.append(np.sum(np.abs(c - exact)[act]) / np.sum(exact[act]))
    assert errs[1] < errs[0]


def test_outflow_interior_mass_balance():
    """A block leaving through the right wall: the interior mass falls by
    exactly what the ghost rows take from interior columns (the interior
    columns still hold their whole porous volume), step by step."""
    n, dt, g = 16, 0.8, 1
    mesh = _grid(n, g)
    vel = inputs.sample_velocity(mesh, inputs.constant_field((1.0 / 16.0, 0.0)))
    T = otr.build_transfer(mesh, vel, dt, layout="subcell", n_ghost=g)
    ghost = T["ghost"]
    act = ~ghost
    rows = otr.csr_rows(T["row_ptr"])
    col = T["col"]
    A = T["A"]
    vol = T["cell_vol"]
    # interior columns keep their porous volume; interior rows their targets
    cs = np.bincount(col, weights=A, minlength=vol.size)
    rs = np.bincount(rows, weights=A, minlength=vol.size)
    assert np.max(np.abs(cs - T["b"])[act]) <= 1e-13 * T["b"].max()
    assert np.max(np.abs(rs - T["b"])[act]) <= 1e-13 * T["b"].max()
    c = _block(n, g, 12 / 16, 15.5 / 16, 6 / 16, 10 / 16)
    for _ in range(4):
        m0 = otr.mass(mesh["phi"], vol, c, act)
        out = np.sum(A[ghost[rows] & act[col]] * c[col[ghost[rows] & act[col]]])
        inn = np.sum(A[act[rows] & ghost[col]] * c[col[act[rows] & ghost[col]]])
        c = otr.apply(T["row_ptr"], T["col"], T["A"], T["b"], c)
        c[ghost] = 0.0
        m1 = otr.mass(mesh["phi"], vol, c, act)
        assert abs((m1 - m0) - (inn - out)) <= 1e-13 * m0
    assert out > 0.0


def test_translation_without_ghost_cells_is_held_still():
    """Without ghost cells every constraint is kept and each horizontal
    chain of cells must map onto itself: the least-change transfer of a
    translation through the walls is the identity (Sec. 3.2, Remark on
    inflow and outflow, is what removes this)."""
    n, dt = 16, 0.8
    mesh = inputs.cartesian_mesh((n, n))
    vel = inputs.sample_velocity(mesh, inputs.constant_field((1.0 / 16.0, 0.0)))
    T = otr.build_transfer(mesh, vel, dt, layout="subcell")
    rows = otr.csr_rows(T["row_ptr"])
    off = rows != T["col"]
    assert np.max(np.abs(T["A"][off])) <= 1e-12 * T["b"].max()
