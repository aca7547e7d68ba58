"""Pins of whole oracle steps: conservation, constants, maximum principle,
mass summation, and an accuracy sanity check on a case with an exact
solution (not a parity pin: the paper does not fix its ball positions)."""

import math

import numpy as np
import pytest

from oracle import transfer as otr
from paper_1908_05834_amd import inputs


def _checks(T, c0, nc):
    rows = otr.csr_rows(T["row_ptr"])
    A = T["A"]
    b = T["b"]
    # local and global constraints (eqs. localmassconsMat / globalmassconsMat)
    np.testing.assert_allclose(np.bincount(rows, weights=A, minlength=nc), b, rtol=2e-14)
    np.testing.assert_allclose(np.bincount(T["col"], weights=A, minlength=nc), b, rtol=2e-14)
    # constants are preserved
    one = otr.apply(T["row_ptr"], T["col"], A, b, np.ones(nc))
    assert np.max(np.abs(one - 1.0)) < 1e-13
    # mass is conserved
    c1 = otr.apply(T["row_ptr"], T["col"], A, b, c0)
    phi = b / T["cell_vol"]
    m0 = otr.mass(phi, T["cell_vol"], c0)
    m1 = otr.mass(phi, T["cell_vol"], c1)
    assert abs(m1 - m0) <= 1e-12 * abs(m0)
    if T["qp"]["level"] <= 1:
        assert np.all(A >= 0)
        assert c1.min() >= c0.min() - 1e-13 and c1.max() <= c0.max() + 1e-13
    return c1


@pytest.mark.parametrize("layout", ["subcell", "inscribed", "equal_measure"])
def test_step_2d_rotation_stretch(layout):
    mesh = inputs.cartesian_mesh((16, 16))
    vel = inputs.sample_velocity(mesh, inputs.rotation_stretch_2d)
    T = otr.build_transfer(mesh, vel, 0.8, layout=layout)
    c0 = inputs.uniform_c(mesh, 1)
    _checks(T, c0, 256)


def test_step_3d_swirl_subcell():
    w = inputs.swirl_hex(8)
    T = otr.build_transfer(w["mesh"], w["vel_fn"](0), 0.05, layout="subcell")
    assert T["qp"]["level"] == 0
    _checks(T, w["c0"] + inputs.uniform_c(w["mesh"], 2), 512)


def test_step_variable_porosity():
    n = (12, 12)
    phi = inputs.lognormal_phi(144, 5834)
    mesh = inputs.cartesian_mesh(n, phi=phi)
    vel = inputs.sample_velocity(mesh, inputs.rotation_stretch_2d)
    T = otr.build_transfer(mesh, vel, 0.6, layout="subcell")
    assert not np.allclose(T["r_hat"], T["radii"])
    _checks(T, inputs.uniform_c(mesh, 3), 144)


def test_solid_body_workload_levels():
    w = inputs.solid_body_32()
    T = otr.build_transfer(w["mesh"], w["vel_fn"](0), w["dt"], layout="equal_measure")
    assert T["qp"]["level"] >= 1          # the paper's box cannot hold (inflow/outflow)
    _checks(T, w["c0"], 1024)


def test_mass_is_correctly_rounded():
    rng = np.random.default_rng(0)
    c = rng.uniform(0, 1, 10000) * 10.0 ** rng.integers(-8, 8, 10000)
    phi = rng.uniform(0.05, 1.0, 10000)
    exact = sum(map(lambda t: __import__("fractions").Fraction(t),
                    (phi * 0.5 * c).tolist()))
    assert otr.mass(phi, 0.5, c) == float(exact)


def test_reversing_flow_returns_sanity():
    """2D deformation field (zero normal velocity on the walls) that
    reverses at T/2: after T the exact solution is c^0 again.  B-char
    smears the bump but must bring it back near its start: the relative L1
    error stays well below that of a bump that did not come back, and well
    below 1 (accuracy sanity, not a parity pin)."""
    mesh = inputs.cartesian_mesh((32, 32))
    x = inputs.cell_centroids(mesh)
    r = np.minimum(4.0 * np.sqrt((x[:, 0] - 0.35) ** 2 + (x[:, 1] - 0.5) ** 2), 1.0)
    c0 = 0.5 * (1.0 + np.cos(math.pi * r))
    steps, T = 16, 1.0
    dt = T / steps
    c = c0.copy()
    for k in range(steps):
        vel = inputs.sample_velocity(
            mesh, lambda p, t: inputs.deformation_2d(p, t, period=T), (k + 0.5) * dt)
        Tr = otr.build_transfer(mesh, vel, dt, layout="subcell")
        c = otr.apply(Tr["row_ptr"], Tr["col"], Tr["A"], Tr["b"], c)
    e1 = np.sum(np.abs(c - c0)) / np.sum(np.abs(c0))
    assert e1 < 0.5
    assert abs(c.sum() - c0.sum()) < 1e-12 * c0.sum()
