"""Pins of the oracle's weighting, update direction and tracked radius.

Each test fixes a value by hand or by a closed form that a misreading of
the paper changes:

* the weight of a residing ball in eq. fracMaterial is rho_M phi_M times the
  lens (Sec. 3.1, Remark porousBallInt), and the mass carried by a tracked
  ball is rho_K phi_K |B_{K,s}| (eqs. expPhiB and volTracked);
* the update of eq. phys-inter-ELLAM gathers from the residing cells into
  the tracked cell (row K of the transfer), so that material moves with
  +u: a bump under a solid-body rotation turns the way the exact flow does;
* the tracked radius of eq. rTrackedBall is the arithmetic mean of the 2d
  distances from the tracked centre to the tracked cardinal points, which
  one RK4 step on a linear field gives in closed form.
"""

import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import transfer as otr
from paper_1908_05834_amd import inputs


# ---------------------------------------------------------------- eq. fracMaterial


@pytest.mark.parametrize("dim", [2, 3])
def test_v_weights_by_residing_porous_density(dim):
    """Two cells with one ball each, r = 1/4, residing centres 1/2 apart
    along x.  The tracked ball of cell 0 sits half way between them, so its
    two lenses are equal (centre distance r); the tracked ball of cell 1 sits
    on its own residing ball (full overlap) and touches ball 0 (not a
    candidate).  With the lenses equal, the split of cell 0's mass follows
    rho_M phi_M alone: 1.5 : 0.5."""
    r = 0.25
    pad = (0.5,) * (dim - 1)
    centres = np.array([(0.25,) + pad, (0.75,) + pad])
    radii = np.array([r, r])
    traced = np.array([(0.5,) + pad, (0.75,) + pad])
    r_hat = radii.copy()
    ball_cell = np.array([0, 1])
    rho = np.array([1.5, 2.0])
    phi = np.array([1.0, 0.25])
    ia, ib = geo.candidate_pairs(traced, r_hat, centres, radii)
    assert list(zip(ia.tolist(), ib.tolist())) == [(0, 0), (0, 1), (1, 1)]
    rp, col, V = otr.initial_volumes(2, dim, ball_cell, centres, radii, rho, phi,
                                     traced, r_hat, ia, ib)
    ball = math.pi * r * r if dim == 2 else 4.0 / 3.0 * math.pi * r ** 3
    # rho_K phi_K |B|: 1.5 |B| for cell 0, 0.5 |B| for cell 1
    m0, m1 = 1.5 * ball, 0.5 * ball
    # weights rho_M phi_M: 1.5 (cell 0) and 2.0 * 0.25 = 0.5 (cell 1)
    want = {(0, 0): m0 * 1.5 / 2.0, (0, 1): m0 * 0.5 / 2.0, (1, 1): m1}
    got = {(i, int(c)): v for i in range(2) for c, v in
           zip(col[rp[i]:rp[i + 1]], V[rp[i]:rp[i + 1]])}
    assert set(got) == set(want)
    for k in want:
        assert got[k] == pytest.approx(want[k], rel=1e-15, abs=0)


def test_v_weights_with_unequal_lenses():
    """The same two cells in 3D with the tracked ball of cell 0 at distance
    r from residing ball 0 (lens 5 pi r^3 / 12) and at distance 0 from a
    smaller residing ball 1 of radius r/2 (lens = that whole ball,
    pi r^3 / 6): the shares follow rho_M phi_M |lens|."""
    r = 0.25
    centres = np.array([[0.25, 0.5, 0.5], [0.5, 0.5, 0.5]])
    radii = np.array([r, r / 2])
    traced = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    r_hat = np.array([r, r / 2])
    ia, ib = geo.candidate_pairs(traced, r_hat, centres, radii)
    rho = np.array([1.5, 2.0])
    phi = np.array([1.0, 0.25])
    rp, col, V = otr.initial_volumes(2, 3, np.array([0, 1]), centres, radii, rho, phi,
                                     traced, r_hat, ia, ib)
    lens0 = 5.0 * math.pi * r ** 3 / 12.0
    lens1 = 4.0 / 3.0 * math.pi * (r / 2) ** 3
    w0, w1 = 1.5 * lens0, 0.5 * lens1
    m0 = 1.5 * 4.0 / 3.0 * math.pi * r ** 3
    assert col[rp[0]:rp[1]].tolist() == [0, 1]
    assert V[rp[0]] == pytest.approx(m0 * w0 / (w0 + w1), rel=1e-14)
    assert V[rp[0] + 1] == pytest.approx(m0 * w1 / (w0 + w1), rel=1e-14)


# ---------------------------------------------------------------- eq. phys-inter-ELLAM


def test_update_moves_material_with_the_flow():
    """Solid-body rotation u = 2 pi (-(y - 1/2), x - 1/2) on 24 x 24 cells
    (2 x 2 sub-cell balls), a disk of material at (1/2, 3/4), dt = 0.01:
    after 10 steps the exact flow has turned it by 36 degrees
    counter-clockwise.  The porous-mass-weighted centroid of c follows the
    exact rotation of the initial centroid to half a cell; the
    mirror motion (the transposed transfer) would land it 0.29 away."""
    n = 24
    mesh = inputs.cartesian_mesh((n, n))
    vel = inputs.sample_velocity(mesh, inputs.solid_body_2d)
    dt, steps = 0.01, 10
    cen = inputs.cell_centroids(mesh)
    c = inputs.disk_indicator(mesh, (0.5, 0.75), 0.15)
    T = otr.build_transfer(mesh, vel, dt, layout="subcell")
    x0 = (c[:, None] * cen).sum(0) / c.sum()
    for _ in range(steps):
        c = otr.apply(T["row_ptr"], T["col"], T["A"], T["b"], c)
    x1 = (c[:, None] * cen).sum(0) / c.sum()
    th = 2.0 * math.pi * dt * steps
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    want = R @ (x0 - 0.5) + 0.5
    assert np.linalg.norm(x1 - want) < 0.5 / n, (x1, want)
    mirror = np.array([1.0 - want[0], want[1]])
    assert np.linalg.norm(x1 - mirror) > 0.25


# ---------------------------------------------------------------- eq. rTrackedBall


def _rk4_factor(z):
    """Amplification of one classical RK4 step on y' = lambda y, z = lambda tau."""
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


@pytest.mark.parametrize("dim", [2, 3])
def test_tracked_radius_is_mean_cardinal_distance(dim):
    """Linear stagnation-point flow u = alpha (x - 1/2, -(y - 1/2)) in 2D,
    alpha (x - 1/2, -(y - 1/2)/2, -(z - 1/2)/2) in 3D (divergence free),
    with phi = 1 except one corner cell (phi not constant, so the cardinal
    points are tracked).  The nodal interpolant reproduces the field, and
    one backward RK4 step of length tau maps a displacement along axis a
    from the stagnation point by the factor P(-lambda_a tau), P the RK4
    polynomial.  So the cardinal points C +- r e_a end at distance
    r P(-lambda_a tau) from the tracked centre, and r_hat is their mean."""
    n = 16
    alpha, dt = 1.0, 0.1
    phi = np.ones(n ** dim)
    phi[0] = 0.5
    mesh = inputs.cartesian_mesh((n,) * dim, phi=phi)
    lam = [alpha] + [-alpha / (dim - 1)] * (dim - 1)

    def field(p, t=0.0):
        return np.stack([lam[a] * (p[:, a] - 0.5) for a in range(dim)], axis=1)

    vel = inputs.sample_velocity(mesh, field)
    C, r, _ = geo.ball_layout(mesh["n"], mesh["origin"], mesh["h"], "subcell")
    keep = np.all(np.abs(C - 0.5) < 0.2, axis=1)
    C, r = C[keep], r[keep]
    traced = geo.trace_points(C, mesh, vel, dt)
    f = [_rk4_factor(-lam[a] * dt) for a in range(dim)]
    np.testing.assert_allclose(traced - 0.5, (C - 0.5) * np.array(f), rtol=1e-12, atol=1e-15)
    r_hat = geo.tracked_radius(C, r, traced, mesh, vel, dt)
    want = r * sum(2.0 * fa for fa in f) / (2 * dim)
    np.testing.assert_allclose(r_hat, want, rtol=1e-12)
    # the mean differs from the largest distance by several per cent
    assert np.all(np.abs(r_hat - r * max(f)) > 0.01 * r)
