"""Pins of the oracle's ball-intersection measure (disk lens, sphere lens).

The oracle writes the lens as two circular segments / spherical caps cut by
the radical line / plane.  These tests pin it to facts that do not depend
on that construction: special values, the derivative of the overlap with
respect to the centre distance (minus the chord length in 2D, minus the
area of the intersection disk in 3D), symmetry, and Monte Carlo.
"""

import math

import numpy as np
import pytest

from oracle import geometry as geo


@pytest.mark.parametrize("dim", [2, 3])
def test_disjoint_and_contained(dim):
    r1, r2 = 0.3, 0.2
    assert geo.lens_measure(r1, r2, 0.5, dim) == 0.0          # tangent from outside
    assert geo.lens_measure(r1, r2, 0.7, dim) == 0.0
    full = math.pi * r2 ** 2 if dim == 2 else 4.0 / 3.0 * math.pi * r2 ** 3
    assert geo.lens_measure(r1, r2, 0.0, dim) == pytest.approx(full, rel=1e-15)
    assert geo.lens_measure(r1, r2, 0.1, dim) == pytest.approx(full, rel=1e-15)  # internal tangency
    assert geo.lens_measure(r1, r2, 0.05, dim) == pytest.approx(full, rel=1e-15)


def test_equal_radii_half_distance_2d():
    # two unit-spaced circles through each other's centres: r^2 (2pi/3 - sqrt(3)/2)
    for r in (1.0, 0.25, 3.0e-3):
        want = r * r * (2.0 * math.pi / 3.0 - math.sqrt(3.0) / 2.0)
        assert geo.disk_lens_area(r, r, r) == pytest.approx(want, rel=4e-15)


def test_equal_radii_half_distance_3d():
    # two spheres through each other's centres: 5 pi r^3 / 12
    for r in (1.0, 0.25, 3.0e-3):
        assert geo.sphere_lens_volume(r, r, r) == pytest.approx(5.0 * math.pi * r ** 3 / 12.0,
                                                                rel=4e-15)


def _half_chord(r1, r2, d):
    t1 = (d * d + r1 * r1 - r2 * r2) / (2.0 * d)
    return math.sqrt(r1 * r1 - t1 * t1)


@pytest.mark.parametrize("r1,r2,d", [(1.0, 1.0, 1.3), (1.0, 0.6, 0.9), (0.4, 1.0, 1.1),
                                     (1.0, 0.7, 0.45), (0.25, 0.25, 0.2)])
def test_derivative_identity(r1, r2, d):
    """d|lens|/dd = -(chord length) in 2D and -(pi rho^2) in 3D, rho the
    radius of the circle where the two spheres meet."""
    eps = 1e-6
    rho = _half_chord(r1, r2, d)
    dA = (geo.disk_lens_area(r1, r2, d + eps) - geo.disk_lens_area(r1, r2, d - eps)) / (2 * eps)
    assert dA == pytest.approx(-2.0 * rho, rel=1e-7)
    dV = (geo.sphere_lens_volume(r1, r2, d + eps)
          - geo.sphere_lens_volume(r1, r2, d - eps)) / (2 * eps)
    assert dV == pytest.approx(-math.pi * rho * rho, rel=1e-7)


def test_symmetry():
    rng = np.random.default_rng(1)
    r1 = rng.uniform(0.1, 1.0, 200)
    r2 = rng.uniform(0.1, 1.0, 200)
    d = rng.uniform(0.0, 2.0, 200)
    for dim in (2, 3):
        a = geo.lens_measure(r1, r2, d, dim)
        b = geo.lens_measure(r2, r1, d, dim)
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("r1,r2,d", [(0.5, 0.5, 0.6), (0.5, 0.3, 0.55), (0.5, 0.3, 0.3)])
def test_monte_carlo(dim, r1, r2, d):
    rng = np.random.default_rng(1908 + dim)
    n = 2_000_000
    lo = np.array([-r1] + [-r1] * (dim - 1))
    hi = np.array([max(r1, d + r2)] + [r1] * (dim - 1))
    box = float(np.prod(hi - lo))
    hits = 0
    for _ in range(2):
        p = rng.uniform(lo, hi, size=(n, dim))
        in1 = np.sum(p * p, axis=1) < r1 * r1
        q = p.copy()
        q[:, 0] -= d
        in2 = np.sum(q * q, axis=1) < r2 * r2
        hits += int(np.count_nonzero(in1 & in2))
    frac = hits / (2 * n)
    est = frac * box
    sigma = math.sqrt(frac * (1 - frac) / (2 * n)) * box
    assert abs(est - geo.lens_measure(r1, r2, d, dim)) < 4.0 * sigma + 1e-12


def test_ball_measure():
    assert geo.ball_measure(2.0, 2) == pytest.approx(4.0 * math.pi)
    assert geo.ball_measure(2.0, 3) == pytest.approx(32.0 * math.pi / 3.0)
