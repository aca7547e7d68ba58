"""Oracle pins for simplicial meshes: volumes, centroid balls, point
location, tracking and whole transfers on jittered triangles/tetrahedra."""

import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import transfer as otr
from paper_1908_05834_amd import inputs


@pytest.mark.parametrize("jitter", [0.0, 0.1])
def test_tet_volumes_fill_the_cube(jitter):
    m = inputs.kuhn_tets(3, jitter=jitter, seed=7)
    vol = geo.simplex_volumes(m["vertices"], m["cells"])
    assert vol.size == 6 * 27 and np.all(vol > 0)
    assert abs(vol.sum() - 1.0) < 1e-14
    if jitter == 0.0:
        # every Kuhn tetrahedron of a cube of side h has volume h^3 / 6
        assert np.allclose(vol, (1.0 / 3) ** 3 / 6.0, rtol=0, atol=1e-16)


def test_triangle_areas_fill_the_square():
    m = inputs.triangulated_square(5, jitter=0.1, seed=3)
    area = geo.simplex_volumes(m["vertices"], m["cells"])
    assert np.all(area > 0) and abs(area.sum() - 1.0) < 1e-14


def test_volume_is_the_determinant():
    # against numpy's determinant of the edge matrix
    m = inputs.kuhn_tets(2, jitter=0.1, seed=11)
    V, C = m["vertices"], m["cells"]
    E = np.stack([V[C[:, i]] - V[C[:, 0]] for i in (1, 2, 3)], axis=1)
    ref = np.abs(np.linalg.det(E)) / 6.0
    assert np.allclose(geo.simplex_volumes(V, C), ref, rtol=1e-13, atol=0)


def test_equal_measure_balls():
    m = inputs.kuhn_tets(2, jitter=0.0, seed=0)
    c, r, cell = geo.simplex_ball_layout(m)
    h = 0.5
    # Kuhn tetrahedron: |B| = h^3/6 gives r = h (1 / (8 pi))^(1/3) = 0.341 h
    assert np.allclose(r, h * (1.0 / (8.0 * math.pi)) ** (1.0 / 3.0), rtol=1e-15)
    assert np.allclose(geo.ball_measure(r, 3), h ** 3 / 6.0, rtol=1e-14)
    assert np.array_equal(cell, np.arange(m["cells"].shape[0]))
    # centroid = vertex mean
    assert np.allclose(c, m["vertices"][m["cells"]].mean(axis=1), rtol=0, atol=1e-16)


def _barycentric_inside(mesh, cid, x, tol=1e-12):
    V = mesh["vertices"][mesh["cells"][cid]]
    A = np.vstack([V.T, np.ones(V.shape[0])])
    lam = np.linalg.solve(A, np.append(x, 1.0))
    return np.all(lam >= -tol)


@pytest.mark.parametrize("mk", ["tets", "tris"])
def test_point_location(mk):
    m = inputs.kuhn_tets(3, 0.1, 5) if mk == "tets" else inputs.triangulated_square(6, 0.1, 5)
    dim = m["vertices"].shape[1]
    rng = np.random.default_rng(1)
    X = rng.uniform(0.0, 1.0, size=(400, dim))
    cid = geo.locate_points(X, m)
    for x, k in zip(X, cid):
        assert _barycentric_inside(m, k, x)
    # the lowest-numbered containing cell: no lower cell contains the point
    # strictly inside
    V, C = m["vertices"], m["cells"]
    for x, k in zip(X[:60], cid[:60]):
        for j in range(k):
            Vj = V[C[j]]
            A = np.vstack([Vj.T, np.ones(dim + 1)])
            lam = np.linalg.solve(A, np.append(x, 1.0))
            assert not np.all(lam > 1e-12)
    # centroids lie in their own cell
    cen = geo.simplex_centroids(V, C)
    assert np.array_equal(geo.locate_points(cen, m), np.arange(C.shape[0]))


def test_tracking_matches_cartesian_with_constant_phi():
    # with phi constant the mesh only bounds the domain: tracking a point on
    # a simplicial mesh of the unit cube equals tracking on a Cartesian one
    tets = inputs.kuhn_tets(4, 0.1, 2)
    cart = inputs.cartesian_mesh((4, 4, 4))
    vel = inputs.sample_velocity_grid((4, 4, 4), lambda p, t: inputs.swirl_3d(p, t))
    X = np.random.default_rng(0).uniform(0, 1, size=(50, 3))
    a = geo.trace_points(X, tets, vel, 0.05)
    b = geo.trace_points(X, cart, vel, 0.05)
    assert np.array_equal(a, b)


def test_speed_uses_the_located_cell():
    nc = 6 * 27
    m = inputs.kuhn_tets(3, 0.1, 4, phi=inputs.lognormal_phi(nc, 9))
    vel = inputs.sample_velocity_grid((3, 3, 3), inputs.constant_field((1.0, -2.0, 0.5)))
    X = np.random.default_rng(3).uniform(0, 1, size=(40, 3))
    v = geo.speed(X, m, vel)
    cid = geo.locate_points(X, m)
    assert np.allclose(v, np.array([1.0, -2.0, 0.5])[None] / m["phi"][cid][:, None], rtol=1e-15)


@pytest.mark.parametrize("porous", [False, True])
def test_transfer_on_tets(porous):
    n = 3
    nc = 6 * n ** 3
    phi = inputs.lognormal_phi(nc, 21) if porous else None
    m = inputs.kuhn_tets(n, 0.1, 8, phi=phi)
    vel = inputs.sample_velocity_grid((n, n, n), lambda p, t: inputs.swirl_3d(p, t))
    T = otr.build_transfer(m, vel, 0.02, layout="equal_measure")
    b = T["b"]
    rp, col = T["row_ptr"], T["col"]
    rows = otr.csr_rows(rp)
    # V: rows hold |K|_phi (eq. ball_int shares sum to the tracked mass)
    rs = np.bincount(rows, weights=T["V"], minlength=nc)
    assert np.allclose(rs, b, rtol=1e-13, atol=0)
    # final A: both sums equal |K|_phi, constants kept, mass conserved
    A = T["A"]
    assert np.allclose(np.bincount(rows, weights=A, minlength=nc), b, rtol=0, atol=2e-13 * b.max())
    assert np.allclose(np.bincount(col, weights=A, minlength=nc), b, rtol=0, atol=2e-13 * b.max())
    c0 = inputs.uniform_c(m, 4)
    c1 = otr.apply(rp, col, A, b, c0)
    m0, m1 = otr.mass(m["phi"], T["cell_vol"], c0), otr.mass(m["phi"], T["cell_vol"], c1)
    assert abs(m1 - m0) <= 1e-13 * abs(m0)
    ones = otr.apply(rp, col, A, b, np.ones(nc))
    assert np.max(np.abs(ones - 1.0)) < 1e-12


def test_transfer_on_triangles():
    m = inputs.triangulated_square(8, 0.1, 6)
    nc = m["cells"].shape[0]
    vel = inputs.sample_velocity_grid((8, 8), inputs.rotation_stretch_2d)
    T = otr.build_transfer(m, vel, 0.2, layout="equal_measure")
    rows = otr.csr_rows(T["row_ptr"])
    assert np.allclose(np.bincount(rows, weights=T["V"], minlength=nc), T["b"], rtol=1e-13)
    A = T["A"]
    assert np.allclose(np.bincount(T["col"], weights=A, minlength=nc), T["b"], rtol=0,
                       atol=2e-13 * T["b"].max())


def test_cbrt_rounded_is_nearest():
    """The oracle's cube root is the double nearest to the real root:
    exact on perfect cubes, and a neighbour either side is farther (the
    cubes compared in rational arithmetic)."""
    from fractions import Fraction
    for k in (1.0, 8.0, 27.0, 0.125, 3.375):
        assert float(geo.cbrt_rounded(np.array([k]))[0]) ** 3 == pytest.approx(k, rel=0)
    ys = np.random.default_rng(4).uniform(1e-7, 1.0, 200)
    rs = geo.cbrt_rounded(ys)
    for y, r in zip(ys, rs):
        fy = Fraction(float(y))
        err = abs(Fraction(float(r)) ** 3 - fy)
        for nb in (np.nextafter(r, 0.0), np.nextafter(r, np.inf)):
            assert abs(Fraction(float(nb)) ** 3 - fy) >= err
