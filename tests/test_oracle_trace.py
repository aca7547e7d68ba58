"""Pins of the oracle's tracking: Q1 interpolation and backward RK4."""

import math

import numpy as np
import pytest

from oracle import geometry as geo
from paper_1908_05834_amd import inputs


def _mesh(n, phi=None):
    return inputs.cartesian_mesh(n, phi=phi)


def test_q1_reproduces_linear_field():
    mesh = _mesh((8, 8))
    vel = inputs.sample_velocity(mesh, inputs.solid_body_2d)
    rng = np.random.default_rng(0)
    p = rng.uniform(0.0, 1.0, (500, 2))
    got = geo.q1_interpolate(p, vel["m"], vel["origin"], vel["spacing"], vel["u"])
    np.testing.assert_allclose(got, inputs.solid_body_2d(p), rtol=0, atol=1e-14)


def test_q1_trilinear_exact_and_clamped():
    mesh = _mesh((4, 5, 6))

    def f(p, t=0.0):
        x, y, z = p[:, 0], p[:, 1], p[:, 2]
        return np.stack([1 + 2 * x + 3 * y + 4 * z + 5 * x * y * z, x * y - z, 2 * y * z], 1)
    vel = inputs.sample_velocity(mesh, f)
    rng = np.random.default_rng(1)
    p = rng.uniform(0.0, 1.0, (300, 3))
    got = geo.q1_interpolate(p, vel["m"], vel["origin"], vel["spacing"], vel["u"])
    np.testing.assert_allclose(got, f(p), rtol=0, atol=1e-13)
    # outside the box the query is clamped onto it
    q = np.array([[-0.5, 0.5, 0.5], [1.5, 2.0, -1.0]])
    got = geo.q1_interpolate(q, vel["m"], vel["origin"], vel["spacing"], vel["u"])
    np.testing.assert_allclose(got, f(np.clip(q, 0.0, 1.0)), atol=1e-13)


def test_rk4_solid_body_closed_form():
    """For v = w J (X - c), J = [[0,-1],[1,0]], one backward RK4 step of
    length dt is the degree-4 Taylor polynomial of exp(-w dt J):
    X' = c + [(1 - th^2/2 + th^4/24) I - (th - th^3/6) J](X - c), th = w dt."""
    mesh = _mesh((32, 32))
    vel = inputs.sample_velocity(mesh, inputs.solid_body_2d)
    dt = 0.01
    th = 2.0 * math.pi * dt
    J = np.array([[0.0, -1.0], [1.0, 0.0]])
    R = (1 - th ** 2 / 2 + th ** 4 / 24) * np.eye(2) - (th - th ** 3 / 6) * J
    rng = np.random.default_rng(2)
    X = rng.uniform(0.2, 0.8, (400, 2))
    got = geo.trace_points(X, mesh, vel, dt)
    want = 0.5 + (X - 0.5) @ R.T
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-15)


def test_constant_and_zero_velocity():
    mesh = _mesh((10, 10, 10))
    u = np.array([0.3, -0.2, 0.1])
    vel = inputs.sample_velocity(mesh, inputs.constant_field(u))
    rng = np.random.default_rng(3)
    X = rng.uniform(0.3, 0.7, (100, 3))
    np.testing.assert_allclose(geo.trace_points(X, mesh, vel, 0.5), X - 0.5 * u, atol=1e-15)
    vel0 = inputs.sample_velocity(mesh, inputs.constant_field(np.zeros(3)))
    assert np.array_equal(geo.trace_points(X, mesh, vel0, 0.5), X)


def test_clamped_to_domain():
    mesh = _mesh((10, 10))
    vel = inputs.sample_velocity(mesh, inputs.constant_field([1.0, 0.0]))
    X = np.array([[0.05, 0.5], [0.95, 0.5]])
    got = geo.trace_points(X, mesh, vel, 0.2)
    assert np.allclose(got, [[0.0, 0.5], [0.75, 0.5]])


def test_porosity_divides_speed():
    """v = u / phi: with phi = 2 everywhere the trace equals that of u over
    half the time step (eq. charac)."""
    mesh1 = _mesh((16, 16))
    mesh2 = _mesh((16, 16), phi=np.full(256, 2.0))
    vel = inputs.sample_velocity(mesh1, inputs.rotation_stretch_2d)
    rng = np.random.default_rng(4)
    X = rng.uniform(0.1, 0.9, (200, 2))
    np.testing.assert_allclose(geo.trace_points(X, mesh2, vel, 0.4),
                               geo.trace_points(X, mesh1, vel, 0.2), atol=1e-15)


def test_rk4_fourth_order():
    """On an affine field (reproduced exactly by Q1) the backward trace is
    the flow of a linear ODE, known in closed form via the matrix
    exponential; RK4 with m substeps must show error ratios near 2^4."""
    from scipy.linalg import expm
    A = np.array([[0.3, 0.8], [-0.6, 0.2]])
    bvec = np.array([-0.5, 0.2])

    def f(p, t=0.0):
        return p @ A.T + bvec
    mesh = _mesh((16, 16))
    vel = inputs.sample_velocity(mesh, f)
    rng = np.random.default_rng(5)
    X = rng.uniform(0.45, 0.55, (40, 2))
    dt = 0.6
    # dX/ds = -(A X + b): augmented linear system
    M = np.zeros((3, 3))
    M[:2, :2] = -A
    M[:2, 2] = -bvec
    E = expm(M * dt)
    exact = X @ E[:2, :2].T + E[:2, 2]
    errs = [np.max(np.abs(geo.trace_points(X, mesh, vel, dt, substeps=m) - exact))
            for m in (1, 2, 4)]
    assert 13.0 < errs[0] / errs[1] < 19.0
    assert 13.0 < errs[1] / errs[2] < 19.0


def test_tracked_radius_rules():
    # constant phi: r_hat = r exactly
    mesh = _mesh((8, 8))
    vel = inputs.sample_velocity(mesh, inputs.rotation_stretch_2d)
    C, r, cell = geo.ball_layout(mesh["n"], mesh["origin"], mesh["h"], "subcell")
    Ch = geo.trace_points(C, mesh, vel, 0.4)
    assert np.array_equal(geo.tracked_radius(C, r, Ch, mesh, vel, 0.4), r)
    # variable phi, but u = 0: every cardinal point stays at distance r
    mesh_v = _mesh((8, 8), phi=np.linspace(0.5, 1.0, 64))
    vel0 = inputs.sample_velocity(mesh_v, inputs.constant_field([0.0, 0.0]))
    rh = geo.tracked_radius(C, r, C, mesh_v, vel0, 0.4)
    np.testing.assert_allclose(rh, r, rtol=1e-15)
    # variable phi, constant u: a rigid shift inside one phi region keeps r
    mesh_c = _mesh((8, 8), phi=np.r_[np.full(32, 0.5), np.full(32, 1.0)])
    velc = inputs.sample_velocity(mesh_c, inputs.constant_field([0.1, 0.0]))
    C2 = np.array([[0.5, 0.2]])
    r2 = np.array([0.01])
    Ch2 = geo.trace_points(C2, mesh_c, velc, 0.5)
    np.testing.assert_allclose(geo.tracked_radius(C2, r2, Ch2, mesh_c, velc, 0.5), r2,
                               rtol=1e-12)
