"""Pins of the oracle's non-solenoidal step (Sec. 3.2, Remark on
non-solenoidal fields): the divergence of the Q1 interpolant, the
Liouville growth of a tracked ball (the analogue of eq. expPhiB), the row
targets of eq. volTracked, and one whole step, against closed forms and an
independent ODE integrator."""

import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import geometry as geo
from oracle import transfer as otr
from paper_1908_05834_amd import inputs


def _lattice(dim, field, m=(9, 7, 6), origin=(0.2, -0.1, 0.3), spacing=(0.05, 0.08, 0.07)):
    m, origin, spacing = m[:dim], origin[:dim], spacing[:dim]
    pts = inputs.lattice_nodes(m, origin, spacing)
    u = np.ascontiguousarray(np.asarray(field(pts), dtype=np.float64).T)
    return {"m": m, "origin": origin, "spacing": spacing, "u": u}


def _inside(dim, n, seed, lat):
    rng = np.random.default_rng(seed)
    lo = np.asarray(lat["origin"])
    hi = lo + (np.asarray(lat["m"]) - 1) * np.asarray(lat["spacing"])
    return lo + (hi - lo) * rng.uniform(0.02, 0.98, size=(n, dim))


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_divergence_of_multilinear_field(dim):
    """A multilinear field is its own Q1 interpolant: the divergence of the
    interpolant is the field's, at every point (non-unit spacing and an
    offset origin, so that a dropped 1/spacing or a wrong axis fails)."""
    rng = np.random.default_rng(7 + dim)
    # u_a = sum over subsets S of the axes of c[a, S] prod_{b in S} x_b
    subsets = list(range(2 ** dim))
    c = rng.standard_normal((dim, len(subsets)))

    def field(p):
        out = np.zeros_like(p)
        for a in range(dim):
            for S in subsets:
                term = np.full(p.shape[0], c[a, S])
                for b in range(dim):
                    if (S >> b) & 1:
                        term = term * p[:, b]
                out[:, a] += term
        return out

    def div_exact(p):
        d = np.zeros(p.shape[0])
        for a in range(dim):
            for S in subsets:
                if not (S >> a) & 1:
                    continue
                term = np.full(p.shape[0], c[a, S])
                for b in range(dim):
                    if b != a and (S >> b) & 1:
                        term = term * p[:, b]
                d += term
        return d

    lat = _lattice(dim, field)
    pts = _inside(dim, 500, 3, lat)
    got = geo.q1_divergence(pts, lat["m"], lat["origin"], lat["spacing"], lat["u"])
    want = div_exact(pts)
    assert np.max(np.abs(got - want)) <= 1e-11 * (1 + np.max(np.abs(want)))
    # and the interpolant itself agrees with the field (same lattice)
    v = geo.q1_interpolate(pts, lat["m"], lat["origin"], lat["spacing"], lat["u"])
    assert np.max(np.abs(v - field(pts))) <= 1e-12 * (1 + np.max(np.abs(v)))


def _linear_mesh(dim, phi):
    n = (10,) * dim
    mesh = inputs.cartesian_mesh(n, phi=np.full(int(np.prod(n)), phi))
    return mesh


@pytest.mark.parametrize("dim,phi,substeps", [(2, 1.0, 1), (2, 0.4, 3), (3, 1.0, 1),
                                              (3, 0.7, 2)])
def test_log_growth_of_linear_field_is_exact(dim, phi, substeps):
    """u = A (x - x0) has div u = tr A everywhere: the porous volume of any
    carried region scales by exp(-tr(A) dt / phi) over a backward step
    (Liouville), and RK4 integrates the constant rate exactly."""
    rng = np.random.default_rng(11 * dim + substeps)
    A = 0.6 * rng.standard_normal((dim, dim))
    x0 = np.full(dim, 0.5)
    mesh = _linear_mesh(dim, phi)
    vel = inputs.sample_velocity(mesh, lambda p, t=0.0: (p - x0) @ A.T)
    pts = 0.3 + 0.4 * rng.uniform(size=(200, dim))
    dt = 0.05
    X, lam = geo.log_growth(pts, mesh, vel, dt, substeps)
    want = -np.trace(A) * dt / phi
    assert np.max(np.abs(lam - want)) <= 1e-14 * max(1.0, abs(want)) * 10
    # the centres are the ones trace_points gives
    assert np.array_equal(X, geo.trace_points(pts, mesh, vel, dt, substeps))


def test_log_growth_converges_at_fourth_order():
    """A field whose dilation varies along the path: Lambda against an
    independent high-accuracy integration of the same ODE system, and the
    error falling about 16-fold per halving of the RK4 step."""
    dim = 2
    mesh = _linear_mesh(dim, 1.0)
    # bilinear (Q1-exact): u = (0.8 x y, 0.6 x y + 0.3 y), div = 0.8 y + 0.6 x + 0.3

    def field(p, t=0.0):
        x, y = p[:, 0], p[:, 1]
        return np.stack([0.8 * x * y, 0.6 * x * y + 0.3 * y], axis=1)

    vel = inputs.sample_velocity(mesh, field)
    pts = np.array([[0.6, 0.7], [0.4, 0.5], [0.8, 0.3]])
    dt = 0.4

    def rhs(s, z):
        x, y = z[0], z[1]
        return [-0.8 * x * y, -(0.6 * x * y + 0.3 * y), -(0.8 * y + 0.6 * x + 0.3)]

    errs = []
    for sub in (4, 8):
        _, lam = geo.log_growth(pts, mesh, vel, dt, sub)
        e = 0.0
        for i, p in enumerate(pts):
            sol = solve_ivp(rhs, (0.0, dt), [p[0], p[1], 0.0], rtol=1e-13, atol=1e-15,
                            method="DOP853")
            e = max(e, abs(lam[i] - sol.y[2, -1]))
        errs.append(e)
    assert errs[1] < 1e-7
    ratio = errs[0] / errs[1]
    assert 10.0 < ratio < 24.0, (errs, ratio)


def _sine_back(x, a, dt):
    """Exact backward flow of dx/dt = a sin(pi x) over dt:
    tan(pi x_hat / 2) = tan(pi x / 2) exp(-a pi dt)."""
    return (2.0 / math.pi) * np.arctan(np.tan(0.5 * math.pi * x) * math.exp(-a * math.pi * dt))


def _exact_traceback_volumes(n, amp, dt):
    """|F_{-dt}(K)| of every cell of the unit box for the separable sine
    compression: the product over the axes of the traced cell edges."""
    dim = len(n)
    vols = np.ones(int(np.prod(n)))
    ids = np.indices(n[::-1]).reshape(dim, -1)[::-1]   # x-fastest cell indices
    for a in range(dim):
        e = np.linspace(0.0, 1.0, n[a] + 1)
        eh = _sine_back(e, amp[a], dt)
        vols = vols * (eh[ids[a] + 1] - eh[ids[a]])
    return vols


@pytest.mark.parametrize("dim,n,amp", [(2, (32, 32), (0.5, -0.4)),
                                       (3, (12, 12, 12), (0.5, -0.4, 0.3))])
def test_row_targets_match_exact_traceback_volumes(dim, n, amp):
    """The separable sine compression has closed-form trace-back regions:
    the row targets (eq. volTracked, rescaled) approximate them far better
    than |K| does, and a sign error in the growth would double the error."""
    mesh = inputs.cartesian_mesh(n)
    vel = inputs.sample_velocity(mesh, inputs.sine_compression(amp))
    dt = 0.05
    out = otr.build_transfer(mesh, vel, dt, layout="subcell", stop_after="v", solenoidal=False)
    exact = _exact_traceback_volumes(n, amp, dt)
    kvol = out["cell_vol"]
    err_method = np.max(np.abs(out["b_loc"] - exact) / exact)
    err_plain = np.max(np.abs(kvol - exact) / exact)
    assert err_plain > 0.05                       # the flow compresses visibly
    assert err_method < 0.03 * err_plain, (err_method, err_plain)
    assert abs(out["target_scale"] - 1.0) < 5e-3
    # the rescaled targets sum to the column targets' sum
    assert math.isclose(math.fsum(out["b_loc"].tolist()), math.fsum(out["b"].tolist()),
                        rel_tol=1e-14)
    # V's rows carry the tracked masses (eq. ball_int sums to eq. volTracked)
    rows = otr.csr_rows(out["row_ptr"])
    rs = np.bincount(rows, weights=out["V"], minlength=kvol.size)
    assert np.max(np.abs(rs - out["T"]) / out["T"]) < 1e-13


def test_full_step_compresses_a_constant_state():
    """From c = 1 the exact update gives c_K = |F_{-dt}(K)|_phi / |K|_phi;
    the step reproduces that ratio to the accuracy of its targets, and the
    porous mass is conserved to rounding."""
    n, amp, dt = (16, 16), (0.5, -0.4), 0.05
    mesh = inputs.cartesian_mesh(n)
    vel = inputs.sample_velocity(mesh, inputs.sine_compression(amp))
    out = otr.build_transfer(mesh, vel, dt, layout="subcell", solenoidal=False)
    c0 = np.ones(mesh_cells(mesh))
    c1 = otr.apply(out["row_ptr"], out["col"], out["A"], out["b"], c0)
    # rows of the final matrix meet the targets: c1 = b_loc / |K|_phi
    assert np.max(np.abs(c1 - out["b_loc"] / out["b"])) < 1e-12
    exact = _exact_traceback_volumes(n, amp, dt) / out["cell_vol"]
    assert np.max(np.abs(c1 - exact)) < 0.1 * np.max(np.abs(exact - 1.0))
    m0 = otr.mass(mesh["phi"], out["cell_vol"], c0)
    m1 = otr.mass(mesh["phi"], out["cell_vol"], c1)
    assert abs(m1 - m0) <= 1e-13 * m0


def mesh_cells(mesh):
    return int(np.prod(mesh["n"]))


@pytest.mark.parametrize("dim", [2, 3])
def test_general_mode_on_a_solenoidal_linear_field(dim):
    """A rotation's Q1 interpolant has zero divergence: the general mode
    gives zero growth (up to the rounding of the corner sums), radii equal
    to r up to RK4's error on the tracked cardinal points, and rows of V
    equal to the solenoidal ones (cells away from the boundary, where no
    cardinal point is clamped into the box)."""
    n = (12,) * dim
    mesh = inputs.cartesian_mesh(n)
    if dim == 2:
        field = inputs.solid_body_2d
    else:
        def field(p, t=0.0):
            return np.stack([-(p[:, 1] - 0.5), p[:, 0] - 0.5, np.zeros(p.shape[0])], axis=1)
    vel = inputs.sample_velocity(mesh, field)
    dt = 0.01
    free = otr.build_transfer(mesh, vel, dt, layout="subcell", stop_after="v")
    gen = otr.build_transfer(mesh, vel, dt, layout="subcell", stop_after="v",
                             solenoidal=False)
    assert np.max(np.abs(gen["lam"])) <= 1e-15
    inner_ball = np.all(np.abs(gen["centres"] - 0.5) < 0.4, axis=1)
    assert np.max(np.abs(gen["r_hat"] - free["r_hat"])[inner_ball]) <= 1e-10
    cen = inputs.cell_centroids(mesh)
    inner = np.nonzero(np.all(np.abs(cen - 0.5) < 0.3, axis=1))[0]
    assert inner.size > 4
    for K in inner:
        a = slice(free["row_ptr"][K], free["row_ptr"][K + 1])
        g = slice(gen["row_ptr"][K], gen["row_ptr"][K + 1])
        assert np.array_equal(free["col"][a], gen["col"][g])
        assert np.max(np.abs(free["V"][a] - gen["V"][g])) <= 1e-9 * np.max(free["V"][a])


@pytest.mark.parametrize("dim", [2, 3])
def test_liouville_growth_agrees_with_tracked_radius(dim):
    """Isotropic expansion u = (delta/d)(x - x0): the tracked ball is a ball
    of radius r exp(-delta dt / d) (up to RK4's error), so the geometric
    route |B_hat| = omega_d r_hat^d (eq. rTrackedBall) and the Liouville
    route |B| exp(Lambda) agree."""
    delta = 0.8
    x0 = np.full(dim, 0.5)
    n = (8,) * dim
    mesh = inputs.cartesian_mesh(n)
    vel = inputs.sample_velocity(mesh, lambda p, t=0.0: (delta / dim) * (p - x0))
    dt = 0.05
    out = otr.build_transfer(mesh, vel, dt, layout="subcell", stop_after="pairs",
                             solenoidal=False)
    geom = geo.ball_measure(out["r_hat"], dim)
    liou = geo.ball_measure(out["radii"], dim) * np.exp(out["lam"])
    # the boundary balls' cardinal points are clamped: interior balls only
    inner = np.all(np.abs(out["centres"] - 0.5) < 0.35, axis=1)
    assert inner.sum() > 10
    assert np.max(np.abs(geom[inner] / liou[inner] - 1.0)) < 1e-7
    assert np.allclose(out["lam"], -delta * dt, rtol=1e-13, atol=0)


def test_row_targets_rescale_each_component():
    """Hand-worked: rows {0, 1} reach columns {0, 1} only and row 2 column 2
    only; each component's targets total its columns' porous volumes."""
    ball_cell = np.array([0, 0, 1, 2])
    ball_mass = np.array([0.25, 0.75, 2.0, 3.0])       # T = (1, 2, 3)
    b = np.array([1.0, 2.0, 2.5])
    rows = np.array([0, 0, 1, 2])
    cols = np.array([0, 1, 1, 2])
    b_loc, T, scale, ncomp = otr.row_targets(3, ball_cell, ball_mass, b, rows, cols)
    assert ncomp == 2
    assert np.array_equal(T, [1.0, 2.0, 3.0])
    assert np.array_equal(b_loc, [1.0, 2.0, 2.5])
    assert scale == 5.5 / 6.0


def test_disconnected_pattern_stays_consistent():
    """Small random balls leave cells whose tracked balls reach only their
    own residing balls (many components of V's pattern): each component's
    targets total its columns' porous volumes, and the least-change problem
    is solved (a single global factor would leave it inconsistent)."""
    w = inputs.swirl_hex(8)
    mesh = inputs.random_subcell_balls(w["mesh"], 5)
    vel = inputs.sample_velocity(w["mesh"], inputs.compressible_swirl_3d)
    out = otr.build_transfer(mesh, vel, 0.03, layout="custom", solenoidal=False)
    assert out["n_groups"] > 10
    rows = otr.csr_rows(out["row_ptr"])
    rs = np.bincount(rows, weights=out["A"], minlength=out["b"].size)
    cs = np.bincount(out["col"], weights=out["A"], minlength=out["b"].size)
    assert np.max(np.abs(rs - out["b_loc"])) <= 1e-13 * out["b"].max()
    assert np.max(np.abs(cs - out["b"])) <= 1e-13 * out["b"].max()
