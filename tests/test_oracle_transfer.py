"""Pins of the oracle's candidate search, V, scaling sweeps and A_hat."""

import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import qp as oqp
from oracle import transfer as otr
from paper_1908_05834_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- candidates

def _loop_pairs(tc, tr, rc, rr, ft=float):
    out = []
    for a in range(len(tc)):
        for b in range(len(rc)):
            s = ft(0.0)
            for k in range(len(tc[a])):
                d = ft(tc[a][k]) - ft(rc[b][k])
                s = s + d * d
            rs = ft(tr[a]) + ft(rr[b])
            if s < rs * rs:
                out.append((a, b))
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_candidates_match_plain_loops(dim):
    rng = np.random.default_rng(10 + dim)
    tc = rng.uniform(0, 1, (60, dim))
    rc = rng.uniform(0, 1, (70, dim))
    tr = rng.uniform(0.02, 0.15, 60)
    rr = rng.uniform(0.02, 0.15, 70)
    want = _loop_pairs(tc, tr, rc, rr)
    ia, ib = geo.candidate_pairs(tc, tr, rc, rr)
    assert list(zip(ia.tolist(), ib.tolist())) == want
    # the k-d tree branch gives the same set
    ia2, ib2 = geo.candidate_pairs(tc, tr, rc, rr, brute_force_limit=0)
    assert np.array_equal(ia, ia2) and np.array_equal(ib, ib2)


def test_candidates_fp32_predicate():
    rng = np.random.default_rng(7)
    tc = rng.uniform(0, 1, (50, 3))
    rc = rng.uniform(0, 1, (50, 3))
    tr = np.full(50, 0.1)
    rr = np.full(50, 0.1)
    want = _loop_pairs(tc.astype(np.float32), tr.astype(np.float32), rc.astype(np.float32),
                       rr.astype(np.float32), ft=np.float32)
    ia, ib = geo.candidate_pairs(tc, tr, rc, rr, precision="fp32")
    assert list(zip(ia.tolist(), ib.tolist())) == want


def test_tangent_balls_are_not_candidates():
    tc = np.array([[0.25, 0.25], [0.25, 0.25]])
    rc = np.array([[0.75, 0.25], [0.5, 0.25]])
    r = np.array([0.25, 0.25])
    ia, ib = geo.candidate_pairs(tc, r, rc, r)
    assert list(zip(ia.tolist(), ib.tolist())) == [(0, 1), (1, 1)]


# ---------------------------------------------------------------- layout

@pytest.mark.parametrize("layout", ["subcell", "inscribed", "equal_measure"])
@pytest.mark.parametrize("n", [(8, 4), (4, 2, 8)])
def test_layout_density(layout, n):
    mesh = inputs.cartesian_mesh(n)
    dim = len(n)
    C, r, cell = geo.ball_layout(n, mesh["origin"], mesh["h"], layout)
    nc = int(np.prod(n))
    per = {"subcell": 2 ** dim}.get(layout, 1)
    assert C.shape == (nc * per, dim) and np.array_equal(cell, np.repeat(np.arange(nc), per))
    kvol = geo.cell_volume(mesh["h"])
    rho = geo.porous_density(nc, np.full(nc, kvol), r, cell, dim)
    tot = np.bincount(cell, weights=rho[cell] * geo.ball_measure(r, dim))
    np.testing.assert_allclose(tot, kvol, rtol=1e-15)          # eq. def:porous.density
    if layout == "equal_measure":
        np.testing.assert_allclose(rho, 1.0, rtol=1e-14)
    else:
        # balls lie inside their cell and do not overlap
        lo = geo.cell_centroids(n, mesh["origin"], mesh["h"])[cell] - 0.5 * np.asarray(mesh["h"])
        hi = lo + np.asarray(mesh["h"])
        assert np.all(C - r[:, None] >= lo - 1e-15) and np.all(C + r[:, None] <= hi + 1e-15)
        ia, ib = geo.candidate_pairs(C, r, C, r)
        assert np.array_equal(ia, ib)


# ---------------------------------------------------------------- V

def _build(mesh, vel, dt, layout, stop="v"):
    return otr.build_transfer(mesh, vel, dt, layout=layout, stop_after=stop)


@pytest.mark.parametrize("layout", ["subcell", "inscribed", "equal_measure"])
def test_v_rows_sum_to_porous_volume(layout):
    """sum_M V_{K,M} = |K|_phi (Sec. 3.2, via eq. volTracked)."""
    n = (12, 12)
    phi = np.random.default_rng(3).uniform(0.3, 1.0, 144)
    mesh = inputs.cartesian_mesh(n, phi=phi)
    vel = inputs.sample_velocity(mesh, inputs.rotation_stretch_2d)
    T = _build(mesh, vel, 0.8, layout)
    rows = otr.csr_rows(T["row_ptr"])
    rs = np.bincount(rows, weights=T["V"], minlength=144)
    np.testing.assert_allclose(rs, T["b"], rtol=1e-14)
    assert np.all(T["V"] > 0)
    assert all(np.all(np.diff(T["col"][T["row_ptr"][i]:T["row_ptr"][i + 1]]) > 0)
               for i in range(144))


@pytest.mark.parametrize("layout", ["subcell", "inscribed"])
@pytest.mark.parametrize("n", [(8, 4), (4, 2, 8)])
def test_identity_at_zero_velocity(layout, n):
    mesh = inputs.cartesian_mesh(n)
    vel = inputs.sample_velocity(mesh, inputs.constant_field(np.zeros(len(n))))
    T = _build(mesh, vel, 0.5, layout, stop="all")
    nc = int(np.prod(n))
    assert np.array_equal(T["row_ptr"], np.arange(nc + 1))
    assert np.array_equal(T["col"], np.arange(nc))
    np.testing.assert_allclose(T["A"], T["b"], rtol=1e-15)


def test_v_relabel_invariance():
    """Reflecting the mesh and the field maps V onto itself (cells relabelled)."""
    n = (10, 8)
    mesh = inputs.cartesian_mesh(n)
    f = inputs.deformation_2d
    vel = inputs.sample_velocity(mesh, f)

    def fr(p, t=0.0):
        q = p.copy()
        q[:, 0] = 1.0 - q[:, 0]
        u = f(q, t)
        u[:, 0] = -u[:, 0]
        return u
    velr = inputs.sample_velocity(mesh, fr)
    A = _build(mesh, vel, 0.05, "subcell")
    B = _build(mesh, velr, 0.05, "subcell")
    ij = geo.cell_index_grid(n)
    mirror = (n[0] - 1 - ij[:, 0]) + n[0] * ij[:, 1]

    def dense(T):
        D = np.zeros((80, 80))
        D[otr.csr_rows(T["row_ptr"]), T["col"]] = T["V"]
        return D
    np.testing.assert_allclose(dense(B), dense(A)[np.ix_(mirror, mirror)], rtol=1e-10,
                               atol=1e-15)


# ---------------------------------------------------------------- scaling

def _fraction_sweeps(Aint, b_loc, b_glob, N):
    n = len(Aint)
    A = [[Fraction(v) for v in row] for row in Aint]
    for _ in range(N):
        cs = [sum(A[i][j] for i in range(n)) for j in range(n)]
        A = [[A[i][j] * b_glob[j] / cs[j] if A[i][j] else Fraction(0) for j in range(n)]
             for i in range(n)]
        rs = [sum(A[i]) for i in range(n)]
        A = [[A[i][j] * b_loc[i] / rs[i] for j in range(n)] for i in range(n)]
    return A


def test_scaling_exact_rational():
    """eq. volAdj evaluated in exact rational arithmetic."""
    Aint = [[5, 1, 0, 2], [0, 3, 1, 0], [1, 0, 4, 1], [2, 0, 1, 6]]
    b = [Fraction(6), Fraction(5), Fraction(7), Fraction(8)]
    want = _fraction_sweeps(Aint, b, b, 3)
    Ad = np.array(Aint, dtype=float)
    r, c = np.nonzero(Ad)
    rp = np.searchsorted(r, np.arange(5))
    got = otr.scaling_sweeps(rp, c, Ad[r, c], np.array(b, float), np.array(b, float), 3)
    np.testing.assert_allclose(got, [float(want[i][j]) for i, j in zip(r, c)], rtol=1e-14)


def test_scaling_marginals_and_fixed_point():
    rng = np.random.default_rng(8)
    n = 30
    D = rng.uniform(0, 1, (n, n)) * (rng.uniform(0, 1, (n, n)) < 0.2) + np.eye(n)
    r, c = np.nonzero(D)
    rp = np.searchsorted(r, np.arange(n + 1))
    b = rng.uniform(0.5, 2.0, n)
    b *= b.sum() / b.sum()
    A1 = otr.scaling_sweeps(rp, c, D[r, c], b, b, 1)
    np.testing.assert_allclose(np.bincount(r, weights=A1, minlength=n), b, rtol=1e-14)
    # half step: columns exact
    half = D[r, c] * (b / np.bincount(c, weights=D[r, c], minlength=n))[c]
    np.testing.assert_allclose(np.bincount(c, weights=half, minlength=n), b, rtol=1e-14)
    # a matrix that already has the marginals is left alone
    P = np.diag(b)
    r2, c2 = np.nonzero(P)
    A2 = otr.scaling_sweeps(np.arange(n + 1), c2, P[r2, c2], b, b, 10)
    np.testing.assert_allclose(A2, b, rtol=1e-15)


# ---------------------------------------------------------------- A_hat

def test_ahat_worked_example():
    with open(os.path.join(GOLDEN, "ahat_worked_example.json")) as fh:
        g = json.load(fh)
    sym = {"a": 2.0, "b": 3.0, "c": 5.0, "d": 7.0, "e": 11.0, "0": 0.0}
    # complete the printed 2 x 3 corner with a third row touching only column 2
    A = np.array([[sym[v] for v in row] for row in g["A_top_left"]] + [[0.0, 0.0, 13.0]])
    r, c = np.nonzero(A)
    rp = np.searchsorted(r, np.arange(4))
    Ah = oqp.constraint_matrix(rp, c, A[r, c], 3)
    want_rows = np.array([[sym[v] for v in row] for row in g["Ahat_row_block"]])
    want_cols = np.array([[sym[v] for v in row] for row in g["Ahat_col_block"]])
    np.testing.assert_array_equal(Ah[:2, :5], want_rows)
    np.testing.assert_array_equal(Ah[3:6, :5], want_cols)
    # A_hat 1 = [row sums; column sums]
    np.testing.assert_allclose(Ah @ np.ones(Ah.shape[1]), np.r_[A.sum(1), A.sum(0)])
