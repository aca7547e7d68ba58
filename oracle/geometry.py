"""Oracle, geometric part: ball layout, tracking, overlap search, lens measure.

Test infrastructure only (see ``oracle/__init__.py``).  Plain NumPy, binary64.

Conventions shared with the inputs (not with the HIP path):

* A Cartesian mesh is ``n`` cells per axis (x first), ``origin`` and ``h``
  per axis; cell ids run x-fastest: ``id = i + n0*(j + n1*k)``.
* A velocity lattice is ``m`` nodes per axis, ``origin``, ``spacing`` and an
  array ``u`` of shape ``(dim, prod(m))`` stored x-fastest.
* Ball layouts (the paper lets the user choose the balls of each cell,
  Sec. 3; it uses 4 balls per square and 8 per cube in Sec. 4 without
  stating where they sit):

  - ``"subcell"``: 2^d balls per cell at the centres of the 2^d half-size
    sub-cells, radius min(h)/4 (disjoint, strictly inside the cell, and one
    quarter of the smallest face diameter as Sec. 3 recommends);
  - ``"inscribed"``: one ball at the centroid, radius min(h)/2;
  - ``"equal_measure"``: one ball at the centroid whose measure equals
    |K| (it overlaps its neighbours; kept because a workload asks for the
    equal-area disk).

  Within a cell, ``subcell`` balls are numbered s = sx + 2 sy (+ 4 sz).

* A simplicial mesh is ``{"kind": "simplex", "vertices", "cells", "phi"}``:
  vertex coordinates (n_vertices, dim), the dim + 1 vertex ids of every cell
  (triangles in 2D, tetrahedra in 3D) and the porosity per cell.  The paper
  gives no ball packing for such cells (its open problem in the
  conclusion); each cell gets one ball at its centroid whose measure equals
  |K| (``"equal_measure"``, rho_K = 1 up to rounding).  The domain is the
  bounding box of the vertices.  phi(x) during tracking is phi of the cell
  containing x clamped into that box, located by ``locate_points``.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

LAYOUTS = ("subcell", "inscribed", "equal_measure")


# --------------------------------------------------------------------------
# Mesh and balls (Sec. 3, eq. def:porous.density)
# --------------------------------------------------------------------------

def is_simplex(mesh):
    return mesh.get("kind", "cartesian") == "simplex"


def mesh_dim(mesh):
    return int(np.asarray(mesh["vertices"]).shape[1]) if is_simplex(mesh) else len(mesh["n"])


def mesh_n_cells(mesh):
    return int(np.asarray(mesh["cells"]).shape[0]) if is_simplex(mesh) else int(np.prod(mesh["n"]))


def domain_box(mesh):
    """(lo, hi) corners of the domain box."""
    if is_simplex(mesh):
        V = np.asarray(mesh["vertices"], dtype=np.float64)
        return V.min(axis=0), V.max(axis=0)
    lo = np.asarray(mesh["origin"], dtype=np.float64)
    return lo, lo + np.asarray(mesh["n"], dtype=np.float64) * np.asarray(mesh["h"], dtype=np.float64)


def _orient(a, b, c, d=None):
    """Signed d! |simplex| of the points a, b, c (2D) or a, b, c, d (3D),
    arrays of shape (..., dim): the determinant of the edge vectors from a,
    expanded along the first edge, each operation rounded on its own in the
    order written."""
    e1, e2 = b - a, c - a
    if d is None:
        return e1[..., 0] * e2[..., 1] - e1[..., 1] * e2[..., 0]
    e3 = d - a
    m0 = e2[..., 1] * e3[..., 2] - e2[..., 2] * e3[..., 1]
    m1 = e2[..., 0] * e3[..., 2] - e2[..., 2] * e3[..., 0]
    m2 = e2[..., 0] * e3[..., 1] - e2[..., 1] * e3[..., 0]
    return (e1[..., 0] * m0 - e1[..., 1] * m1) + e1[..., 2] * m2


def simplex_volumes(vertices, cells):
    """|K| = |det(v1 - v0, ..., vd - v0)| / d!."""
    V = np.asarray(vertices, dtype=np.float64)
    C = np.asarray(cells, dtype=np.int64)
    P = [V[C[:, i]] for i in range(C.shape[1])]
    if V.shape[1] == 2:
        return np.abs(_orient(P[0], P[1], P[2])) / 2.0
    return np.abs(_orient(P[0], P[1], P[2], P[3])) / 6.0


def simplex_centroids(vertices, cells):
    """(((v0 + v1) + v2) (+ v3)) / (dim + 1), summed in vertex order."""
    V = np.asarray(vertices, dtype=np.float64)
    C = np.asarray(cells, dtype=np.int64)
    acc = V[C[:, 0]] + V[C[:, 1]]
    for i in range(2, C.shape[1]):
        acc = acc + V[C[:, i]]
    return acc / float(C.shape[1])


def cbrt_rounded(y):
    """The binary64 number nearest to the real cube root of each y > 0.

    A library cube root (within a few units in the last place) gives a
    start; among it and its two neighbours on each side the one whose
    rounding interval holds y^(1/3) is taken, deciding exactly: r is the
    nearest double iff the cubes of the midpoints to its neighbours, in
    rational arithmetic, bracket y."""
    from fractions import Fraction
    y = np.asarray(y, dtype=np.float64)
    out = np.empty_like(y)
    for i, v in enumerate(y.ravel()):
        fv = Fraction(float(v))
        r = float(np.cbrt(v))
        cand = [r]
        for _ in range(2):
            cand.insert(0, float(np.nextafter(cand[0], 0.0)))
            cand.append(float(np.nextafter(cand[-1], np.inf)))
        best = None
        for k in range(1, len(cand) - 1):
            lo = (Fraction(cand[k - 1]) + Fraction(cand[k])) / 2
            hi = (Fraction(cand[k]) + Fraction(cand[k + 1])) / 2
            if lo ** 3 <= fv <= hi ** 3:
                best = cand[k]
                break
        if best is None:
            raise ArithmeticError("cube root start more than two places off")
        out.flat[i] = best
    return out


def simplex_ball_layout(mesh):
    """One ball per simplex at its centroid with |B| = |K| (2D sqrt(|K|/pi),
    3D the correctly rounded (3 |K| / (4 pi))^(1/3)).  Returns centres,
    radii, cell."""
    V = np.asarray(mesh["vertices"], dtype=np.float64)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    dim = V.shape[1]
    vol = simplex_volumes(V, C)
    centres = simplex_centroids(V, C)
    if dim == 2:
        radii = np.sqrt(vol / math.pi)
    else:
        radii = cbrt_rounded(3.0 * vol / (4.0 * math.pi))
    return centres, radii, np.arange(C.shape[0], dtype=np.int64)


PACK_SHRINK = 0.875


def simplex_packed_layout(mesh, shrink=PACK_SHRINK):
    """Several disjoint balls per simplex (``"packed"``; the paper leaves the
    packing of generic cells open, Sec. 5).

    Per cell, in this order: the inscribed ball (centre the incentre
    I = sum_i w_i v_i / sum_i w_i, w_i the measure of the facet opposite
    v_i, radius r = dim |K| / sum_i w_i), then for every vertex v_i the
    ball tangent to the dim facets through v_i and to the inscribed ball:
    centre v_i + t (I - v_i), radius t r, t = (L - r) / (L + r), L = |v_i -
    I|.  Every radius is then multiplied by ``shrink`` (each ball keeps its
    centre, so tangencies become gaps and the balls lie strictly inside).
    A cell whose balls still overlap (possible for very flat simplices)
    keeps its inscribed ball only.  Sums run in vertex and axis order;
    every operation is rounded on its own.
    Returns (centres (n_balls, dim), radii, ball_cell).
    """
    V = np.asarray(mesh["vertices"], dtype=np.float64)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    dim = V.shape[1]
    nc = C.shape[0]
    P = [V[C[:, i]] for i in range(dim + 1)]
    vol = simplex_volumes(V, C)
    w = []
    for i in range(dim + 1):
        o = [j for j in range(dim + 1) if j != i]
        if dim == 2:
            e = P[o[1]] - P[o[0]]
            w.append(np.sqrt(e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]))
        else:
            u = P[o[1]] - P[o[0]]
            v = P[o[2]] - P[o[0]]
            c0 = u[:, 1] * v[:, 2] - u[:, 2] * v[:, 1]
            c1 = u[:, 2] * v[:, 0] - u[:, 0] * v[:, 2]
            c2 = u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0]
            w.append(np.sqrt((c0 * c0 + c1 * c1) + c2 * c2) / 2.0)
    W = w[0] + w[1]
    for i in range(2, dim + 1):
        W = W + w[i]
    inc = np.zeros((nc, dim))
    for a in range(dim):
        acc = w[0] * P[0][:, a] + w[1] * P[1][:, a]
        for i in range(2, dim + 1):
            acc = acc + w[i] * P[i][:, a]
        inc[:, a] = acc / W
    r = (dim * vol) / W
    cen = [inc]
    rad = [shrink * r]
    for i in range(dim + 1):
        d = P[i] - inc
        L2 = d[:, 0] * d[:, 0]
        for a in range(1, dim):
            L2 = L2 + d[:, a] * d[:, a]
        L = np.sqrt(L2)
        t = (L - r) / (L + r)
        cen.append(P[i] + t[:, None] * (inc - P[i]))
        rad.append(shrink * (t * r))
    nb = dim + 2
    # disjointness of every pair after the shrink
    ok = np.ones(nc, dtype=bool)
    for a in range(nb):
        for b in range(a + 1, nb):
            d = cen[a] - cen[b]
            d2 = d[:, 0] * d[:, 0]
            for k in range(1, dim):
                d2 = d2 + d[:, k] * d[:, k]
            ok &= np.sqrt(d2) >= rad[a] + rad[b]
    centres, radii, cell = [], [], []
    for K in range(nc):
        take = range(nb) if ok[K] else range(1)
        for q in take:
            centres.append(cen[q][K])
            radii.append(rad[q][K])
            cell.append(K)
    return np.array(centres), np.array(radii), np.array(cell, dtype=np.int64)


def locate_points(points, mesh, chunk=2048):
    """Cell of a simplicial mesh holding each point.

    Candidates are the cells whose bounding box (min and max of the vertex
    coordinates) contains the point, closed.  The point lies in a cell when,
    for every vertex, the orientation of the cell with that vertex replaced
    by the point (``_orient``) is zero or has the sign of the cell's own
    orientation; the lowest-numbered such candidate is taken.  If rounding
    leaves a point in none, the candidate whose centroid is nearest is
    taken (squared distance summed over the axes in order, the lowest
    number on ties).  Brute force over all cells, in chunks of points."""
    V = np.asarray(mesh["vertices"], dtype=np.float64)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    X = np.asarray(points, dtype=np.float64)
    dim = V.shape[1]
    P = [V[C[:, i]] for i in range(dim + 1)]
    blo = np.minimum.reduce(P)
    bhi = np.maximum.reduce(P)
    own = _orient(*P)
    cen = simplex_centroids(V, C)
    out = np.empty(X.shape[0], dtype=np.int64)
    for s0 in range(0, X.shape[0], chunk):
        x = X[s0:s0 + chunk][:, None, :]                       # (m, 1, dim)
        cand = np.all((x >= blo[None]) & (x <= bhi[None]), axis=2)   # (m, nc)
        inside = cand & (own[None] != 0.0)
        for i in range(dim + 1):
            Q = [np.broadcast_to(p[None], (x.shape[0],) + p.shape) for p in P]
            Q[i] = np.broadcast_to(x, Q[0].shape)
            o = _orient(*Q)
            inside &= np.where(own[None] > 0.0, o >= 0.0, o <= 0.0)
        for r in range(x.shape[0]):
            hit = np.nonzero(inside[r])[0]
            if hit.size:
                out[s0 + r] = hit[0]
                continue
            cids = np.nonzero(cand[r])[0]
            if cids.size == 0:
                raise ValueError("point outside every cell's bounding box")
            dx = x[r, 0] - cen[cids]
            d2 = dx[:, 0] * dx[:, 0] + dx[:, 1] * dx[:, 1]
            if dim == 3:
                d2 = d2 + dx[:, 2] * dx[:, 2]
            out[s0 + r] = cids[int(np.argmin(d2))]
    return out


def cell_index_grid(n):
    """Integer (i, j[, k]) of every cell, x-fastest, shape (n_cells, dim)."""
    dim = len(n)
    nc = int(np.prod(n))
    ids = np.arange(nc, dtype=np.int64)
    out = np.empty((nc, dim), dtype=np.int64)
    rem = ids.copy()
    for a in range(dim):
        out[:, a] = rem % n[a]
        rem //= n[a]
    return out


def cell_centroids(n, origin, h):
    ijk = cell_index_grid(n).astype(np.float64)
    return np.asarray(origin, dtype=np.float64) + (ijk + 0.5) * np.asarray(h, dtype=np.float64)


def cell_volume(h):
    """|K| of a Cartesian cell (all cells equal)."""
    v = 1.0
    for x in h:
        v *= float(x)
    return v


def ball_measure(r, dim):
    """|B| of a ball of radius r: pi r^2 (2D) or 4/3 pi r^3 (3D)."""
    r = np.asarray(r, dtype=np.float64)
    if dim == 2:
        return math.pi * r * r
    if dim == 3:
        return (4.0 / 3.0) * math.pi * r * r * r
    raise ValueError("dim must be 2 or 3")


def ball_layout(n, origin, h, layout):
    """Balls of every cell.

    Returns ``centres`` (n_balls, dim), ``radii`` (n_balls,), ``cell``
    (n_balls,) with balls ordered cell-major.
    """
    dim = len(n)
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    h = np.asarray(h, dtype=np.float64)
    origin = np.asarray(origin, dtype=np.float64)
    ijk = cell_index_grid(n).astype(np.float64)
    nc = ijk.shape[0]
    if layout == "subcell":
        nb_per = 2 ** dim
        offs = np.array([[(s >> a) & 1 for a in range(dim)] for s in range(nb_per)],
                        dtype=np.float64)
        # sub-cell centre = cell corner + (1/4 or 3/4) h per axis
        frac = 0.25 + 0.5 * offs                         # (nb_per, dim)
        centres = origin + (ijk[:, None, :] + frac[None, :, :]) * h
        centres = centres.reshape(nc * nb_per, dim)
        radii = np.full(nc * nb_per, float(h.min()) / 4.0)
        cell = np.repeat(np.arange(nc, dtype=np.int64), nb_per)
    elif layout == "inscribed":
        centres = origin + (ijk + 0.5) * h
        radii = np.full(nc, float(h.min()) / 2.0)
        cell = np.arange(nc, dtype=np.int64)
    elif layout == "equal_measure":
        centres = origin + (ijk + 0.5) * h
        vol = cell_volume(h)
        if dim == 2:
            r = math.sqrt(vol / math.pi)
        else:
            r = float(cbrt_rounded(np.array([3.0 * vol / (4.0 * math.pi)]))[0])
        radii = np.full(nc, r)
        cell = np.arange(nc, dtype=np.int64)
    else:
        raise ValueError(f"unknown layout {layout!r}")
    return centres, radii, cell


def porous_density(n_cells, cell_vol, radii, cell, dim):
    """rho_K with rho_K * sum_s |B_{K,s}|_phi = |K|_phi (eq. def:porous.density).

    With |B_{K,s}|_phi = phi_K |B_{K,s}| (phi is constant on K), phi cancels
    and rho_K = |K| / sum_s |B_{K,s}|.
    """
    per_cell = np.bincount(cell, weights=ball_measure(radii, dim), minlength=n_cells)
    return np.asarray(cell_vol, dtype=np.float64) / per_cell


# --------------------------------------------------------------------------
# Velocity and porosity evaluation
# --------------------------------------------------------------------------

def q1_interpolate(points, m, origin, spacing, u):
    """Multilinear (Q1) interpolation of a nodal lattice field.

    The query point is first clamped into the lattice box; the lattice cell
    is floor((x - origin)/spacing) clamped to [0, m-2].  Returns
    (n_points, dim) values.
    """
    pts = np.asarray(points, dtype=np.float64)
    npnt, dim = pts.shape
    m = [int(v) for v in m]
    org = np.asarray(origin, dtype=np.float64)
    sp = np.asarray(spacing, dtype=np.float64)
    upper = org + (np.asarray(m) - 1) * sp
    q = np.minimum(np.maximum(pts, org), upper)
    t = (q - org) / sp
    idx = np.minimum(np.floor(t).astype(np.int64), np.asarray(m) - 2)
    idx = np.maximum(idx, 0)
    f = t - idx
    out = np.zeros((npnt, dim), dtype=np.float64)
    strides = [1]
    for a in range(1, dim):
        strides.append(strides[-1] * m[a - 1])
    for corner in range(2 ** dim):
        w = np.ones(npnt)
        node = np.zeros(npnt, dtype=np.int64)
        for a in range(dim):
            bit = (corner >> a) & 1
            w = w * (f[:, a] if bit else (1.0 - f[:, a]))
            node = node + (idx[:, a] + bit) * strides[a]
        for c in range(dim):
            out[:, c] += w * u[c][node]
    return out


def cell_of_point(points, n, origin, h):
    """Id of the Cartesian cell containing each point (clamped to the mesh)."""
    pts = np.asarray(points, dtype=np.float64)
    dim = pts.shape[1]
    cid = np.zeros(pts.shape[0], dtype=np.int64)
    stride = 1
    for a in range(dim):
        ia = np.floor((pts[:, a] - origin[a]) / h[a]).astype(np.int64)
        ia = np.clip(ia, 0, n[a] - 1)
        cid += ia * stride
        stride *= n[a]
    return cid


def q1_divergence(points, m, origin, spacing, u):
    """div of the multilinear (Q1) interpolant of a nodal lattice field.

    The point is clamped and its lattice cell chosen exactly as in
    ``q1_interpolate``; on that cell the interpolant is the sum over the
    corners of prod_b w_b times the nodal value, w_b = f_b or 1 - f_b, so
    d/dx_a of it is (1/spacing_a) times the sum over the corners of
    (+1 if the corner's bit a is set, else -1) prod_{b != a} w_b u_a(node).
    Evaluated per axis a: the corners in binary order, the product over
    the axes b != a in increasing order, then divided by spacing_a; the
    divergence is the sum of the axes' terms in axis order.
    """
    pts = np.asarray(points, dtype=np.float64)
    npnt, dim = pts.shape
    m = [int(v) for v in m]
    org = np.asarray(origin, dtype=np.float64)
    sp = np.asarray(spacing, dtype=np.float64)
    upper = org + (np.asarray(m) - 1) * sp
    q = np.minimum(np.maximum(pts, org), upper)
    t = (q - org) / sp
    idx = np.minimum(np.floor(t).astype(np.int64), np.asarray(m) - 2)
    idx = np.maximum(idx, 0)
    f = t - idx
    strides = [1]
    for a in range(1, dim):
        strides.append(strides[-1] * m[a - 1])
    div = np.zeros(npnt)
    for a in range(dim):
        acc = np.zeros(npnt)
        for corner in range(2 ** dim):
            g = np.ones(npnt)
            node = np.zeros(npnt, dtype=np.int64)
            for b in range(dim):
                bit = (corner >> b) & 1
                if b != a:
                    g = g * (f[:, b] if bit else (1.0 - f[:, b]))
                node = node + (idx[:, b] + bit) * strides[b]
            term = g * u[a][node]
            acc = acc + (term if (corner >> a) & 1 else -term)
        div = div + acc / sp[a]
    return div


def phi_at(points, mesh):
    """phi of the cell holding each point (the rule of ``speed``)."""
    phi = np.asarray(mesh["phi"], dtype=np.float64)
    if phi_is_constant(phi):
        return np.full(np.asarray(points).shape[0], phi[0])
    if is_simplex(mesh):
        # the cell of the point clamped into the domain box (a cardinal
        # point of a boundary ball starts outside it)
        lo, hi = domain_box(mesh)
        cid = locate_points(np.minimum(np.maximum(points, lo), hi), mesh)
    else:
        cid = cell_of_point(points, mesh["n"], mesh["origin"], mesh["h"])
    return phi[cid]


def speed(points, mesh, vel):
    """v(x) = u^{(n+1)}(x) / phi(x), the right-hand side of eq. charac."""
    u = q1_interpolate(points, vel["m"], vel["origin"], vel["spacing"], vel["u"])
    return u / phi_at(points, mesh)[:, None]


def dilation(points, mesh, vel):
    """delta(x) = div u(x) / phi(x): the rate at which the flow of u/phi
    dilates volume inside a cell of constant porosity (div of the Q1
    interpolant, ``q1_divergence``)."""
    d = q1_divergence(points, vel["m"], vel["origin"], vel["spacing"], vel["u"])
    return d / phi_at(points, mesh)


def phi_is_constant(phi):
    phi = np.asarray(phi)
    return bool(np.all(phi == phi[0]))


# --------------------------------------------------------------------------
# Tracking (Sec. 2, eq. charac; Sec. 3, tracking of the centres)
# --------------------------------------------------------------------------

def trace_points(points, mesh, vel, dt, substeps=1):
    """Points moved backward by dt along the flow of u/phi.

    F_{-dt}(x) solves dX/ds = -v(X) on [0, dt] with X(0) = x.  Each of the
    ``substeps`` sub-intervals of length tau = dt/substeps takes one
    classical fourth-order Runge-Kutta step with the velocity frozen over
    the time step, and the result is clamped, axis by axis, into the domain
    box (the velocity is tangential on the boundary, Sec. 1.1, so exact
    trajectories never leave it).
    """
    X = np.array(points, dtype=np.float64, copy=True)
    dim = X.shape[1]
    lo, hi = domain_box(mesh)
    tau = float(dt) / int(substeps)
    for _ in range(int(substeps)):
        k1 = speed(X, mesh, vel)
        k2 = speed(X - 0.5 * tau * k1, mesh, vel)
        k3 = speed(X - 0.5 * tau * k2, mesh, vel)
        k4 = speed(X - tau * k3, mesh, vel)
        X = X - (tau / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        X = np.minimum(np.maximum(X, lo), hi)
    assert X.shape[1] == dim
    return X


def log_growth(points, mesh, vel, dt, substeps=1):
    """Lambda = log(|B_hat|_phi / |B|_phi) of a ball tracked from each point.

    The generalised Liouville formula (eq. genLiouville) says that the
    porous volume W(t) of a region carried by the flow changes at the rate
    of the integral of div u over it.  With that integral replaced by
    delta(X(t)) W(t), delta = div u / phi at the tracked centre X(t) (exact
    where div u / phi is constant over the ball), W(t^n) = W(t^{n+1})
    exp(-int delta(X(t)) dt): the analogue of eq. expPhiB for a
    non-solenoidal u.  The integral is taken by the same RK4 steps as the
    centre (``trace_points``): the stage points are the centre's, and each
    sub-interval adds -(tau/6) (d1 + 2 d2 + 2 d3 + d4), left to right.
    Returns (traced centres, Lambda).
    """
    X = np.array(points, dtype=np.float64, copy=True)
    lo, hi = domain_box(mesh)
    tau = float(dt) / int(substeps)
    lam = np.zeros(X.shape[0])
    for _ in range(int(substeps)):
        k1 = speed(X, mesh, vel)
        d1 = dilation(X, mesh, vel)
        Y = X - 0.5 * tau * k1
        k2 = speed(Y, mesh, vel)
        d2 = dilation(Y, mesh, vel)
        Y = X - 0.5 * tau * k2
        k3 = speed(Y, mesh, vel)
        d3 = dilation(Y, mesh, vel)
        Y = X - tau * k3
        k4 = speed(Y, mesh, vel)
        d4 = dilation(Y, mesh, vel)
        X = X - (tau / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        X = np.minimum(np.maximum(X, lo), hi)
        lam = lam - (tau / 6.0) * (d1 + 2.0 * d2 + 2.0 * d3 + d4)
    return X, lam


def tracked_radius(centres, radii, traced_centres, mesh, vel, dt, substeps=1,
                   solenoidal=True):
    """Radius r_hat of every tracked ball.

    phi constant in the domain and u solenoidal: r_hat = r exactly
    (eq. ball_volChange).  Otherwise (non-constant phi, or a non-solenoidal
    u, Sec. 3.2, Remark on non-solenoidal fields) the 2d cardinal points
    C +- r e_a are tracked like the centre and r_hat is the mean of their
    distances to the tracked centre (eq. rTrackedBall; the paper writes the
    2D case with 4 points, the 3D analogue uses the 6 points on the
    coordinate axes).
    """
    phi = np.asarray(mesh["phi"])
    if solenoidal and phi_is_constant(phi):
        return np.array(radii, dtype=np.float64, copy=True)
    C = np.asarray(centres, dtype=np.float64)
    dim = C.shape[1]
    r = np.asarray(radii, dtype=np.float64)
    acc = np.zeros(C.shape[0])
    for a in range(dim):
        for sgn in (1.0, -1.0):
            P = C.copy()
            P[:, a] += sgn * r
            Ph = trace_points(P, mesh, vel, dt, substeps)
            acc += np.sqrt(np.sum((Ph - traced_centres) ** 2, axis=1))
    return acc / (2 * dim)


# --------------------------------------------------------------------------
# Overlap predicate and candidate pairs
# --------------------------------------------------------------------------

def overlap_predicate(dx, rsum):
    """((dx0*dx0 + dx1*dx1) + dx2*dx2) < rsum*rsum, left to right.

    Evaluated in the dtype of the inputs (float64 or float32); NumPy applies
    no fused multiply-add, so every product and sum is rounded once.
    Tangent balls (distance == r1 + r2) are not candidates.
    """
    s = dx[..., 0] * dx[..., 0]
    for a in range(1, dx.shape[-1]):
        s = s + dx[..., a] * dx[..., a]
    return s < rsum * rsum


def candidate_pairs(tc, tr, rc, rr, precision="fp64", brute_force_limit=2e7):
    """All (tracked ball a, residing ball b) whose balls overlap.

    ``precision="fp64"`` evaluates the predicate in binary64;
    ``"fp32"`` rounds centres and radii to binary32 and evaluates it there.
    Small problems are searched by brute force over all pairs; larger ones
    take a k-d tree superset (distance <= max radii sum, slightly widened)
    and filter it with the same predicate.  Returns (ia, ib) sorted by
    (a, b).
    """
    tc = np.asarray(tc, dtype=np.float64)
    rc = np.asarray(rc, dtype=np.float64)
    tr = np.asarray(tr, dtype=np.float64)
    rr = np.asarray(rr, dtype=np.float64)
    ft = np.float32 if precision == "fp32" else np.float64
    tcp, trp, rcp, rrp = tc.astype(ft), tr.astype(ft), rc.astype(ft), rr.astype(ft)
    na, nb = tc.shape[0], rc.shape[0]
    if na == 0 or nb == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if float(na) * float(nb) <= brute_force_limit:
        ia_l, ib_l = [], []
        chunk = max(1, int(brute_force_limit // max(nb, 1) // 4) or 1)
        for s in range(0, na, chunk):
            e = min(na, s + chunk)
            dx = tcp[s:e, None, :] - rcp[None, :, :]
            rs = trp[s:e, None] + rrp[None, :]
            m = overlap_predicate(dx, rs)
            a, b = np.nonzero(m)
            ia_l.append(a + s)
            ib_l.append(b)
        ia = np.concatenate(ia_l).astype(np.int64)
        ib = np.concatenate(ib_l).astype(np.int64)
    else:
        reach = (float(tr.max()) + float(rr.max())) * (1.0 + 1e-6) + 1e-300
        ta = cKDTree(tc)
        tb = cKDTree(rc)
        coo = ta.sparse_distance_matrix(tb, reach, output_type="ndarray")
        ia = coo["i"].astype(np.int64)
        ib = coo["j"].astype(np.int64)
        dx = tcp[ia] - rcp[ib]
        rs = trp[ia] + rrp[ib]
        keep = overlap_predicate(dx, rs)
        ia, ib = ia[keep], ib[keep]
    order = np.lexsort((ib, ia))
    return ia[order], ib[order]


# --------------------------------------------------------------------------
# Measure of the intersection of two balls (the "lens")
# --------------------------------------------------------------------------

def _segment_area(r, t):
    """Area of the part of a disk of radius r beyond a chord at signed
    distance t from its centre (|t| <= r): r^2 alpha - t sqrt(r^2 - t^2),
    alpha the half-angle the chord subtends (cos alpha = t/r), taken as
    atan2(sqrt(r^2 - t^2), t) with r^2 - t^2 = (r - t)(r + t) so that it
    stays accurate when the chord nearly touches the circle."""
    t = np.clip(t, -r, r)
    s = np.sqrt(np.maximum((r - t) * (r + t), 0.0))
    return r * r * np.arctan2(s, t) - t * s


def _cap_volume(r, t):
    """Volume of the part of a ball of radius r beyond a plane at signed
    distance t from its centre (|t| <= r): a cap of height H = r - t has
    volume pi H^2 (3 r - H) / 3."""
    H = r - t
    return math.pi * H * H * (3.0 * r - H) / 3.0


def _lens(r1, r2, d, dim):
    r1 = np.asarray(r1, dtype=np.float64)
    r2 = np.asarray(r2, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    r1, r2, d = np.broadcast_arrays(r1, r2, d)
    out = np.zeros(d.shape, dtype=np.float64)
    rmin = np.minimum(r1, r2)
    inside = d <= np.abs(r1 - r2)
    apart = d >= r1 + r2
    out[inside] = ball_measure(rmin[inside], dim)
    mid = ~(inside | apart)
    if np.any(mid):
        a, b, dd = r1[mid], r2[mid], d[mid]
        # the radical plane sits at distance t1 from centre 1, t2 from centre 2
        t1 = (dd * dd + a * a - b * b) / (2.0 * dd)
        t2 = dd - t1
        if dim == 2:
            v = _segment_area(a, t1) + _segment_area(b, t2)
        else:
            v = _cap_volume(a, t1) + _cap_volume(b, t2)
        out[mid] = np.maximum(v, 0.0)
    return out


def disk_lens_area(r1, r2, d):
    """|B(c1, r1) cap B(c2, r2)| in 2D for centre distance d."""
    return _lens(r1, r2, d, 2)


def sphere_lens_volume(r1, r2, d):
    """|B(c1, r1) cap B(c2, r2)| in 3D for centre distance d."""
    return _lens(r1, r2, d, 3)


def lens_measure(r1, r2, d, dim):
    return _lens(r1, r2, d, dim)
