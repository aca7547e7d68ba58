"""Seeded synthetic inputs: meshes, porosity, velocity lattices, c^0.

This module only *describes problems*; it holds none of the B-char
arithmetic (no balls, no tracking, no intersections, no adjustment).  Both
the HIP path and the CPU oracle receive what it produces.

* A Cartesian mesh is a dict ``{"n", "origin", "h", "phi"}``: cells per
  axis (x first), the domain corner, the cell size per axis and the
  porosity per cell (cell ids x-fastest).
* A velocity lattice is a dict ``{"m", "origin", "spacing", "u"}``: nodes
  per axis, the first node, the node spacing and ``u`` of shape
  ``(dim, prod(m))`` stored x-fastest.  For a Cartesian mesh the lattice
  nodes are the mesh vertices, so the Q1 interpolant of the nodal values is
  a piecewise polynomial on the mesh as the scheme assumes.
* A simplicial mesh is a dict ``{"kind": "simplex", "vertices", "cells",
  "phi"}``: vertex coordinates (n_vertices, dim), the dim + 1 vertex ids of
  every triangle or tetrahedron, and the porosity per cell.
* A time-dependent field is sampled at the middle of each time interval.
"""

from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# meshes and lattices
# --------------------------------------------------------------------------

def cartesian_mesh(n, length=1.0, origin=None, phi=None):
    n = tuple(int(v) for v in n)
    dim = len(n)
    if origin is None:
        origin = (0.0,) * dim
    L = (float(length),) * dim if np.isscalar(length) else tuple(float(v) for v in length)
    h = tuple(L[a] / n[a] for a in range(dim))
    nc = int(np.prod(n))
    if phi is None:
        phi = np.ones(nc)
    return {"n": n, "origin": tuple(float(v) for v in origin), "h": h,
            "phi": np.ascontiguousarray(phi, dtype=np.float64)}


def simplex_mesh(vertices, cells, phi=None):
    V = np.ascontiguousarray(vertices, dtype=np.float64)
    C = np.ascontiguousarray(cells, dtype=np.int32)
    if phi is None:
        phi = np.ones(C.shape[0])
    return {"kind": "simplex", "vertices": V, "cells": C,
            "phi": np.ascontiguousarray(phi, dtype=np.float64)}


def _grid_vertices(n, jitter, seed):
    """(n+1)^dim vertices of the unit square/cube, x-fastest; interior
    vertices moved by U(-jitter, jitter) h per axis (seeded)."""
    dim = len(n)
    m = tuple(v + 1 for v in n)
    h = tuple(1.0 / v for v in n)
    V = lattice_nodes(m, (0.0,) * dim, h)
    if jitter > 0:
        ids = np.arange(V.shape[0])
        rem = ids.copy()
        interior = np.ones(V.shape[0], dtype=bool)
        for a in range(dim):
            i = rem % m[a]
            rem //= m[a]
            interior &= (i > 0) & (i < m[a] - 1)
        rng = np.random.default_rng(seed)
        J = rng.uniform(-jitter, jitter, size=V.shape) * np.asarray(h)
        V[interior] += J[interior]
    return V, m


def kuhn_tets(n, jitter=0.1, seed=1908, phi=None):
    """n^3 cubes of the unit cube, each split into the 6 Kuhn tetrahedra
    (corner 000 to corner 111 along the 6 orders of the axes), interior
    vertices jittered by up to ``jitter`` h."""
    n3 = (int(n),) * 3
    V, m = _grid_vertices(n3, jitter, seed)
    ijk = np.stack(np.meshgrid(*(np.arange(v) for v in n3), indexing="ij"), -1)
    ijk = ijk.transpose(2, 1, 0, 3).reshape(-1, 3)          # x fastest
    def vid(off):
        q = ijk + np.asarray(off)
        return q[:, 0] + m[0] * (q[:, 1] + m[1] * q[:, 2])
    cells = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        p = [0, 0, 0]
        path = [vid(p)]
        for a in perm:
            p[a] = 1
            path.append(vid(tuple(p)))
        cells.append(np.stack(path, 1))
    C = np.stack(cells, 1).reshape(-1, 4)                  # cube-major
    return simplex_mesh(V, C, phi)


def triangulated_square(n, jitter=0.1, seed=1908, phi=None):
    """n^2 squares of the unit square, each split along its diagonal from
    corner 00 to corner 11; interior vertices jittered by up to ``jitter`` h."""
    n2 = (int(n),) * 2
    V, m = _grid_vertices(n2, jitter, seed)
    j, i = np.meshgrid(np.arange(n2[1]), np.arange(n2[0]), indexing="ij")
    i, j = i.ravel(), j.ravel()
    v00 = i + m[0] * j
    v10, v01, v11 = v00 + 1, v00 + m[0], v00 + m[0] + 1
    C = np.stack([np.stack([v00, v10, v11], 1), np.stack([v00, v01, v11], 1)], 1).reshape(-1, 3)
    return simplex_mesh(V, C, phi)


def n_cells(mesh):
    return int(mesh["cells"].shape[0]) if mesh.get("kind") == "simplex" else int(np.prod(mesh["n"]))


def cell_centroids(mesh):
    if mesh.get("kind") == "simplex":
        return mesh["vertices"][mesh["cells"]].mean(axis=1)
    n, o, h = mesh["n"], mesh["origin"], mesh["h"]
    dim = len(n)
    ids = np.arange(int(np.prod(n)))
    out = np.empty((ids.size, dim))
    rem = ids.copy()
    for a in range(dim):
        out[:, a] = o[a] + ((rem % n[a]) + 0.5) * h[a]
        rem //= n[a]
    return out


def lattice_nodes(m, origin, spacing):
    dim = len(m)
    ids = np.arange(int(np.prod(m)))
    out = np.empty((ids.size, dim))
    rem = ids.copy()
    for a in range(dim):
        out[:, a] = origin[a] + (rem % m[a]) * spacing[a]
        rem //= m[a]
    return out


def sample_velocity_grid(n, field, t=0.0):
    """Lattice of (n+1)^dim nodes on the unit square/cube (the unjittered
    vertex grid of ``kuhn_tets`` / ``triangulated_square``)."""
    m = tuple(int(v) + 1 for v in n)
    h = tuple(1.0 / int(v) for v in n)
    pts = lattice_nodes(m, (0.0,) * len(n), h)
    u = np.ascontiguousarray(np.asarray(field(pts, t), dtype=np.float64).T)
    return {"m": m, "origin": (0.0,) * len(n), "spacing": h, "u": u}


def sample_velocity(mesh, field, t=0.0):
    """Nodal lattice on the mesh vertices of ``field(points, t)``."""
    m = tuple(v + 1 for v in mesh["n"])
    pts = lattice_nodes(m, mesh["origin"], mesh["h"])
    u = np.ascontiguousarray(np.asarray(field(pts, t), dtype=np.float64).T)
    return {"m": m, "origin": mesh["origin"], "spacing": mesh["h"], "u": u}


# --------------------------------------------------------------------------
# velocity fields
# --------------------------------------------------------------------------

def solid_body_2d(p, t=0.0):
    """u = 2 pi (-(y - 1/2), x - 1/2): one turn per unit time."""
    x, y = p[:, 0], p[:, 1]
    return np.stack([-2.0 * math.pi * (y - 0.5), 2.0 * math.pi * (x - 0.5)], axis=1)


def rotation_stretch_2d(p, t=0.0):
    """u = ((1-2y)(x-x^2), -(1-2x)(y-y^2)): divergence free, tangential on
    the unit square (the rotation-with-stretching field of the 2D tests)."""
    x, y = p[:, 0], p[:, 1]
    return np.stack([(1 - 2 * y) * (x - x * x), -(1 - 2 * x) * (y - y * y)], axis=1)


def swirl_3d(p, t=0.0, period=1.0, amplitude=1.0):
    """Divergence-free 3D swirl, reversing at t = period/2:
    u = (2 sin^2(pi x) sin(2 pi y) sin(2 pi z),
         -sin(2 pi x) sin^2(pi y) sin(2 pi z),
         -sin(2 pi x) sin(2 pi y) sin^2(pi z)) cos(pi t / period)."""
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    s = amplitude * math.cos(math.pi * t / period)
    sx, sy, sz = np.sin(math.pi * x), np.sin(math.pi * y), np.sin(math.pi * z)
    s2x, s2y, s2z = np.sin(2 * math.pi * x), np.sin(2 * math.pi * y), np.sin(2 * math.pi * z)
    return s * np.stack([2 * sx * sx * s2y * s2z, -s2x * sy * sy * s2z, -s2x * s2y * sz * sz],
                        axis=1)


def deformation_2d(p, t=0.0, period=1.0, amplitude=1.0):
    """2D analogue: u = (sin^2(pi x) sin(2 pi y), -sin^2(pi y) sin(2 pi x)) cos(pi t/T)."""
    x, y = p[:, 0], p[:, 1]
    s = amplitude * math.cos(math.pi * t / period)
    return s * np.stack([np.sin(math.pi * x) ** 2 * np.sin(2 * math.pi * y),
                         -np.sin(math.pi * y) ** 2 * np.sin(2 * math.pi * x)], axis=1)


def sine_compression(amp):
    """Non-solenoidal field u_a = amp_a sin(pi x_a), one axis at a time:
    tangential on the unit box boundary, div u = pi sum_a amp_a cos(pi x_a)
    (compression where it is negative, expansion where positive)."""
    amp = tuple(float(v) for v in amp)

    def f(p, t=0.0):
        return np.stack([amp[a] * np.sin(math.pi * p[:, a]) for a in range(len(amp))], axis=1)
    return f


def compressible_swirl_3d(p, t=0.0, squeeze=0.3):
    """The 3D swirl plus a sine compression of amplitude ``squeeze`` on
    every axis (non-solenoidal, tangential on the unit cube boundary)."""
    return swirl_3d(p, t) + sine_compression((squeeze,) * 3)(p, t)


def constant_field(vec):
    vec = np.asarray(vec, dtype=np.float64)

    def f(p, t=0.0):
        return np.broadcast_to(vec, p.shape).copy()
    return f


def fourier_modes_field(dim, seed, n_modes=4):
    """Sum of ``n_modes`` divergence-free modes a_m curl(psi_m e_alpha) with
    psi_m = prod_axes sin(k_axis pi x_axis), k in {1,2,3}, a_m ~ N(0,1);
    tangential on the unit box boundary."""
    rng = np.random.default_rng(seed)
    modes = []
    for _ in range(n_modes):
        k = rng.integers(1, 4, size=dim)
        amp = rng.standard_normal()
        alpha = 2 if dim == 2 else int(rng.integers(0, 3))
        modes.append((k, amp, alpha))

    def f(p, t=0.0):
        out = np.zeros_like(p)
        for k, amp, alpha in modes:
            s = [np.sin(k[a] * math.pi * p[:, a]) for a in range(dim)]
            c = [k[a] * math.pi * np.cos(k[a] * math.pi * p[:, a]) for a in range(dim)]
            if dim == 2:
                # curl(psi e_z) = (d psi/dy, -d psi/dx)
                out[:, 0] += amp * s[0] * c[1]
                out[:, 1] += -amp * c[0] * s[1]
            else:
                psi_d = []
                for a in range(3):
                    term = c[a].copy()
                    for b in range(3):
                        if b != a:
                            term = term * s[b]
                    psi_d.append(term)
                # curl(psi e_alpha): e_alpha x ... written component-wise
                if alpha == 0:
                    out[:, 1] += amp * psi_d[2]
                    out[:, 2] += -amp * psi_d[1]
                elif alpha == 1:
                    out[:, 0] += -amp * psi_d[2]
                    out[:, 2] += amp * psi_d[0]
                else:
                    out[:, 0] += amp * psi_d[1]
                    out[:, 1] += -amp * psi_d[0]
        return out
    return f


# --------------------------------------------------------------------------
# initial concentrations and porosity
# --------------------------------------------------------------------------

def disk_indicator(mesh, centre, radius):
    """c^0 = 1 on cells whose centroid is within ``radius`` of ``centre``."""
    x = cell_centroids(mesh)
    d2 = np.sum((x - np.asarray(centre)) ** 2, axis=1)
    return (d2 < radius * radius).astype(np.float64)


def uniform_c(mesh, seed):
    return np.random.default_rng(seed).uniform(0.0, 1.0, n_cells(mesh))


def lognormal_phi(n_cells, seed, sigma=0.5, lo=0.05, hi=1.0):
    z = np.random.default_rng(seed).standard_normal(n_cells)
    return np.clip(np.exp(sigma * z), lo, hi)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def solid_body_32():
    """2D solid-body rotation: unit square, 32 x 32 cells, phi = 1,
    u = 2 pi (-(y-1/2), x-1/2), c^0 = indicator of the disk of radius 0.15
    at (0.5, 0.75), dt = 0.01, 10 steps (velocity time independent)."""
    mesh = cartesian_mesh((32, 32))
    vel = sample_velocity(mesh, solid_body_2d)
    c0 = disk_indicator(mesh, (0.5, 0.75), 0.15)
    return {"name": "solid_body_2d_32x32", "mesh": mesh, "vel_fn": lambda step: vel,
            "c0": c0, "dt": 0.01, "steps": 10, "time_dependent": False}


def swirl_hex(n=64, steps=None):
    """3D swirl on the unit cube, n^3 hexahedra, phi = 1, dt = 1/128, the
    field sampled at t^{n+1/2} each step, c^0 = indicator of the ball of
    radius 0.15 at (0.35, 0.35, 0.35); 128 steps reach t = 1 where the
    flow has returned."""
    mesh = cartesian_mesh((n, n, n))
    dt = 1.0 / 128.0

    def vel_fn(step):
        return sample_velocity(mesh, lambda p, t: swirl_3d(p, t), (step + 0.5) * dt)
    c0 = disk_indicator(mesh, (0.35, 0.35, 0.35), 0.15)
    return {"name": f"swirl_hex_{n}^3", "mesh": mesh, "vel_fn": vel_fn, "c0": c0, "dt": dt,
            "steps": 128 if steps is None else steps, "time_dependent": True}


def compressible_swirl_hex(n=64, steps=None, squeeze=0.3):
    """``swirl_hex`` with the sine compression of amplitude ``squeeze`` added
    on every axis (a non-solenoidal field, tangential on the walls; the
    swirl part reverses with cos(pi t), the compression does not)."""
    mesh = cartesian_mesh((n, n, n))
    dt = 1.0 / 128.0

    def vel_fn(step):
        return sample_velocity(mesh, lambda p, t: compressible_swirl_3d(p, t, squeeze),
                               (step + 0.5) * dt)
    c0 = disk_indicator(mesh, (0.35, 0.35, 0.35), 0.15)
    return {"name": f"compressible_swirl_hex_{n}^3", "mesh": mesh, "vel_fn": vel_fn, "c0": c0,
            "dt": dt, "steps": 128 if steps is None else steps, "time_dependent": True}


def porous_swirl_hex(n=32, seed=5834, steps=20):
    """3D swirl with a lognormal porosity phi = clip(exp(0.5 Z), 0.05, 1)
    per cell, c^0 ~ U[0,1]; exercises the tracked-radius rule for
    non-constant phi."""
    nc = n ** 3
    mesh = cartesian_mesh((n, n, n), phi=lognormal_phi(nc, seed))
    dt = 1.0 / 128.0

    def vel_fn(step):
        return sample_velocity(mesh, lambda p, t: swirl_3d(p, t), (step + 0.5) * dt)
    c0 = uniform_c(mesh, 33)
    return {"name": f"porous_swirl_hex_{n}^3", "mesh": mesh, "vel_fn": vel_fn, "c0": c0,
            "dt": dt, "steps": steps, "time_dependent": True}


def mixed_problem(p, n_lo=4.0e3, n_hi=2.0e5, steps=10):
    """Problem ``p`` of a batch of independent small problems (seed p): a 2D
    triangulated unit square (each of n^2 squares cut along the same
    diagonal, 2 n^2 triangles, one centroid ball of equal measure) or a 3D
    cube of n^3 hexahedra (8 sub-cell balls), with probability 1/2 each;
    about N ~ logU[n_lo, n_hi] cells (n = round(sqrt(N / 2)) or
    round(N^(1/3))); phi = 1; u the sum of four divergence-free Fourier
    modes (seed p); dt such that dt max over cell centroids |u| / h is a
    CFL number drawn from U[0.5, 4]; c^0 ~ U[0, 1]; the transfer is built
    once and applied ``steps`` times (u does not depend on time)."""
    rng = np.random.default_rng(p)
    tri = bool(rng.random() < 0.5)
    N = math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))
    cfl = float(rng.uniform(0.5, 4.0))
    if tri:
        n = max(2, int(round(math.sqrt(N / 2.0))))
        mesh = triangulated_square(n, 0.0, p)
        dim, layout = 2, "equal_measure"
    else:
        n = max(2, int(round(N ** (1.0 / 3.0))))
        mesh = cartesian_mesh((n, n, n))
        dim, layout = 3, "subcell"
    field = fourier_modes_field(dim, seed=p)
    u0 = field(cell_centroids(mesh))
    umax = float(np.max(np.sqrt(np.sum(u0 ** 2, axis=1))))
    h = 1.0 / n
    dt = cfl * h / umax
    vel = sample_velocity_grid((n,) * dim, field)
    return {"name": f"mixed_{p}_{'tri' if tri else 'hex'}_{n}", "mesh": mesh, "layout": layout,
            "vel": vel, "dt": dt, "cfl": cfl, "c0": uniform_c(mesh, 100000 + p),
            "steps": steps, "time_dependent": False}


def jittered_tets(n=96, jitter=0.1, seed=1908, phi_seed=5834, cfl=4.0, steps=20):
    """3D unstructured workload: n^3 cubes split into 6 Kuhn tetrahedra
    (6 n^3 cells), interior vertices jittered by up to 10 % of h, phi =
    clip(exp(0.5 Z), 0.05, 1) per cell, the swirl scaled so that the CFL
    number of the characteristic speed, dt max over cell centroids of
    (|u| / phi_K) / h, is ``cfl``; c^0 ~ U[0,1], dt = 1/128."""
    nc = 6 * n ** 3
    mesh = kuhn_tets(n, jitter, seed, phi=lognormal_phi(nc, phi_seed))
    dt = 1.0 / 128.0
    h = 1.0 / n
    u0 = swirl_3d(cell_centroids(mesh), 0.0)
    umax = float(np.max(np.sqrt(np.sum(u0 ** 2, axis=1)) / mesh["phi"]))
    amp = cfl * h / (umax * dt)

    def vel_fn(step):
        return sample_velocity_grid((n, n, n), lambda p, t: swirl_3d(p, t, amplitude=amp),
                                    (step + 0.5) * dt)
    c0 = uniform_c(mesh, 33)
    return {"name": f"jittered_tets_{n}", "mesh": mesh, "vel_fn": vel_fn, "c0": c0, "dt": dt,
            "steps": steps, "time_dependent": True}


# --------------------------------------------------------------------------
# caller-chosen balls (layout "custom")
# --------------------------------------------------------------------------

def random_subcell_balls(mesh, seed):
    """Balls of a Cartesian mesh chosen at random, as a caller might: every
    cell gets, with even odds, one ball near its centre or 2^d balls near
    its sub-cell centres (each centre moved by up to 1/32 of the cell per
    axis, radius U(0.9, 1) times the distance to the boundary of the cell or
    sub-cell), so a cell's balls are disjoint and strictly inside it.
    Returns the mesh dict extended with ``ball_centres``, ``ball_radii``,
    ``ball_cell``."""
    rng = np.random.default_rng(seed)
    n, o, h = mesh["n"], np.asarray(mesh["origin"]), np.asarray(mesh["h"])
    dim = len(n)
    nc = int(np.prod(n))
    ids = np.arange(nc)
    ijk = np.empty((nc, dim))
    rem = ids.copy()
    for a in range(dim):
        ijk[:, a] = rem % n[a]
        rem //= n[a]
    cen, rad, cell = [], [], []
    for K in range(nc):
        if rng.uniform() < 0.5:
            fracs, half = [np.full(dim, 0.5)], 0.5
        else:
            fracs = [np.array([0.25 + 0.5 * ((s >> a) & 1) for a in range(dim)])
                     for s in range(2 ** dim)]
            half = 0.25
        for frac in fracs:
            jit = rng.uniform(-1.0 / 32, 1.0 / 32, dim)
            cen.append(o + (ijk[K] + frac + jit) * h)
            rad.append(np.min(h * (half - np.abs(jit))) * rng.uniform(0.9, 1.0))
            cell.append(K)
    out = dict(mesh)
    out["ball_centres"] = np.array(cen)
    out["ball_radii"] = np.array(rad)
    out["ball_cell"] = np.array(cell, dtype=np.int32)
    return out


def corner_balls_simplex(mesh, shrink=0.9):
    """d + 1 balls per simplex, as a caller might place them: one per
    vertex, centred half way from the centroid G to the vertex, each with
    the measure of |K| / (d + 1) times ``shrink``^d (the balls of a cell may
    overlap each other and the neighbours')."""
    V, Cc = mesh["vertices"], mesh["cells"]
    dim = V.shape[1]
    P = V[Cc]                                   # (nc, d+1, dim)
    G = P.mean(axis=1)
    if dim == 2:
        vol = 0.5 * np.abs((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                           - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0]))
        r = shrink * np.sqrt(vol / (3 * math.pi))
    else:
        e = P[:, 1:, :] - P[:, :1, :]
        vol = np.abs(np.linalg.det(e)) / 6.0
        r = shrink * np.cbrt(3.0 * vol / (4 * 4.0 * math.pi))
    cen = 0.5 * (G[:, None, :] + P)
    out = dict(mesh)
    out["ball_centres"] = cen.reshape(-1, dim)
    out["ball_radii"] = np.repeat(r, dim + 1)
    out["ball_cell"] = np.repeat(np.arange(Cc.shape[0], dtype=np.int32), dim + 1)
    return out
