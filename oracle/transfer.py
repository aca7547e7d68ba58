"""Oracle, algebraic part: V, the scaling sweeps, apply, mass, one full step.

Test infrastructure only (see ``oracle/__init__.py``).  Plain NumPy/SciPy,
binary64.

A sparse matrix is kept as CSR arrays ``(row_ptr, col, val)`` with the
columns of each row strictly ascending; row i is the tracked cell K_i and
column j the residing cell M_j (Sec. 3.2).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from . import geometry as geo
from .qp import solve_mass_qp


class VoidRowError(RuntimeError):
    """A tracked ball overlaps no residing ball: the denominator of
    eq. fracMaterial is zero and its mass cannot be placed."""

    def __init__(self, ball, cell):
        super().__init__(f"tracked ball {ball} of cell {cell} meets no residing ball")
        self.ball, self.cell = ball, cell


class VoidColumnError(RuntimeError):
    """Column j of A^(0) sums to zero (Sec. 3.2: no tracked ball reaches a
    ball of M_j), so the column scaling of eq. volAdj is undefined."""

    def __init__(self, col):
        super().__init__(f"residing cell {col} receives no tracked ball")
        self.col = col


def csr_from_coo(nrows, rows, cols, vals):
    """Sum duplicate (row, col) entries; columns ascending within rows."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    ncols = int(cols.max()) + 1 if cols.size else 1
    key = rows * ncols + cols
    uniq, inv = np.unique(key, return_inverse=True)
    v = np.zeros(uniq.size, dtype=np.float64)
    np.add.at(v, inv, vals)
    r = uniq // ncols
    c = uniq % ncols
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, c.astype(np.int64), v


def csr_rows(row_ptr):
    """Row index of every stored entry."""
    return np.repeat(np.arange(row_ptr.size - 1, dtype=np.int64), np.diff(row_ptr))


# --------------------------------------------------------------------------
# Sec. 3.1: initial approximation V
# --------------------------------------------------------------------------

def tracked_ball_mass(ball_cell, radii, rho, phi, dim, lam=None):
    """rho_K phi_hat_{K,s} |B_hat_{K,s}| of every tracked ball.

    Solenoidal u: rho_K phi_K |B_{K,s}| (eq. expPhiB).  Otherwise that
    times exp(Lambda_{K,s}), Lambda from ``geometry.log_growth`` (the
    analogue of eq. expPhiB, Sec. 3.2, Remark on non-solenoidal fields),
    the product taken in that order.
    """
    ball_cell = np.asarray(ball_cell, dtype=np.int64)
    m = rho[ball_cell] * phi[ball_cell] * geo.ball_measure(radii, dim)
    if lam is not None:
        m = m * np.exp(np.asarray(lam, dtype=np.float64))
    return m


def row_targets(nc, ball_cell, ball_mass, b, rows, cols):
    """Row targets of a non-solenoidal step: |F_{-dt}(K)|_phi.

    eq. volTracked gives T_K = sum_s rho_K phi_hat_{K,s} |B_hat_{K,s}| (the
    balls of K in order).  The trace-back regions of all cells cover the
    domain once, so the exact targets of any set of tracked cells that
    takes its material from a set of residing cells alone total the
    porous volume of those residing cells.  The sets are the connected
    components of the bipartite graph of V's pattern (row K -- column M
    for every entry); within a component T is rescaled by
    sum_{M in it} |M|_phi / sum_{K in it} T_K (both correctly rounded):
    b_loc[K] = T_K * scale(component of K).  Without that the constraints
    of eq. opti_masscons would be inconsistent on every component.
    Returns (b_loc, T, scale of the whole domain, number of components).
    """
    T = np.zeros(nc)
    for a in range(ball_mass.size):
        T[ball_cell[a]] = T[ball_cell[a]] + ball_mass[a]
    g = sp.coo_matrix((np.ones(len(rows)), (np.asarray(rows), nc + np.asarray(cols))),
                      shape=(2 * nc, 2 * nc))
    ncomp, lab = connected_components(g, directed=False)
    b_loc = np.empty(nc)
    for c in range(ncomp):
        R = np.nonzero(lab[:nc] == c)[0]
        Cc = np.nonzero(lab[nc:] == c)[0]
        sc = math.fsum(np.asarray(b)[Cc].tolist()) / math.fsum(T[R].tolist())
        b_loc[R] = T[R] * sc
    scale = math.fsum(np.asarray(b).tolist()) / math.fsum(T.tolist())
    return b_loc, T, scale, ncomp


def initial_volumes(nc, dim, ball_cell, centres, radii, rho, phi,
                    traced, r_hat, ia, ib, precision="fp64", lam=None, ghost=None):
    """V_{K_hat, M} of eq. ball_int, as CSR.

    For a candidate pair (tracked ball a of cell K, residing ball b of cell
    M) the weight is omega = rho_M phi_M |B_hat_a cap B_b| (Remark
    porousBallInt).  S_a = sum of omega over the pairs of a is the
    denominator of eq. fracMaterial.  The tracked ball carries the porous
    mass rho_K phi_hat |B_hat| (``tracked_ball_mass``: rho_K phi_K |B_a|
    for a solenoidal u, eq. expPhiB), and that mass is split over the
    residing balls in the ratios omega / S_a; V_{K,M} sums those shares
    over the balls of K and of M.

    ``precision="fp32"`` (FP32-volume mode) rounds centres and radii to
    binary32 before the distance and the lens, which are then evaluated in
    binary64 on those rounded inputs.
    """
    ball_cell = np.asarray(ball_cell, dtype=np.int64)
    phi = np.asarray(phi, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    if precision == "fp32":
        def rd(x):
            return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    else:
        def rd(x):
            return np.asarray(x, dtype=np.float64)
    tc, rc = rd(traced), rd(centres)
    r1, r2 = rd(r_hat)[ia], rd(radii)[ib]
    d = np.sqrt(np.sum((tc[ia] - rc[ib]) ** 2, axis=1))
    lens = geo.lens_measure(r1, r2, d, dim)
    cb = ball_cell[ib]
    ca = ball_cell[ia]
    omega = rho[cb] * phi[cb] * lens
    nballs = ball_cell.size
    S = np.bincount(ia, weights=omega, minlength=nballs)
    bad = S <= 0.0
    if ghost is not None:
        # a ghost cell's ball tracked into nothing carries its mass out of
        # the problem (Sec. 3.2, Remark on inflow and outflow)
        bad &= ~np.asarray(ghost)[ball_cell]
    void = np.nonzero(bad)[0]
    if void.size:
        raise VoidRowError(int(void[0]), int(ball_cell[void[0]]))
    mass = tracked_ball_mass(ball_cell, radii, rho, phi, dim, lam)
    share = mass[ia] * omega / S[ia]
    return csr_from_coo(nc, ca, cb, share)


# --------------------------------------------------------------------------
# Sec. 3.2: mass adjustment sweeps, eq. volAdj
# --------------------------------------------------------------------------

def scaling_sweeps(row_ptr, col, val, b_loc, b_glob, n_sweeps, active=None):
    """A^(N) from A^(0) = V by N sweeps of eq. volAdj.

    Each sweep first scales every column j to sum |M_j|_phi, then every row
    i to sum |F_{-dt}(K_i)|_phi (= |K_i|_phi for solenoidal u, eq.
    exactVol_traceback).  Rows therefore hold exactly after every sweep.
    ``active`` (per cell, optional): only those rows and columns are scaled
    (ghost cells have no target).
    """
    a = np.array(val, dtype=np.float64, copy=True)
    rows = csr_rows(row_ptr)
    nc = row_ptr.size - 1
    act = None if active is None else np.asarray(active, dtype=bool)
    for _ in range(int(n_sweeps)):
        cs = np.bincount(col, weights=a, minlength=nc)
        bad = cs <= 0.0 if act is None else (cs <= 0.0) & act
        if np.any(bad):
            raise VoidColumnError(int(np.nonzero(bad)[0][0]))
        if act is None:
            a = a * (np.asarray(b_glob)[col] / cs[col])
        else:
            with np.errstate(divide="ignore", invalid="ignore"):
                a = a * np.where(act[col], np.asarray(b_glob)[col] / cs[col], 1.0)
        rs = np.bincount(rows, weights=a, minlength=nc)
        if act is None:
            a = a * (np.asarray(b_loc)[rows] / rs[rows])
        else:
            with np.errstate(divide="ignore", invalid="ignore"):
                a = a * np.where(act[rows], np.asarray(b_loc)[rows] / rs[rows], 1.0)
    return a


def check_columns(col, val, nc, active=None):
    cs = np.bincount(col, weights=val, minlength=nc)
    bad = cs <= 0.0 if active is None else (cs <= 0.0) & np.asarray(active)
    if np.any(bad):
        raise VoidColumnError(int(np.nonzero(bad)[0][0]))


# --------------------------------------------------------------------------
# Sec. 2: the update and the mass
# --------------------------------------------------------------------------

def apply(row_ptr, col, val, b_loc, c):
    """c^{n+1}_K = (1/|K|_phi) sum_M |M cap F_{-dt}(K)|_phi c^n_M
    (eq. phys-inter-ELLAM) with the final volumes as the matrix."""
    rows = csr_rows(row_ptr)
    c = np.asarray(c, dtype=np.float64)
    num = np.bincount(rows, weights=np.asarray(val) * c[col], minlength=row_ptr.size - 1)
    return num / np.asarray(b_loc, dtype=np.float64)


def mass(phi, cell_vol, c, active=None):
    """sum_K phi_K |K| c_K (Sec. 2.1), correctly rounded (math.fsum); over
    the ``active`` cells only when given (the domain without its ghost
    cells)."""
    terms = np.asarray(phi, dtype=np.float64) * np.asarray(cell_vol, dtype=np.float64) \
        * np.asarray(c, dtype=np.float64)
    if active is not None:
        terms = terms[np.asarray(active, dtype=bool)]
    return math.fsum(terms.tolist())


def ghost_cells(n, n_ghost):
    """Ghost flag of every cell of a Cartesian grid of n cells per axis
    (ids x-fastest): the cells within n_ghost of the grid's boundary."""
    dim = len(n)
    ids = np.indices(tuple(int(v) for v in n[::-1])).reshape(dim, -1)[::-1]
    g = np.zeros(ids.shape[1], dtype=bool)
    for a in range(dim):
        g |= (ids[a] < n_ghost) | (ids[a] >= int(n[a]) - n_ghost)
    return g


# --------------------------------------------------------------------------
# One time step of Algorithm 1 plus the update
# --------------------------------------------------------------------------

def build_transfer(mesh, vel, dt, layout="subcell", n_sweeps=10, substeps=1,
                   precision="fp64", box_policy="paper_then_relax", stop_after="all",
                   traced_override=None, balls_override=None, qp_tol=1e-14,
                   solenoidal=True, n_ghost=0):
    """Transfer matrix of one time step: Algorithm 1 of Sec. 3.3.

    ``mesh``: dict with ``n``, ``origin``, ``h`` (Cartesian) or ``kind =
    "simplex"``, ``vertices``, ``cells``, and ``phi`` (per cell).  ``vel``: velocity lattice dict (``m``, ``origin``,
    ``spacing``, ``u``).  Returns a dict holding every intermediate stage.
    ``traced_override`` replaces the tracked centres and ``balls_override``
    = (centres, radii) the residing balls of the layout (to compare the
    later stages on identical geometry); rho_K follows the given radii.

    ``solenoidal=False`` (Sec. 3.2, Remark on non-solenoidal fields): r_hat
    from the cardinal points whatever phi (eq. rTrackedBall), the tracked
    ball masses from ``geometry.log_growth`` (``tracked_ball_mass``), and
    the row targets from eq. volTracked (``row_targets``) instead of
    |K|_phi; the column targets stay |M|_phi and the update still divides
    by |K|_phi (eq. phys-inter-ELLAM).

    ``n_ghost > 0`` (Cartesian meshes; Sec. 3.2, Remark on inflow and
    outflow, option b): the grid's outer ``n_ghost`` layers are ghost cells.
    They carry balls and are tracked like the others, but their rows and
    columns have no target: they are not scaled, the least-change problem
    constrains the interior cells' rows and columns only (the ghost cells'
    multipliers stay 0), and a ghost ball tracked into nothing or a ghost
    column that nothing reaches is no void.  Material then enters the
    interior from ghost cells (whose concentrations are the inflow data)
    and leaves it into ghost cells.
    """
    dim = geo.mesh_dim(mesh)
    nc = geo.mesh_n_cells(mesh)
    phi = np.asarray(mesh["phi"], dtype=np.float64)
    if phi.shape != (nc,) or not np.all(np.isfinite(phi)) or np.any(phi <= 0):
        raise ValueError("phi must be finite and > 0 on every cell (Sec. 1.2)")
    if geo.is_simplex(mesh):
        if layout not in ("equal_measure", "custom", "packed"):
            raise ValueError("simplicial meshes take the equal_measure, packed or custom layout")
        kvol = geo.simplex_volumes(mesh["vertices"], mesh["cells"])
        if layout == "equal_measure":
            centres, radii, bcell = geo.simplex_ball_layout(mesh)
        elif layout == "packed":
            centres, radii, bcell = geo.simplex_packed_layout(mesh)
    else:
        n = tuple(int(v) for v in mesh["n"])
        h = tuple(float(v) for v in mesh["h"])
        kvol = np.full(nc, geo.cell_volume(h))
        if layout != "custom":
            centres, radii, bcell = geo.ball_layout(n, mesh["origin"], h, layout)
    if layout == "custom":
        # the caller's balls (Sec. 3: any points C_{K,s} inside K with radii)
        centres = np.asarray(mesh["ball_centres"], dtype=np.float64)
        radii = np.asarray(mesh["ball_radii"], dtype=np.float64)
        bcell = np.asarray(mesh["ball_cell"], dtype=np.int64)
    if balls_override is not None:
        centres = np.asarray(balls_override[0], dtype=np.float64).reshape(centres.shape)
        radii = np.asarray(balls_override[1], dtype=np.float64).reshape(radii.shape)
    rho = geo.porous_density(nc, kvol, radii, bcell, dim)
    b = phi * kvol                      # |K|_phi = b_loc = b_glob (eq. exactVol_traceback)
    out = {"centres": centres, "radii": radii, "ball_cell": bcell, "rho": rho, "b": b,
           "cell_vol": kvol}
    ghost = active = None
    if n_ghost:
        if geo.is_simplex(mesh) or not solenoidal:
            raise ValueError("ghost cells: Cartesian meshes and solenoidal steps")
        ghost = ghost_cells(mesh["n"], int(n_ghost))
        active = ~ghost
    out["ghost"] = ghost
    lam = None
    if solenoidal:
        if traced_override is None:
            traced = geo.trace_points(centres, mesh, vel, dt, substeps)
        else:
            traced = np.asarray(traced_override, dtype=np.float64)
    else:
        if traced_override is not None:
            raise ValueError("a non-solenoidal step tracks its own centres")
        traced, lam = geo.log_growth(centres, mesh, vel, dt, substeps)
    out["lam"] = lam
    r_hat = geo.tracked_radius(centres, radii, traced, mesh, vel, dt, substeps,
                               solenoidal=solenoidal)
    out["traced"], out["r_hat"] = traced, r_hat
    ia, ib = geo.candidate_pairs(traced, r_hat, centres, radii, precision=precision)
    out["pairs"] = (ia, ib)
    if stop_after == "pairs":
        return out
    rp, cl, V = initial_volumes(nc, dim, bcell, centres, radii, rho, phi, traced, r_hat,
                                ia, ib, precision=precision, lam=lam, ghost=ghost)
    out["row_ptr"], out["col"], out["V"] = rp, cl, V
    if solenoidal:
        b_loc = b
    else:
        bm = tracked_ball_mass(bcell, radii, rho, phi, dim, lam)
        b_loc, out["T"], out["target_scale"], out["n_groups"] = \
            row_targets(nc, bcell, bm, b, csr_rows(rp), cl)
    out["b_loc"] = b_loc
    if stop_after == "v":
        return out
    check_columns(cl, V, nc, active)
    AN = scaling_sweeps(rp, cl, V, b_loc, b, n_sweeps, active)
    out["AN"] = AN
    if stop_after == "sinkhorn":
        return out
    res = solve_mass_qp(csr_rows(rp), cl, AN, b_loc, b, box_policy=box_policy, tol=qp_tol,
                        active=active)
    out["qp"] = res
    out["A"] = AN * (1.0 + res["x"])
    return out


def run(mesh, vel_fn, c0, dt, steps, **kw):
    """``steps`` time steps; ``vel_fn(step)`` returns the velocity lattice
    of the interval (t^n, t^{n+1}).  Returns the list of concentrations."""
    cs = [np.asarray(c0, dtype=np.float64)]
    for s in range(steps):
        T = build_transfer(mesh, vel_fn(s), dt, **kw)
        cs.append(apply(T["row_ptr"], T["col"], T["A"], T["b"], cs[-1]))
    return cs
