"""Oracle: the least-change bounded problem of Sec. 3.2 (eq. opti_masscons).

Test infrastructure only (see ``oracle/__init__.py``).

Statement.  One unknown x_k per stored entry a_k of A^(N) (the paper
writes x as indexed by cells, which cannot be meant: A_hat has n_z
columns, so x has n_z entries, one per nonzero).  Minimise x^T x subject to

    sum_{k in row i} a_k (1 + x_k) = b_row[i]      (local, eq. localmassconsMat)
    sum_{k in col j} a_k (1 + x_k) = b_col[j]      (global, eq. globalmassconsMat)
    lo <= x_k <= hi.

The paper asks for 1 + x positive and at most 2.  Read as the closed box
-1 <= x <= 1 (a strictly convex objective over a closed convex set has a
unique minimiser; an open bound would have none when it is active).  The
box can be infeasible (a tracked cell that must take more than twice what
it overlaps); ``box_policy="paper_then_relax"`` then drops the upper cap
(level 1: x >= -1, volumes stay non-negative) and, if that is still
infeasible, keeps the equalities alone (level 2).  ``"strict"`` raises
``QPInfeasible`` instead.

Method.  The minimiser is unique, so any exact method yields it.  This one
works on the dual: with multipliers mu (rows) and nu (columns), the
stationarity condition gives x_k = clip(a_k (mu_i + nu_j), lo, hi); the
dual function theta(mu, nu) = sum_k psi(a_k (mu_i + nu_j)) - mu.r - nu.s
(psi' = clip) is convex and C^1, its gradient is the constraint residual,
and it is minimised by a damped semismooth Newton method whose linear
systems are solved directly (SuperLU), with an Armijo backtracking line
search.  The returned x is *defined* as clip(A_hat^T lambda), so it
satisfies stationarity and the bounds exactly; ``verify_kkt`` then checks
primal feasibility, which together certify optimality.  Feasibility of a
box level, when Newton does not converge, is decided by a linear program
(HiGHS).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.optimize import linprog

BOX_LEVELS = {0: (-1.0, 1.0), 1: (-1.0, np.inf), 2: (-np.inf, np.inf)}


class QPInfeasible(RuntimeError):
    pass


class QPNotConverged(RuntimeError):
    pass


def constraint_matrix(row_ptr, col, val, n_cols):
    """A_hat (2 n_c x n_z) of Sec. 3.2, built as the paper describes it.

    The nonzeros of each row of A^(N) are laid side by side (row i's
    entries occupy the unknown slots row_ptr[i] .. row_ptr[i+1]-1, in
    ascending column order): the first n_c rows of A_hat carry row i's
    entries on its slots; row n_c + j carries, on the slot of every entry
    a_{i,j} of column j, that same value.  Returned dense (small cases)."""
    nr = len(row_ptr) - 1
    nz = len(val)
    Ah = np.zeros((nr + n_cols, nz))
    for i in range(nr):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            Ah[i, k] = val[k]
            Ah[nr + col[k], k] = val[k]
    return Ah


def constraint_rhs(rows, cols, a, b_row, b_col):
    """r, s: what sum a_k x_k must equal on each row / column."""
    nr, nc = len(b_row), len(b_col)
    r = np.asarray(b_row, dtype=np.float64) - np.bincount(rows, weights=a, minlength=nr)
    s = np.asarray(b_col, dtype=np.float64) - np.bincount(cols, weights=a, minlength=nc)
    return r, s


def residual(rows, cols, a, x, r, s):
    nr, nc = r.size, s.size
    ax = a * x
    return np.concatenate([np.bincount(rows, weights=ax, minlength=nr) - r,
                           np.bincount(cols, weights=ax, minlength=nc) - s])


def _dpsi(t, d, lo, hi):
    """psi(t + d) - psi(t), where psi is the primitive of clip(., lo, hi)
    vanishing at 0, evaluated without cancelling large terms: psi(u) =
    c^2/2 + c (u - c) with c = clip(u)."""
    u = t + d
    c1 = np.clip(t, lo, hi)
    c2 = np.clip(u, lo, hi)
    free1 = c1 == t
    free2 = c2 == u
    out = 0.5 * (c2 * c2 - c1 * c1) + c2 * np.where(free2, 0.0, u - c2) \
        - c1 * np.where(free1, 0.0, t - c1)
    both = free1 & free2
    out[both] = d[both] * (t[both] + 0.5 * d[both])
    same = (~free1) & (~free2) & (c1 == c2)
    out[same] = c1[same] * d[same]
    return out


def feasible_lp(rows, cols, a, b_row, b_col, lo, hi, active=None):
    """Is {lo <= x <= hi, row/col sums of a(1+x) = b} non-empty?  Decided
    with an LP on y = a(1+x) >= 0 plus slacks: minimise the total slack.
    ``active`` (per cell, optional): only those rows and columns are
    constrained."""
    nz = a.size
    nr, nc = len(b_row), len(b_col)
    ylo = a * (1.0 + lo) if np.isfinite(lo) else np.full(nz, -np.inf)
    yhi = a * (1.0 + hi) if np.isfinite(hi) else np.full(nz, np.inf)
    # A_eq [y; sp; sm] = b with sp, sm >= 0
    E = sp.vstack([
        sp.csr_matrix((np.ones(nz), (rows, np.arange(nz))), shape=(nr, nz)),
        sp.csr_matrix((np.ones(nz), (cols, np.arange(nz))), shape=(nc, nz)),
    ]).tocsr()
    beq_all = np.concatenate([b_row, b_col])
    if active is not None:
        keep = np.concatenate([np.asarray(active), np.asarray(active)])
        E = E[keep]
        b_row, b_col = beq_all[keep], np.zeros(0)
    m = E.shape[0]
    I = sp.identity(m, format="csr")
    Aeq = sp.hstack([E, I, -I]).tocsr()
    beq = np.concatenate([b_row, b_col])
    cvec = np.concatenate([np.zeros(nz), np.ones(2 * m)])
    bounds = [(ylo[k] if np.isfinite(ylo[k]) else None,
               yhi[k] if np.isfinite(yhi[k]) else None) for k in range(nz)]
    bounds += [(0, None)] * (2 * m)
    res = linprog(cvec, A_eq=Aeq, b_eq=beq, bounds=bounds, method="highs")
    if res.status != 0:
        raise RuntimeError("feasibility LP failed: " + res.message)
    scale = max(float(np.max(np.abs(beq))), 1e-300)
    return res.fun <= 1e-9 * scale, res.fun


def _cell_coordinates_matrix(rows, cols, w, nr):
    """Newton matrix in per-cell coordinates.

    In the multipliers y = (mu, -nu) the Newton matrix is the graph
    Laplacian of the bipartite graph rows-columns with weights w.  Cells
    that barely move couple their row and column by a weight near 1 and to
    everything else by slivers; their "gauge" (mu_K up, nu_K down) is then a
    near-null mode whose eigenvalue is lost to rounding when the Laplacian
    diagonal is formed as a sum including the large weight.  The change of
    variables s_K = (y_rK + y_cK)/2, g_K = y_rK - y_cK (rows and columns are
    both indexed by cells) keeps that mode: an entry (K, M) contributes
    w v v^T with v = e_sK - e_sM + (e_gK + e_gM)/2 for K != M and v = e_gK
    for K = M, so the s block is assembled from the off-diagonal weights
    alone.  Unknowns: s_0..s_{n-1}, g_0..g_{n-1}."""
    off = rows != cols
    di = ~off
    ro, co, wo = rows[off], cols[off], w[off]
    parts = [(ro, 1.0), (co, -1.0), (nr + ro, 0.5), (nr + co, 0.5)]
    I, J, V = [], [], []
    for pi, ci in parts:
        for pj, cj in parts:
            I.append(pi)
            J.append(pj)
            V.append(wo * (ci * cj))
    I.append(nr + rows[di])
    J.append(nr + rows[di])
    V.append(w[di])
    return sp.csr_matrix((np.concatenate(V), (np.concatenate(I), np.concatenate(J))),
                         shape=(2 * nr, 2 * nr))


def _newton(rows, cols, a, r, s, lo, hi, tol, max_iter, active=None):
    """Damped semismooth Newton on the dual; inputs already scaled so that
    max |b| = 1.  Returns (x, t, mu, nu, residual_inf, iterations, ok).

    t_k = a_k (mu_i + nu_j) is carried entry by entry and updated by the
    increments a_k (dmu_i + dnu_j): weakly coupled cells give multipliers
    of very different sizes, and recomputing t from them would cancel
    digits.  Each Newton system J d = -F (J = A_hat diag(free) A_hat^T) is
    solved in the per-cell coordinates of ``_cell_coordinates_matrix``
    (symmetrically scaled to unit diagonal, a relative 1e-14 diagonal shift
    for the exactly singular directions, sparse LU, two refinement steps).
    The increments of t are formed from (s, g) directly: a_k g_K for the
    diagonal entry of cell K, a_k ((s_K - s_M) + (g_K + g_M)/2) otherwise.
    The step length is chosen by Armijo backtracking on theta, whose change
    is summed entry by entry (psi differences) rather than as a difference
    of two large totals.
    """
    nr, nc = r.size, s.size
    assert nr == nc, "rows and columns are both indexed by cells"
    # cells whose row and column are unconstrained (ghost cells) keep
    # multipliers 0: their residuals are dropped and their (s, g) unknowns
    # removed from every Newton system
    act = np.ones(nr, dtype=bool) if active is None else np.asarray(active, dtype=bool)
    act2 = np.concatenate([act, act])
    keep = np.nonzero(act2)[0]

    def resid(x):
        return np.where(act2, residual(rows, cols, a, x, r, s), 0.0)

    mu = np.zeros(nr)
    nu = np.zeros(nc)
    t = np.zeros(a.size)
    rs = np.where(act2, np.concatenate([r, s]), 0.0)
    off = rows != cols
    a2 = a * a
    x = np.clip(t, lo, hi)
    F = resid(x)
    for it in range(1, max_iter + 1):
        fn = float(np.max(np.abs(F)))
        if fn <= tol:
            return x, t, mu, nu, fn, it - 1, True
        free = (t > lo) & (t < hi)
        Jz = _cell_coordinates_matrix(rows, cols, a2 * free, nr)[keep][:, keep]
        dg = Jz.diagonal()
        dg = np.where(dg > 0, dg, max(float(dg.max(initial=0.0)), 1e-300))
        Jz = Jz + sp.diags(1e-14 * dg)
        # right-hand side: y-space (-F_row, F_col) mapped to (s, g)
        fr, fc = -F[:nr], F[nr:]
        bz = np.concatenate([fr + fc, 0.5 * (fr - fc)])[keep]
        Dh = 1.0 / np.sqrt(Jz.diagonal())
        lu = spla.splu((sp.diags(Dh) @ Jz @ sp.diags(Dh)).tocsc())
        zk = Dh * lu.solve(Dh * bz)
        for _ in range(2):
            zk = zk + Dh * lu.solve(Dh * (bz - Jz @ zk))
        z = np.zeros(2 * nr)
        z[keep] = zk
        zs, zg = z[:nr], z[nr:]
        dt = a * np.where(off, (zs[rows] - zs[cols]) + 0.5 * (zg[rows] + zg[cols]), zg[rows])
        dmu = zs + 0.5 * zg
        dnu = -(zs - 0.5 * zg)
        d = np.concatenate([dmu, dnu])
        slope = float(F @ d)
        if not slope < 0.0:
            return x, t, mu, nu, fn, it, False
        step = 1.0
        while True:
            dtheta = float(np.sum(_dpsi(t, step * dt, lo, hi))) - step * float(d @ rs)
            if dtheta <= 1e-4 * step * slope:
                break
            # near the solution theta changes by less than its rounding;
            # accept a full step that shrinks the residual
            if step == 1.0:
                xt = np.clip(t + dt, lo, hi)
                Ft = resid(xt)
                if float(np.max(np.abs(Ft))) < 0.5 * fn:
                    break
            step *= 0.5
            if step < 1e-12:
                return x, t, mu, nu, fn, it, False
        t = t + step * dt
        mu, nu = mu + step * dmu, nu + step * dnu
        x = np.clip(t, lo, hi)
        F = resid(x)
        if not np.all(np.isfinite(F)) or float(np.max(np.abs(t))) > 1e12:
            return x, t, mu, nu, float(np.max(np.abs(F))), it, False
    fn = float(np.max(np.abs(F)))
    return x, t, mu, nu, fn, max_iter, fn <= tol


def solve_mass_qp(rows, cols, a, b_row, b_col, box_policy="paper_then_relax",
                  tol=1e-14, max_iter=200, levels=None, active=None):
    """Unique minimiser of eq. opti_masscons; see the module docstring.

    ``tol`` bounds max |A_hat(1+x) - b| relative to max |b|.  ``active``
    (per cell, optional): the cells whose row and column are constrained
    (ghost cells, Sec. 3.2, Remark on inflow and outflow, are not).
    Returns a dict: ``x`` (n_z), ``mu``, ``nu`` (dual, in the units of the
    scaled problem a / max|b|), ``level``, ``residual`` (relative),
    ``iterations``, ``lo``, ``hi``.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    a = np.asarray(a, dtype=np.float64)
    b_row = np.asarray(b_row, dtype=np.float64)
    b_col = np.asarray(b_col, dtype=np.float64)
    scale = float(max(np.max(np.abs(b_row)), np.max(np.abs(b_col))))
    As, bR, bC = a / scale, b_row / scale, b_col / scale
    r, s = constraint_rhs(rows, cols, As, bR, bC)
    if levels is None:
        levels = (0,) if box_policy == "strict" else (0, 1, 2)
    for level in levels:
        lo, hi = BOX_LEVELS[level]
        x, t, mu, nu, res, it, ok = _newton(rows, cols, As, r, s, lo, hi, tol, max_iter,
                                            active)
        if ok:
            return {"x": x, "t": t, "mu": mu, "nu": nu, "level": level, "residual": res,
                    "iterations": it, "lo": lo, "hi": hi, "scale": scale}
        if level < 2:
            feas, _ = feasible_lp(rows, cols, As, bR, bC, lo, hi, active)
            if feas:
                raise QPNotConverged(f"Newton stalled at level {level} (residual {res:.3e})"
                                     " although the LP finds the box feasible")
        elif not ok:
            raise QPNotConverged(f"equality-only level did not converge ({res:.3e})")
    raise QPInfeasible("box infeasible at every allowed level")


def verify_kkt(rows, cols, a, b_row, b_col, x, mu, nu, lo, hi, scale, tol, active=None):
    """Certificate of optimality for a returned (x, lambda): x lies in the
    box, meets every constraint to ``tol`` (relative to ``scale``), and
    equals clip(a (mu_i + nu_j)) entrywise up to the rounding of the sum
    mu_i + nu_j (the multipliers of weakly coupled cells can be large, so
    the check allows 1e-12 of |a| (|mu_i| + |nu_j|)).  Returns the worst
    violation of each condition and ``ok``."""
    As = np.asarray(a) / scale
    t = As * (mu[rows] + nu[cols])
    mag = np.abs(As) * (np.abs(mu[rows]) + np.abs(nu[cols]))
    stat = float(np.max((np.abs(np.clip(t, lo, hi) - x)) / (1.0 + mag), initial=0.0))
    box = float(max(np.max(lo - x, initial=-np.inf), np.max(x - hi, initial=-np.inf), 0.0))
    r, s = constraint_rhs(rows, cols, As, np.asarray(b_row) / scale, np.asarray(b_col) / scale)
    F = residual(rows, cols, As, x, r, s)
    if active is not None:
        F = np.where(np.concatenate([active, active]), F, 0.0)
    prim = float(np.max(np.abs(F), initial=0.0))
    return {"stationarity": stat, "box": box, "primal": prim,
            "ok": stat <= 1e-12 and box == 0.0 and prim <= tol}


def verify_kkt_sg(rows, cols, a, b_row, b_col, x, s, g, lo, hi, scale, tol, s_lo=None,
                  g_lo=None):
    """The certificate of ``verify_kkt`` with the multipliers given in the
    per-cell coordinates s, g (mu_K = s_K + g_K / 2, nu_M = -(s_M - g_M / 2)):
    t_k = a_k ((s_K - s_M) + (g_K + g_M) / 2) off the diagonal and a_k g_K on
    it, which stays accurate where mu and nu are huge and nearly cancel.
    Stationarity is the largest |clip(t_k) - x_k| (x lies in [-1, 1] on the
    paper's box, so this bounds the change of every volume a_k (1 + x_k)
    relative to a_k).  ``s_lo``, ``g_lo`` (optional) are the parts of the
    multipliers below the rounding of s and g; the differences are formed
    part by part."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    As = np.asarray(a) / scale
    sl = np.zeros_like(s) if s_lo is None else s_lo
    gl = np.zeros_like(g) if g_lo is None else g_lo

    def two_sum(x, y):
        # x + y = h + e exactly (Knuth)
        h = x + y
        yy = h - x
        return h, (x - (h - yy)) + (y - yy)

    # differences of multipliers of 1e9 and more: the leading difference
    # kept exactly, then the small parts
    dh, de = two_sum(s[rows], -s[cols])
    ds = dh + (de + (sl[rows] - sl[cols]))
    gh, ge = two_sum(g[rows], g[cols])
    sg = gh + (ge + (gl[rows] + gl[cols]))
    t = np.where(rows != cols, As * (ds + 0.5 * sg), As * (g[rows] + gl[rows]))
    stat = float(np.max(np.abs(np.clip(t, lo, hi) - x), initial=0.0))
    box = float(max(np.max(lo - x, initial=-np.inf), np.max(x - hi, initial=-np.inf), 0.0))
    r, sv = constraint_rhs(rows, cols, As, np.asarray(b_row) / scale, np.asarray(b_col) / scale)
    prim = float(np.max(np.abs(residual(rows, cols, As, x, r, sv)), initial=0.0))
    return {"stationarity": stat, "box": box, "primal": prim,
            "ok": stat <= 1e-12 and box == 0.0 and prim <= tol}
