"""Pins of the oracle's least-change bounded problem (eq. opti_masscons).

The minimiser is unique, so the oracle's dual Newton method is compared
with independent solvers: SciPy's SLSQP on small dense cases, NumPy's
minimum-norm least squares for the equality-only level, linprog (HiGHS)
for feasibility, and the KKT certificate.
"""

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import qp as oqp
from oracle import transfer as otr
from paper_1908_05834_amd import inputs


def _random_transfer(n, seed, density=0.3, noise=0.05, small=0.0):
    """A positive matrix like A^(N): rows sum to b exactly, columns are off
    by a few percent.  ``small`` > 0 adds weak entries whose relative
    change must be large, which pushes them onto the box."""
    rng = np.random.default_rng(seed)
    D = rng.uniform(0.2, 1, (n, n)) * (rng.uniform(0, 1, (n, n)) < density) + 2.0 * np.eye(n)
    if small:
        D += small * np.roll(np.eye(n), 1, axis=1)
    b = rng.uniform(1.0, 2.0, n)
    r, c = np.nonzero(D)
    rp = np.searchsorted(r, np.arange(n + 1))
    a = otr.scaling_sweeps(rp, c, D[r, c], b, b, 200)
    a = a * (1.0 + noise * rng.uniform(-1, 1, n))[c]
    a = a * (b / np.bincount(r, weights=a, minlength=n))[r]
    return r, c, a, b


def _slsqp(r, c, a, b, lo, hi):
    n = b.size
    E = np.zeros((2 * n, a.size))
    E[r, np.arange(a.size)] = a
    E[n + c, np.arange(a.size)] = a
    rhs = np.r_[b, b] - E @ np.ones(a.size)
    # the row and column sums share their total: drop one redundant equation
    E, rhs = E[:-1], rhs[:-1]
    bounds = [(None if not np.isfinite(lo) else lo, None if not np.isfinite(hi) else hi)] * a.size
    res = minimize(lambda x: x @ x, np.zeros(a.size), jac=lambda x: 2 * x, method="SLSQP",
                   constraints=[{"type": "eq", "fun": lambda x: E @ x - rhs, "jac": lambda x: E}],
                   bounds=bounds, options={"ftol": 1e-16, "maxiter": 500})
    assert res.success, res.message
    return res.x


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_slsqp_box(seed):
    r, c, a, b = _random_transfer(8, seed)
    out = oqp.solve_mass_qp(r, c, a, b, b)
    assert out["level"] == 0
    x_ref = _slsqp(r, c, a, b, -1.0, 1.0)
    np.testing.assert_allclose(out["x"], x_ref, atol=1e-8)
    assert oqp.verify_kkt(r, c, a, b, b, out["x"], out["mu"], out["nu"], out["lo"], out["hi"],
                          out["scale"], 1e-13)["ok"]


def test_active_bounds_are_exercised():
    r, c, a, b = _random_transfer(8, 0)
    out = oqp.solve_mass_qp(r, c, a, b, b)
    x = out["x"]
    # this instance has entries pinned to the box; the unconstrained
    # minimum-norm solution leaves it
    assert np.any(np.abs(x) == 1.0)
    x_ref = _slsqp(r, c, a, b, -1.0, 1.0)
    np.testing.assert_allclose(x, x_ref, atol=1e-8)


def test_equality_only_is_min_norm():
    r, c, a, b = _random_transfer(12, 3)
    out = oqp.solve_mass_qp(r, c, a, b, b, levels=(2,))
    n = b.size
    E = np.zeros((2 * n, a.size))
    E[r, np.arange(a.size)] = a
    E[n + c, np.arange(a.size)] = a
    rhs = np.r_[b, b] - E @ np.ones(a.size)
    x_ref = np.linalg.lstsq(E, rhs, rcond=None)[0]
    np.testing.assert_allclose(out["x"], x_ref, atol=1e-12)


def test_feasible_matrix_gives_zero():
    rng = np.random.default_rng(4)
    n = 10
    P = rng.uniform(0, 1, (n, n)) * (rng.uniform(0, 1, (n, n)) < 0.4) + np.eye(n)
    # Sinkhorn to convergence gives exact marginals b = 1
    r, c = np.nonzero(P)
    rp = np.searchsorted(r, np.arange(n + 1))
    a = otr.scaling_sweeps(rp, c, P[r, c], np.ones(n), np.ones(n), 2000)
    out = oqp.solve_mass_qp(r, c, a, np.ones(n), np.ones(n))
    assert np.max(np.abs(out["x"])) < 1e-12


def test_relaxation_levels_agree_with_lp():
    """The 2D solid-body workload with one disk per cell cannot meet the
    paper's box: the oracle must find that, and drop the cap."""
    w = inputs.solid_body_32()
    mesh = inputs.cartesian_mesh((16, 16))
    vel = inputs.sample_velocity(mesh, inputs.solid_body_2d)
    T = otr.build_transfer(mesh, vel, 0.02, layout="inscribed", stop_after="sinkhorn")
    rows = otr.csr_rows(T["row_ptr"])
    b = T["b"]
    s = b.max()
    feas0, _ = oqp.feasible_lp(rows, T["col"], T["AN"] / s, b / s, b / s, -1.0, 1.0)
    feas1, _ = oqp.feasible_lp(rows, T["col"], T["AN"] / s, b / s, b / s, -1.0, np.inf)
    out = oqp.solve_mass_qp(rows, T["col"], T["AN"], b, b)
    assert out["level"] == (0 if feas0 else (1 if feas1 else 2))
    assert not feas0
    assert w["dt"] == 0.01


def test_strict_policy_raises():
    mesh = inputs.cartesian_mesh((16, 16))
    vel = inputs.sample_velocity(mesh, inputs.solid_body_2d)
    T = otr.build_transfer(mesh, vel, 0.02, layout="inscribed", stop_after="sinkhorn")
    with pytest.raises(oqp.QPInfeasible):
        oqp.solve_mass_qp(otr.csr_rows(T["row_ptr"]), T["col"], T["AN"], T["b"], T["b"],
                          box_policy="strict")


def test_planted_mistake_is_caught():
    """A wrong sign in the stationarity map (x = clip(-a(mu+nu))) would make
    the returned x fail the primal check: verify_kkt must see it."""
    r, c, a, b = _random_transfer(8, 11)
    out = oqp.solve_mass_qp(r, c, a, b, b)
    bad = np.clip(-(a / out["scale"]) * (out["mu"][r] + out["nu"][c]), -1, 1)
    chk = oqp.verify_kkt(r, c, a, b, b, bad, out["mu"], out["nu"], -1.0, 1.0, out["scale"],
                         1e-13)
    assert not chk["ok"]


def test_kkt_in_cell_coordinates():
    """The (s, g) form of the certificate accepts the oracle's own solution
    (s = (mu - nu) / 2, g = mu + nu) and rejects a solution moved by 1e-9 on
    one free entry, and multipliers with a sign error in g."""
    r, c, a, b = _random_transfer(30, 5, small=1e-3)
    out = oqp.solve_mass_qp(r, c, a, b, b)
    mu, nu = out["mu"], out["nu"]
    s, g = 0.5 * (mu - nu), mu + nu
    lo, hi = out["lo"], out["hi"]
    ok = oqp.verify_kkt_sg(r, c, a, b, b, out["x"], s, g, lo, hi, out["scale"], 1e-13)
    assert ok["ok"], ok
    free = np.nonzero((out["x"] > lo + 1e-3) & (out["x"] < hi - 1e-3))[0]
    x2 = out["x"].copy()
    x2[free[0]] += 1e-9
    bad = oqp.verify_kkt_sg(r, c, a, b, b, x2, s, g, lo, hi, out["scale"], 1e-7)
    assert not bad["ok"] and bad["stationarity"] >= 0.9e-9
    bad = oqp.verify_kkt_sg(r, c, a, b, b, out["x"], s, -g, lo, hi, out["scale"], 1e-13)
    assert not bad["ok"]
