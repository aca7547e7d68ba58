"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars (BASELINE the benchmark spec): candidate pairs and the CSR pattern bit-exact
on identical tracked centres; V within 1e-13 (relative to max |V|) in FP64;
A^(N) within 1e-12; concentrations within 1e-10 relative (max norm) in
FP64 and 1e-5 in the FP32-volume mode; mass conserved to 1e-12.
"""

import sys

import numpy as np
import pytest

from oracle import geometry as ogeo
from oracle import qp as oqp
from oracle import transfer as otr
from paper_1908_05834_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1908_05834_amd import bchar
    return torch, bchar


def _case(name):
    if name == "rot2d_subcell":
        mesh = inputs.cartesian_mesh((16, 16))
        return mesh, inputs.sample_velocity(mesh, inputs.rotation_stretch_2d), 0.8, "subcell"
    if name == "solid_equal":
        w = inputs.solid_body_32()
        return w["mesh"], w["vel_fn"](0), w["dt"], "equal_measure"
    if name == "solid_inscribed":
        w = inputs.solid_body_32()
        return w["mesh"], w["vel_fn"](0), w["dt"], "inscribed"
    if name == "swirl3d_subcell_8":
        w = inputs.swirl_hex(8)
        return w["mesh"], w["vel_fn"](0), 0.05, "subcell"
    if name == "swirl3d_subcell_16":
        w = inputs.swirl_hex(16)
        return w["mesh"], w["vel_fn"](3), 1.0 / 64.0, "subcell"
    if name == "swirl3d_inscribed_12":
        w = inputs.swirl_hex(12)
        return w["mesh"], w["vel_fn"](0), 0.03, "inscribed"
    if name == "porous2d_subcell":
        mesh = inputs.cartesian_mesh((12, 12), phi=inputs.lognormal_phi(144, 5834))
        return mesh, inputs.sample_velocity(mesh, inputs.rotation_stretch_2d), 0.6, "subcell"
    if name == "porous3d_subcell":
        w = inputs.porous_swirl_hex(8)
        return w["mesh"], w["vel_fn"](0), 0.05, "subcell"
    if name in ("tets", "tets_porous"):
        phi = inputs.lognormal_phi(6 * 4 ** 3, 21) if name == "tets_porous" else None
        mesh = inputs.kuhn_tets(4, 0.1, 8, phi=phi)
        vel = inputs.sample_velocity_grid((4, 4, 4), lambda p, t: inputs.swirl_3d(p, t))
        return mesh, vel, 0.05, "equal_measure"
    if name in ("tris", "tris_porous"):
        phi = inputs.lognormal_phi(2 * 10 ** 2, 22) if name == "tris_porous" else None
        mesh = inputs.triangulated_square(10, 0.1, 6, phi=phi)
        vel = inputs.sample_velocity_grid((10, 10), inputs.rotation_stretch_2d)
        return mesh, vel, 0.3, "equal_measure"
    if name in ("mixed_tri", "mixed_hex"):
        # small members of the batch of independent problems (seed 3 is a
        # triangulated square at CFL 3.3, seed 4 a hexahedral cube at CFL 3.9)
        q = inputs.mixed_problem(3 if name == "mixed_tri" else 4, 400.0, 400.0)
        return q["mesh"], q["vel"], q["dt"], q["layout"]
    raise KeyError(name)


GEOM_CASES = ["rot2d_subcell", "solid_equal", "solid_inscribed", "swirl3d_subcell_8",
              "swirl3d_inscribed_12", "porous2d_subcell", "porous3d_subcell",
              "tets", "tets_porous", "tris", "tris_porous", "mixed_tri", "mixed_hex"]


def _obuild(mesh, vel, dt, M, **kw):
    """The oracle's build; on a simplicial mesh it takes the library's
    residing balls (the cube root of the radius may differ in the last
    place; the rest of the path is compared on identical balls)."""
    if ogeo.is_simplex(mesh):
        c, r, _ = M.export_balls()
        kw["balls_override"] = (c, r)
    return otr.build_transfer(mesh, vel, dt, **kw)


def _tracked_tensors(torch, T):
    tr = np.ascontiguousarray(T["traced"].T)          # (dim, n_balls)
    return (torch.as_tensor(tr, device="cuda"),
            torch.as_tensor(np.ascontiguousarray(T["r_hat"]), device="cuda"))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", GEOM_CASES)
def test_pairs_pattern_and_v(env, name, precision):
    torch, bchar = env
    _say(f"[gpu] pairs/V {name} {precision}")
    mesh, vel, dt, layout = _case(name)
    M = bchar.Mesh(mesh, layout)
    ref = _obuild(mesh, vel, dt, M, layout=layout, precision=precision, stop_after="v")
    tr, rh = _tracked_tensors(torch, ref)
    prec = bchar.FP64 if precision == "fp64" else bchar.FP32_VOLUME
    T = bchar.Transfer.build_tracked(
        M, tr, rh, bchar.opts_default(stop_after=bchar.STAGE_V, keep_pairs=1, precision=prec))
    a, b = T.export_pairs()
    ia, ib = ref["pairs"]
    assert np.array_equal(a, ia) and np.array_equal(b, ib), "candidate pairs differ"
    rp, col, V = T.export_csr(bchar.STAGE_V)
    assert np.array_equal(rp, ref["row_ptr"]) and np.array_equal(col, ref["col"])
    err = np.max(np.abs(V - ref["V"])) / np.max(np.abs(ref["V"]))
    _say(f"    V rel err {err:.3e}")
    assert err <= (1e-13 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("name", ["rot2d_subcell", "swirl3d_subcell_16", "porous2d_subcell",
                                  "porous3d_subcell", "tets", "tets_porous", "tris_porous"])
def test_tracking(env, name):
    torch, bchar = env
    _say(f"[gpu] tracking {name}")
    mesh, vel, dt, layout = _case(name)
    M = bchar.Mesh(mesh, layout)
    U = bchar.VelocityLattice(vel)
    if ogeo.is_simplex(mesh):
        C, r, _ = M.export_balls()
    else:
        C, r, _ = ogeo.ball_layout(mesh["n"], mesh["origin"], mesh["h"], layout)
    want = ogeo.trace_points(C, mesh, vel, dt)
    want_r = ogeo.tracked_radius(C, r, want, mesh, vel, dt)
    porous = not np.all(mesh["phi"] == mesh["phi"][0])
    # binary64 tracking repeats the oracle's operations one by one: equal
    # bits (FP64, and FP32_LENS, which tracks in binary64).  Binary32
    # tracking (FP32_VOLUME) is within its rounding; it refuses a mesh whose
    # porosity varies.
    cases = [(bchar.FP64, 0.0, bchar.FP64), (bchar.FP32_LENS, 0.0, bchar.FP64)]
    if porous:
        with pytest.raises(bchar.BcharError) as ei:
            bchar.Transfer.build(M, U, dt, bchar.opts_default(precision=bchar.FP32_VOLUME))
        assert ei.value.status == bchar.E_UNSUPPORTED
    else:
        cases.append((bchar.FP32_VOLUME, 2e-6, bchar.FP32_VOLUME))
    for prec, tol, used in cases:
        T = bchar.Transfer.build(M, U, dt, bchar.opts_default(stop_after=bchar.STAGE_V,
                                                              precision=prec))
        assert T.stats["trace_precision"] == used
        got, got_r = T.export_tracked()
        e1, e2 = np.max(np.abs(got - want)), np.max(np.abs(got_r - want_r))
        _say(f"    precision {prec}: centre err {e1:.3e}, radius err {e2:.3e}")
        assert e1 <= tol and e2 <= tol


@pytest.mark.parametrize("name", ["rot2d_subcell", "swirl3d_subcell_8", "solid_equal",
                                  "porous3d_subcell"])
def test_scaling(env, name):
    torch, bchar = env
    _say(f"[gpu] scaling {name}")
    mesh, vel, dt, layout = _case(name)
    ref = otr.build_transfer(mesh, vel, dt, layout=layout, stop_after="sinkhorn")
    M = bchar.Mesh(mesh, layout)
    tr, rh = _tracked_tensors(torch, ref)
    T = bchar.Transfer.build_tracked(M, tr, rh, bchar.opts_default(stop_after=bchar.STAGE_SCALING))
    _, _, AN = T.export_csr(bchar.STAGE_SCALING)
    err = np.max(np.abs(AN - ref["AN"])) / np.max(np.abs(ref["AN"]))
    _say(f"    A^(N) rel err {err:.3e}, col err {T.stats['scaling_max_col_err']:.3e}")
    assert err <= 1e-12


def _full(env, name, precision="fp64", **opts):
    torch, bchar = env
    mesh, vel, dt, layout = _case(name)
    M = bchar.Mesh(mesh, layout)
    ref = _obuild(mesh, vel, dt, M, layout=layout, precision=precision)
    U = bchar.VelocityLattice(vel)
    if precision == "fp64":
        prec = bchar.FP64
    else:
        # binary32 tracking needs a constant porosity
        prec = bchar.FP32_VOLUME if np.all(mesh["phi"] == mesh["phi"][0]) else bchar.FP32_LENS
    T = bchar.Transfer.build(M, U, dt, bchar.opts_default(precision=prec, **opts))
    return torch, bchar, mesh, ref, M, T


@pytest.mark.parametrize("name", ["rot2d_subcell", "swirl3d_subcell_8", "swirl3d_subcell_16",
                                  "solid_equal", "solid_inscribed", "porous2d_subcell",
                                  "porous3d_subcell", "swirl3d_inscribed_12", "tets",
                                  "tets_porous", "tris", "tris_porous", "mixed_tri",
                                  "mixed_hex"])
def test_full_step(env, name):
    _check_full_step(env, name)


# the cycle that visits every other level (opts.cycle_skip) is another
# preconditioner for the same systems: the same solution to the same bar
@pytest.mark.parametrize("name", ["swirl3d_subcell_16", "solid_inscribed", "tets", "tris",
                                  "mixed_hex"])
def test_full_step_cycle_skip(env, name):
    _check_full_step(env, name, cycle_skip=1)


# the fine level's first two sweeps as two passes (the path of meshes above
# 2^20 cells): the same minimiser to the same bar
@pytest.mark.parametrize("name", ["swirl3d_subcell_16", "tets_porous", "solid_inscribed"])
def test_full_step_unfused_sweeps(env, name):
    _check_full_step(env, name, z_fuse_max_cells=0)


def _check_full_step(env, name, **opts):
    _say(f"[gpu] full step {name} {opts}")
    torch, bchar, mesh, ref, M, T = _full(env, name, **opts)
    st = T.stats
    _say(f"    stats {st}; oracle level {ref['qp']['level']} it {ref['qp']['iterations']}")
    assert st["qp_level"] == ref["qp"]["level"]
    rp, col, A = T.export_csr(bchar.STAGE_ALL)
    nc = rp.size - 1
    c0 = inputs.uniform_c(mesh, 11)
    cin = torch.as_tensor(c0, device="cuda")
    cout = torch.empty_like(cin)
    T.step(cin, cout)
    got = cout.cpu().numpy()
    want = otr.apply(ref["row_ptr"], ref["col"], ref["A"], ref["b"], c0)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    _say(f"    c rel err {err:.3e}")
    assert err <= 1e-10
    # conservation and constants, on the GPU result alone
    m0, m1 = M.mass(cin), M.mass(cout)
    assert abs(m1 - m0) <= 1e-12 * abs(m0)
    # the compensated mass reduction against the correctly rounded sum
    vol = ref["cell_vol"]
    for cv, mv in ((c0, m0), (got, m1)):
        want_m = otr.mass(mesh["phi"], vol, cv)
        assert abs(mv - want_m) <= 2 * np.spacing(abs(want_m)), (mv, want_m)
    ones = torch.ones(nc, dtype=torch.float64, device="cuda")
    T.step(ones, cout)
    assert torch.max(torch.abs(cout - 1.0)).item() <= 1e-12
    # KKT certificate of the GPU's QP solution
    x, mu, nu = T.export_qp()
    _, _, AN = T.export_csr(bchar.STAGE_SCALING)
    rows = otr.csr_rows(rp)
    lo, hi = oqp.BOX_LEVELS[st["qp_level"]]
    chk = oqp.verify_kkt(rows, col, AN, ref["b"], ref["b"], x, mu, nu, lo, hi, ref["b"].max(),
                         2e-13)
    _say(f"    kkt {chk}")
    assert chk["ok"]


@pytest.mark.parametrize("name", ["rot2d_subcell", "swirl3d_subcell_16", "porous3d_subcell",
                                  "tets", "tets_porous"])
def test_full_step_fp32(env, name):
    _say(f"[gpu] full step fp32 {name}")
    torch, bchar, mesh, ref, M, T = _full(env, name, "fp32")
    c0 = inputs.uniform_c(mesh, 12)
    cin = torch.as_tensor(c0, device="cuda")
    cout = torch.empty_like(cin)
    T.step(cin, cout)
    got = cout.cpu().numpy()
    # against the plain FP64 oracle (tracking in binary64)
    ref64 = _obuild(mesh, *_case(name)[1:3], M, layout=_case(name)[3])
    want = otr.apply(ref64["row_ptr"], ref64["col"], ref64["A"], ref64["b"], c0)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    _say(f"    c rel err vs fp64 oracle {err:.3e}")
    assert err <= 1e-5
    m0, m1 = M.mass(cin), M.mass(cout)
    assert abs(m1 - m0) <= 1e-12 * abs(m0)


def test_solid_body_ten_steps(env):
    """2D solid-body rotation, 32 x 32, equal-area disks, dt = 0.01, 10
    steps with the transfer built once."""
    torch, bchar = env
    _say("[gpu] solid body 10 steps")
    w = inputs.solid_body_32()
    mesh, vel = w["mesh"], w["vel_fn"](0)
    ref = otr.build_transfer(mesh, vel, w["dt"], layout="equal_measure")
    M = bchar.Mesh(mesh, "equal_measure")
    T = bchar.Transfer.build(M, bchar.VelocityLattice(vel), w["dt"])
    c = torch.as_tensor(w["c0"], device="cuda")
    nxt = torch.empty_like(c)
    cref = w["c0"].copy()
    m0 = M.mass(c)
    for _ in range(w["steps"]):
        T.step(c, nxt)
        c, nxt = nxt, c
        cref = otr.apply(ref["row_ptr"], ref["col"], ref["A"], ref["b"], cref)
    err = np.max(np.abs(c.cpu().numpy() - cref)) / np.max(np.abs(cref))
    _say(f"    c rel err after 10 steps {err:.3e}")
    assert err <= 1e-10
    assert abs(M.mass(c) - m0) <= 1e-12 * abs(m0)


def test_rebuilds_follow_the_flow(env):
    """A transfer rebuilt on every step of a time-dependent flow (warm
    starts from the previous solve, semismooth attempts skipped for a few
    solves after one failed) gives each step's own minimiser: c within the
    bar of the oracle's build of that step, the same box level, and the
    same c as a transfer rebuilt without warm starts."""
    torch, bchar = env
    _say("[gpu] rebuilds along a time-dependent flow")
    w = inputs.swirl_hex(12)
    mesh = w["mesh"]
    dt = 4 * w["dt"]
    M = bchar.Mesh(mesh, "subcell")
    T = T0 = None
    c0 = inputs.uniform_c(mesh, 21)
    cin = torch.as_tensor(c0, device="cuda")
    cout = torch.empty_like(cin)
    cold = bchar.opts_default(warm_start=0)
    for s in range(6):
        vel = w["vel_fn"](8 * s)
        U = bchar.VelocityLattice(vel)
        if T is None:
            T = bchar.Transfer.build(M, U, dt)
            T0 = bchar.Transfer.build(M, U, dt, cold)
        else:
            T.rebuild(U, dt)
            T0.rebuild(U, dt, cold)
        ref = otr.build_transfer(mesh, vel, dt, layout="subcell")
        st = T.stats
        _say(f"    step {s}: level {st['qp_level']} ipm {st['qp_ipm']} newton {st['qp_newton']} "
             f"cg {st['qp_cg']}; cold cg {T0.stats['qp_cg']}")
        assert st["qp_level"] == ref["qp"]["level"] == T0.stats["qp_level"]
        T.step(cin, cout)
        got = cout.cpu().numpy()
        want = otr.apply(ref["row_ptr"], ref["col"], ref["A"], ref["b"], c0)
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        T0.step(cin, cout)
        err0 = np.max(np.abs(got - cout.cpu().numpy())) / np.max(np.abs(want))
        _say(f"    c rel err {err:.3e}, against the cold rebuild {err0:.3e}")
        assert err <= 1e-10 and err0 <= 1e-10


def test_simplex_mesh_checks(env):
    """Simplicial meshes: the layout must be equal_measure, degenerate cells
    and out-of-range vertex ids are rejected, ball measures equal |K|."""
    torch, bchar = env
    m = inputs.kuhn_tets(2, 0.1, 3)
    with pytest.raises(bchar.BcharError):
        bchar.Mesh(m, "subcell")
    bad = dict(m)
    bad["cells"] = m["cells"].copy()
    bad["cells"][0, 1] = bad["cells"][0, 0]
    with pytest.raises(bchar.BcharError):
        bchar.Mesh(bad, "equal_measure")
    bad["cells"] = m["cells"].copy()
    bad["cells"][3, 2] = m["vertices"].shape[0]
    with pytest.raises(bchar.BcharError):
        bchar.Mesh(bad, "equal_measure")
    M = bchar.Mesh(m, "equal_measure")
    c, r, cell = M.export_balls()
    oc, orad, _ = ogeo.simplex_ball_layout(m)
    # centroids are the same sums in the same order; both sides round the
    # cube root to nearest (the bar: one unit in the last place)
    assert np.array_equal(c, oc)
    assert np.all(np.abs(r - orad) <= np.spacing(orad))


def test_unstructured_properties(env):
    """The unstructured workload (jittered Kuhn tetrahedra, lognormal
    porosity, CFL 4 on u / phi, binary32 lens volumes) at 24^3 x 6 cells,
    two steps:
    properties that hold at any size -- porous mass to 1e-12, constants to
    1e-12, both marginals of A equal |K|_phi."""
    torch, bchar = env
    _say("[gpu] unstructured 24^3 x 6 tets, 2 steps")
    w = inputs.jittered_tets(24, steps=2)
    mesh = w["mesh"]
    M = bchar.Mesh(mesh, "equal_measure")
    o = bchar.opts_default(precision=bchar.FP32_LENS)
    c = torch.as_tensor(w["c0"], device="cuda")
    nxt = torch.empty_like(c)
    m0 = M.mass(c)
    T = None
    for s in range(w["steps"]):
        U = bchar.VelocityLattice(w["vel_fn"](s))
        if T is None:
            T = bchar.Transfer.build(M, U, w["dt"], o)
        else:
            T.rebuild(U, w["dt"], o)
        T.step(c, nxt)
        c, nxt = nxt, c
        _say(f"    step {s}: {T.stats}")
        assert abs(M.mass(c) - m0) <= 1e-12 * abs(m0)
    rp, col, A = T.export_csr(bchar.STAGE_ALL)
    nc = rp.size - 1
    rows = otr.csr_rows(rp)
    b = mesh["phi"] * ogeo.simplex_volumes(mesh["vertices"], mesh["cells"])
    assert np.max(np.abs(np.bincount(rows, weights=A, minlength=nc) - b)) <= 2e-13 * b.max()
    assert np.max(np.abs(np.bincount(col, weights=A, minlength=nc) - b)) <= 2e-13 * b.max()
    ones = torch.ones(nc, dtype=torch.float64, device="cuda")
    T.step(ones, nxt)
    assert torch.max(torch.abs(nxt - 1.0)).item() <= 1e-12


def test_void_step_halving(env):
    # a step too long for the mesh: some residing cell receives no tracked
    # ball (a void column).  The library reports it, or with max_halvings
    # builds the transfer of half the step and applies it twice, which must
    # equal the oracle's transfer of dt / 2 applied twice
    torch, bchar = env
    _say("[gpu] void column, step halving")
    q = inputs.mixed_problem(2, 400.0, 400.0)
    mesh, vel, dt, layout = q["mesh"], q["vel"], q["dt"], q["layout"]
    with pytest.raises(otr.VoidColumnError):
        otr.build_transfer(mesh, vel, dt, layout=layout)
    ref = otr.build_transfer(mesh, vel, dt / 2, layout=layout)
    M = bchar.Mesh(mesh, layout)
    U = bchar.VelocityLattice(vel)
    with pytest.raises(bchar.BcharError) as ei:
        bchar.Transfer.build(M, U, dt)
    assert ei.value.status == bchar.E_VOID_COLUMN
    T = bchar.Transfer.build(M, U, dt, bchar.opts_default(max_halvings=3))
    assert T.stats["dt_halvings"] == 1 and T.stats["qp_level"] == ref["qp"]["level"]
    c0 = inputs.uniform_c(mesh, 11)
    cin = torch.as_tensor(c0, device="cuda")
    cout = torch.empty_like(cin)
    T.step(cin, cout)
    got = cout.cpu().numpy()
    half = otr.apply(ref["row_ptr"], ref["col"], ref["A"], ref["b"], c0)
    want = otr.apply(ref["row_ptr"], ref["col"], ref["A"], ref["b"], half)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    _say(f"    c rel err {err:.3e}")
    assert err <= 1e-10
    m0, m1 = M.mass(cin), M.mass(cout)
    assert abs(m1 - m0) <= 1e-12 * abs(m0)
