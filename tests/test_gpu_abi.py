"""GPU tests of the boundary's options: caller-given balls (layout CUSTOM,
Sec. 3: any points C_{K,s} with radii, any number per cell), geometry in
device memory, and the void counts of the statistics.  Parity against the
oracle to the same bars as tests/test_gpu_parity.py."""

import sys

import numpy as np
import pytest

from oracle import geometry as ogeo
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


def _custom_case(name):
    if name == "hex":
        w = inputs.swirl_hex(8)
        return inputs.random_subcell_balls(w["mesh"], 5), w["vel_fn"](0), 0.02
    if name == "square":
        m = inputs.random_subcell_balls(inputs.cartesian_mesh((12, 12)), 6)
        return m, inputs.sample_velocity(m, inputs.rotation_stretch_2d), 0.3
    if name == "tets":
        mesh = inputs.kuhn_tets(4, 0.1, 8)
        vel = inputs.sample_velocity_grid((4, 4, 4), lambda p, t: inputs.swirl_3d(p, t))
        return inputs.corner_balls_simplex(mesh), vel, 0.05
    if name == "tris":
        mesh = inputs.triangulated_square(10, 0.1, 6)
        vel = inputs.sample_velocity_grid((10, 10), inputs.rotation_stretch_2d)
        return inputs.corner_balls_simplex(mesh), vel, 0.3
    raise KeyError(name)


@pytest.mark.parametrize("name", ["hex", "square", "tets", "tris"])
def test_custom_layout(env, name):
    torch, bchar = env
    _say(f"[gpu] custom layout {name}")
    mesh, vel, dt = _custom_case(name)
    M = bchar.Mesh(mesh, "custom")
    assert M.n_balls == len(mesh["ball_radii"]) and M.balls_per_cell == 0
    c, r, cell = M.export_balls()
    assert np.array_equal(c, mesh["ball_centres"]) and np.array_equal(r, mesh["ball_radii"])
    assert np.array_equal(cell, mesh["ball_cell"])
    ref = otr.build_transfer(mesh, vel, dt, layout="custom")
    # candidate pairs and V on the oracle's tracked centres
    tr = torch.as_tensor(np.ascontiguousarray(ref["traced"].T), device="cuda")
    rh = torch.as_tensor(np.ascontiguousarray(ref["r_hat"]), device="cuda")
    Tv = bchar.Transfer.build_tracked(M, tr, rh, bchar.opts_default(stop_after=bchar.STAGE_V,
                                                                   keep_pairs=1))
    a, b = Tv.export_pairs()
    assert np.array_equal(a, ref["pairs"][0]) and np.array_equal(b, ref["pairs"][1])
    rp, col, V = Tv.export_csr(bchar.STAGE_V)
    assert np.array_equal(rp, ref["row_ptr"]) and np.array_equal(col, ref["col"])
    assert np.max(np.abs(V - ref["V"])) <= 1e-13 * np.max(np.abs(ref["V"]))
    # the whole step, tracking included
    T = bchar.Transfer.build(M, bchar.VelocityLattice(vel), dt)
    _say(f"    stats {T.stats}; oracle level {ref['qp']['level']}")
    assert T.stats["qp_level"] == ref["qp"]["level"]
    c0 = inputs.uniform_c(mesh, 13)
    cin = torch.as_tensor(c0, device="cuda")
    cout = torch.empty_like(cin)
    T.step(cin, cout)
    got = cout.cpu().numpy()
    want = otr.apply(ref["row_ptr"], ref["col"], ref["A"], ref["b"], c0)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    _say(f"    c rel err {err:.3e}")
    assert err <= 1e-10
    m0, m1 = M.mass(cin), M.mass(cout)
    assert abs(m1 - m0) <= 1e-12 * abs(m0)
    want_m = otr.mass(mesh["phi"], ref["cell_vol"], got)
    assert abs(m1 - want_m) <= 2 * np.spacing(abs(want_m))


@pytest.mark.parametrize("name", ["tets_equal", "tets_custom", "hex_custom"])
def test_device_geometry(env, name):
    """Vertices, cells and custom balls handed over in device memory give
    the same mesh and the same transfer, bit for bit."""
    torch, bchar = env
    _say(f"[gpu] device geometry {name}")
    if name == "tets_equal":
        mesh, vel, dt = _custom_case("tets")
        layout = "equal_measure"
    elif name == "tets_custom":
        mesh, vel, dt = _custom_case("tets")
        layout = "custom"
    else:
        mesh, vel, dt = _custom_case("hex")
        layout = "custom"
    Mh = bchar.Mesh(mesh, layout)
    Md = bchar.Mesh(mesh, layout, geom_device=True)
    for x, y in zip(Mh.export_balls(), Md.export_balls()):
        assert np.array_equal(x, y)
    U = bchar.VelocityLattice(vel)
    Th = bchar.Transfer.build(Mh, U, dt)
    Td = bchar.Transfer.build(Md, U, dt)
    for x, y in zip(Th.export_csr(), Td.export_csr()):
        assert np.array_equal(x, y)


def test_void_row_count(env):
    """Tracked balls moved to cell corners with a tiny radius overlap no
    inscribed disk: the build reports a void row, the first void ball and
    the number of tracked cells with a void ball."""
    torch, bchar = env
    _say("[gpu] void rows")
    mesh = inputs.cartesian_mesh((8, 8))
    C, r, _ = ogeo.ball_layout(mesh["n"], mesh["origin"], mesh["h"], "inscribed")
    tr = C.copy()
    rh = r.copy()
    h = mesh["h"][0]
    for k in (9, 20, 43):
        tr[k] = C[k] + 0.5 * h
        rh[k] = 0.01 * h
    # the oracle's view of the same geometry
    ia, _ = ogeo.candidate_pairs(tr, rh, C, r)
    void = np.setdiff1d(np.arange(C.shape[0]), ia)
    assert void.tolist() == [9, 20, 43]
    M = bchar.Mesh(mesh, "inscribed")
    with pytest.raises(bchar.BcharError) as ei:
        bchar.Transfer.build_tracked(M, torch.as_tensor(np.ascontiguousarray(tr.T), device="cuda"),
                                     torch.as_tensor(rh, device="cuda"))
    assert ei.value.status == bchar.E_VOID_ROW
    assert ei.value.stats["first_void"] == 9 and ei.value.stats["n_void_rows"] == 3


def test_void_column_count(env):
    """A step too long for a small triangulated square leaves residing
    cells that no tracked ball reaches: the first and the number of zero
    columns of V agree with the oracle's V."""
    torch, bchar = env
    _say("[gpu] void columns")
    q = inputs.mixed_problem(2, 400.0, 400.0)
    mesh, vel, dt, layout = q["mesh"], q["vel"], q["dt"], q["layout"]
    ref = otr.build_transfer(mesh, vel, dt, layout=layout, stop_after="v")
    nc = ref["row_ptr"].size - 1
    colsum = np.bincount(ref["col"], weights=ref["V"], minlength=nc)
    zero = np.nonzero(colsum <= 0)[0]
    assert zero.size > 0
    M = bchar.Mesh(mesh, layout)
    with pytest.raises(bchar.BcharError) as ei:
        bchar.Transfer.build(M, bchar.VelocityLattice(vel), dt)
    assert ei.value.status == bchar.E_VOID_COLUMN
    st = ei.value.stats
    _say(f"    stats {st}; oracle zero columns {zero.tolist()}")
    assert st["first_void"] == zero[0] and st["n_void_cols"] == zero.size
    assert st["n_void_rows"] == 0


@pytest.mark.parametrize("name", ["swirl32", "porous3d", "tets", "hex_custom", "square"])
def test_lds_staging_same_bits(env, name):
    """The assembly staged in LDS and the one reading the hash in global
    memory give the same pairs and the same V, bit for bit."""
    torch, bchar = env
    _say(f"[gpu] LDS staging on/off {name}")
    if name == "swirl32":
        w = inputs.swirl_hex(32)
        mesh, vel, dt, layout = w["mesh"], w["vel_fn"](3), w["dt"], "subcell"
    elif name == "porous3d":
        w = inputs.porous_swirl_hex(8)
        mesh, vel, dt, layout = w["mesh"], w["vel_fn"](0), 0.05, "subcell"
    elif name == "tets":
        mesh, vel, dt = _custom_case("tets")
        layout = "equal_measure"
    elif name == "hex_custom":
        mesh, vel, dt = _custom_case("hex")
        layout = "custom"
    else:
        mesh, vel, dt = _custom_case("square")
        layout = "custom"
    M = bchar.Mesh(mesh, layout)
    U = bchar.VelocityLattice(vel)
    out = []
    for stage in (1, 0):
        T = bchar.Transfer.build(M, U, dt, bchar.opts_default(stop_after=bchar.STAGE_V,
                                                              keep_pairs=1, lds_stage=stage))
        out.append((T.export_pairs(), T.export_csr(bchar.STAGE_V), T.stats["n_pairs"]))
    (p1, c1, n1), (p0, c0, n0) = out
    assert n1 == n0
    for x, y in zip(p1 + c1, p0 + c0):
        assert np.array_equal(x, y)


def _packed_case(name):
    if name == "tris":
        mesh = inputs.triangulated_square(10, 0.1, 6)
        vel = inputs.sample_velocity_grid((10, 10), inputs.rotation_stretch_2d)
        return mesh, vel, 0.022, True
    if name == "tets_porous":
        mesh = inputs.kuhn_tets(4, 0.1, 8, phi=inputs.lognormal_phi(6 * 4 ** 3, 21))
        vel = inputs.sample_velocity_grid((4, 4, 4), lambda p, t: inputs.swirl_3d(p, t))
        return mesh, vel, 0.004, True
    if name == "tets_compressible":
        mesh = inputs.kuhn_tets(4, 0.1, 8)
        vel = inputs.sample_velocity_grid((4, 4, 4),
                                          lambda p, t: inputs.compressible_swirl_3d(p, t))
        return mesh, vel, 0.0125, False
    raise KeyError(name)


@pytest.mark.parametrize("name", ["tris", "tets_porous", "tets_compressible"])
def test_packed_simplex_layout(env, name):
    """Several balls per simplex (layout PACKED): the library's balls equal
    the oracle's rule bit for bit, and the step on them matches the
    oracle's to the parity bars.  (Disjoint balls leave gaps: steps much
    longer than these send the small corner balls into them, a void row.)"""
    torch, bchar = env
    _say(f"[gpu] packed layout {name}")
    mesh, vel, dt, solenoidal = _packed_case(name)
    M = bchar.Mesh(mesh, "packed")
    c, r, cell = M.export_balls()
    oc, orr, ocell = ogeo.simplex_packed_layout(mesh)
    assert np.array_equal(cell, ocell)
    assert np.array_equal(c, oc) and np.array_equal(r, orr)
    dim = mesh["vertices"].shape[1]
    assert np.mean(np.bincount(cell) == dim + 2) > 0.9
    ref = otr.build_transfer(mesh, vel, dt, layout="packed", solenoidal=solenoidal)
    opts = bchar.opts_default(keep_pairs=1,
                              divergence=bchar.DIV_FREE if solenoidal else bchar.DIV_GENERAL)
    T = bchar.Transfer.build(M, bchar.VelocityLattice(vel), dt, opts)
    _say(f"    stats {T.stats}; oracle level {ref['qp']['level']}")
    tr, rh = T.export_tracked()
    assert np.array_equal(tr, ref["traced"]) and np.array_equal(rh, ref["r_hat"])
    a, b = T.export_pairs()
    assert np.array_equal(a, ref["pairs"][0]) and np.array_equal(b, ref["pairs"][1])
    rp, col, V = T.export_csr(bchar.STAGE_V)
    assert np.array_equal(rp, ref["row_ptr"]) and np.array_equal(col, ref["col"])
    assert np.max(np.abs(V - ref["V"])) <= 1e-13 * np.max(np.abs(ref["V"]))
    assert T.stats["qp_level"] == ref["qp"]["level"]
    c0 = inputs.uniform_c(mesh, 23)
    cin = torch.as_tensor(c0, device="cuda")
    cout = torch.empty_like(cin)
    T.step(cin, cout)
    got = cout.cpu().numpy()
    want = otr.apply(ref["row_ptr"], ref["col"], ref["A"], ref["b"], c0)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    _say(f"    c rel err {err:.3e}")
    assert err <= 1e-10
    m0, m1 = M.mass(cin), M.mass(cout)
    assert abs(m1 - m0) <= 1e-12 * abs(m0)


def test_packed_rejected_on_cartesian(env):
    torch, bchar = env
    with pytest.raises(bchar.BcharError) as ei:
        bchar.Mesh(inputs.cartesian_mesh((4, 4)), "packed")
    assert ei.value.status == bchar.E_INVALID_ARG


@pytest.mark.parametrize("name", ["swirl32", "porous3d", "square2d"])
def test_tile_aspect_same_bits(env, name):
    """Every tile shape of the assembly gives the same pairs and the same
    V, bit for bit (the tuner may pick any of them)."""
    torch, bchar = env
    _say(f"[gpu] tile aspects {name}")
    if name == "swirl32":
        w = inputs.swirl_hex(32)
        mesh, vel, dt = w["mesh"], w["vel_fn"](3), w["dt"]
    elif name == "porous3d":
        w = inputs.porous_swirl_hex(8)
        mesh, vel, dt = w["mesh"], w["vel_fn"](0), 0.05
    else:
        mesh = inputs.cartesian_mesh((40, 24))
        vel, dt = inputs.sample_velocity(mesh, inputs.rotation_stretch_2d), 0.6
    M = bchar.Mesh(mesh, "subcell")
    U = bchar.VelocityLattice(vel)
    out = {}
    for a in (0, 1, 2, -1, -2):
        T = bchar.Transfer.build(M, U, dt, bchar.opts_default(stop_after=bchar.STAGE_V,
                                                              keep_pairs=1, tile_aspect=a))
        out[a] = (T.export_pairs(), T.export_csr(bchar.STAGE_V))
    for a in (1, 2, -1, -2):
        for x, y in zip(out[a][0] + out[a][1], out[0][0] + out[0][1]):
            assert np.array_equal(x, y), a


@pytest.mark.parametrize("name", ["swirl32", "porous3d", "tets"])
def test_hash_scale_same_pairs(env, name):
    """Every bucket side of the spatial hash (mesh hash_scale) finds the same
    overlapping pairs; V agrees to rounding (the residing balls of a cell
    may be met in another order) and the step within the parity bar."""
    torch, bchar = env
    _say(f"[gpu] hash scales {name}")
    if name == "swirl32":
        w = inputs.swirl_hex(32)
        mesh, vel, dt, layout = w["mesh"], w["vel_fn"](3), w["dt"], "subcell"
    elif name == "porous3d":
        w = inputs.porous_swirl_hex(8)
        mesh, vel, dt, layout = w["mesh"], w["vel_fn"](0), 0.05, "subcell"
    else:
        mesh = inputs.kuhn_tets(4, 0.1, 8)
        vel = inputs.sample_velocity_grid((4, 4, 4), lambda p, t: inputs.swirl_3d(p, t))
        dt, layout = 0.05, "equal_measure"
    out = {}
    c0 = inputs.uniform_c(mesh, 29)
    for hsc in (0.0, 0.25, 0.5, 2.0, 4.0):
        M = bchar.Mesh(mesh, layout, hash_scale=hsc)
        U = bchar.VelocityLattice(vel)
        T = bchar.Transfer.build(M, U, dt, bchar.opts_default(keep_pairs=1))
        a, b = T.export_pairs()
        o = np.lexsort((b, a))
        cin = torch.as_tensor(c0, device="cuda")
        cout = torch.empty_like(cin)
        T.step(cin, cout)
        out[hsc] = (a[o], b[o], T.export_csr(bchar.STAGE_V), cout.cpu().numpy())
    a0, b0, (rp0, col0, V0), c_ref = out[0.0]
    for hsc in (0.25, 0.5, 2.0, 4.0):
        a, b, (rp, col, V), c = out[hsc]
        assert np.array_equal(a, a0) and np.array_equal(b, b0), hsc
        assert np.array_equal(rp, rp0) and np.array_equal(col, col0), hsc
        dv = np.max(np.abs(V - V0)) / np.max(np.abs(V0))
        dc = np.max(np.abs(c - c_ref)) / np.max(np.abs(c_ref))
        _say(f"    scale {hsc}: V rel diff {dv:.3e}, c rel diff {dc:.3e}")
        assert dv <= 1e-15 and dc <= 1e-10


def test_hash_scale_rejected(env):
    torch, bchar = env
    mesh = inputs.cartesian_mesh((8, 8))
    for hsc in (0.1, 5.0, -1.0):
        with pytest.raises(bchar.BcharError) as ei:
            bchar.Mesh(mesh, "subcell", hash_scale=hsc)
        assert ei.value.status == bchar.E_INVALID_ARG
