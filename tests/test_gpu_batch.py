"""Concurrent builds (bchar_build_transfer_batch) give the same transfers as
builds run alone: the kernels are deterministic and a job depends only on
its own inputs and warm start, so every value must match bit for bit.  The
transfers built alone are the ones the oracle parity tests check."""

import sys

import numpy as np
import pytest

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


def _same(bchar, Ta, Tb):
    for stage in (bchar.STAGE_V, bchar.STAGE_SCALING, bchar.STAGE_ALL):
        ra, ca, va = Ta.export_csr(stage)
        rb, cb, vb = Tb.export_csr(stage)
        assert np.array_equal(ra, rb) and np.array_equal(ca, cb)
        assert np.array_equal(va.view(np.int64), vb.view(np.int64)), stage
    for k in ("qp_level", "qp_cg", "qp_ipm", "qp_newton", "nnz", "n_pairs"):
        assert Ta.stats[k] == Tb.stats[k], k


def _problems(bchar):
    w3 = inputs.swirl_hex(8)
    m3 = bchar.Mesh(w3["mesh"], "subcell")
    w2 = inputs.solid_body_32()
    m2 = bchar.Mesh(w2["mesh"], "equal_measure")
    tri = inputs.triangulated_square(10, 0.1, 6)
    mt = bchar.Mesh(tri, "equal_measure")
    vt = inputs.sample_velocity_grid((10, 10), inputs.rotation_stretch_2d)
    return [(m3, bchar.VelocityLattice(w3["vel_fn"](0)), 0.05),
            (m2, bchar.VelocityLattice(w2["vel_fn"](0)), w2["dt"]),
            (mt, bchar.VelocityLattice(vt), 0.3)]


def test_batch_builds_equal_builds_alone(env):
    torch, bchar = env
    probs = _problems(bchar)
    alone = [bchar.Transfer.build(m, v, dt) for m, v, dt in probs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(2)]
    _say("[gpu] batch of 3 jobs on 2 streams")
    got = bchar.build_batch([(None, m, v, dt) for m, v, dt in probs], streams=streams)
    for a, b in zip(alone, got):
        _same(bchar, a, b)
    # the same jobs again as rebuilds of the batch's transfers, each
    # warm-started from its own first solve, against rebuilds alone
    for a, (m, v, dt) in zip(alone, probs):
        a.rebuild(v, dt)
    torch.cuda.synchronize()
    got = bchar.build_batch([(t, None, v, dt) for t, (m, v, dt) in zip(got, probs)],
                            streams=streams)
    for a, b in zip(alone, got):
        _same(bchar, a, b)


def test_batch_warm_from_another_transfer(env):
    torch, bchar = env
    w = inputs.swirl_hex(10)
    M = bchar.Mesh(w["mesh"], "subcell")
    u = [bchar.VelocityLattice(w["vel_fn"](s)) for s in range(4)]
    dt = w["dt"] * 2
    # alone: the interval-1 transfer warm-started from the interval-0 solve
    ref = bchar.Transfer.build(M, u[0], dt)
    ref.rebuild(u[1], dt)
    ref2 = bchar.Transfer.build(M, u[0], dt)
    ref2.rebuild(u[2], dt)
    torch.cuda.synchronize()
    # batch: A (last solve on interval 0) is itself rebuilt on interval 2
    # while B (last solve on interval 3) takes A's interval-0 solve as its
    # warm start for interval 1: the warm start is taken before A changes
    A = bchar.Transfer.build(M, u[0], dt)
    B = bchar.Transfer.build(M, u[3], dt)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(2)]
    _say("[gpu] batch with warm_from")
    A, B = bchar.build_batch([(A, None, u[2], dt), (B, None, u[1], dt, A)], streams=streams)
    _same(bchar, ref, B)
    _same(bchar, ref2, A)
    # and the result is a valid step: mass and constants preserved
    c0 = torch.as_tensor(inputs.uniform_c(w["mesh"], 5), device="cuda")
    c1 = torch.empty_like(c0)
    B.step(c0, c1)
    m0, m1 = M.mass(c0), M.mass(c1)
    assert abs(m1 - m0) <= 1e-12 * abs(m0)


def test_batch_reports_the_failed_job(env):
    torch, bchar = env
    probs = _problems(bchar)
    m, v, dt = probs[0]
    # the second job is invalid (dt <= 0); the first still completes
    jobs = [(None, m, v, dt), (None, m, v, -1.0)]
    with pytest.raises(bchar.BcharError) as ei:
        bchar.build_batch(jobs, streams=[torch.cuda.Stream()])
    assert ei.value.status == bchar.E_INVALID_ARG
    assert "job 1" in str(ei.value)


def test_server_requests_equal_runs_alone(env):
    torch, bchar = env
    probs = _problems(bchar)
    steps = [3, 1, 4]
    g = torch.Generator().manual_seed(7)
    c0s = [torch.rand(m.n_cells, dtype=torch.float64, generator=g).cuda() for m, _, _ in probs]
    want = []
    for (m, v, dt), k, c0 in zip(probs, steps, c0s):
        T = bchar.Transfer.build(m, v, dt)
        c, nxt = c0.clone(), torch.empty_like(c0)
        for _ in range(k):
            T.step(c, nxt)
            c, nxt = nxt, c
        torch.cuda.synchronize()
        want.append(c.cpu().numpy())
        T.close()
    _say("[gpu] server: 6 requests on 2 workers")
    srv = bchar.Server(2)
    pending = []
    for rep in range(2):
        for i, ((m, v, dt), k, c0) in enumerate(zip(probs, steps, c0s)):
            out, tmp = torch.empty_like(c0), torch.empty_like(c0)
            pending.append((i, out, srv.submit(m, v, dt, k, c0, out, tmp)))
    for i, out, t in pending:
        r = srv.wait(t)
        assert r["status"] == bchar.OK
        assert r["t_submit"] <= r["t_start"] <= r["t_done"]
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.int64), want[i].view(np.int64)), i
        m = probs[i][0]
        m0, m1 = m.mass(c0s[i]), m.mass(out)
        assert abs(m1 - m0) <= 1e-12 * abs(m0)
    srv.close()


def test_server_admission_by_memory(env):
    """A memory budget below two requests: with two workers the second
    request starts only after the first has ended (its worker gives its
    buffers back), a request larger than the budget runs alone, and every
    result equals the same build and updates run alone, bit for bit."""
    torch, bchar = env
    probs = _problems(bchar)
    m, v, dt = probs[0]
    g = torch.Generator().manual_seed(11)
    c0 = torch.rand(m.n_cells, dtype=torch.float64, generator=g).cuda()
    T = bchar.Transfer.build(m, v, dt)
    nxt = torch.empty_like(c0)
    T.step(c0, nxt)
    torch.cuda.synchronize()
    want = nxt.cpu().numpy()
    held = T.stats["device_bytes"]
    T.close()
    assert held > 0
    _say(f"[gpu] server admission: a request holds {held} bytes")
    # declared bytes B, budget 1.5 B: one request at a time
    B = held
    srv = bchar.Server(2, mem_budget=int(1.5 * B))
    outs = [torch.empty_like(c0) for _ in range(3)]
    tickets = [srv.submit(m, v, dt, 1, c0, outs[i], nbytes=B) for i in range(2)]
    # larger than the budget: alone
    tickets.append(srv.submit(m, v, dt, 1, c0, outs[2], nbytes=2 * B))
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for r in res:
        assert r["status"] == bchar.OK
    assert res[1]["t_start"] >= res[0]["t_done"], "the second request did not wait"
    assert res[2]["t_start"] >= max(res[0]["t_done"], res[1]["t_done"])
    for o in outs:
        assert np.array_equal(o.cpu().numpy().view(np.int64), want.view(np.int64))


def test_cg_graph_replay_equals_eager_launches(env):
    """The CG iterations replayed from captured graphs (opts.cg_graphs)
    launch the same kernels on the same buffers as the eager loop: the
    transfers must agree bit for bit, on the null stream (captured on a
    stream of the solve's own) and on a side stream, and with kernel timing
    on, which runs one replay in `every` eagerly."""
    torch, bchar = env
    probs = _problems(bchar)
    w = inputs.swirl_hex(16)
    probs.append((bchar.Mesh(w["mesh"], "subcell"), bchar.VelocityLattice(w["vel_fn"](1)),
                  w["dt"] * 2))
    eager = bchar.opts_default(cg_graphs=0)
    graph = bchar.opts_default(cg_graphs=1)
    side = torch.cuda.Stream()
    for i, (m, v, dt) in enumerate(probs):
        _say(f"[gpu] cg graphs, problem {i}")
        a = bchar.Transfer.build(m, v, dt, opts=eager)
        b = bchar.Transfer.build(m, v, dt, opts=graph)
        with torch.cuda.stream(side):
            c = bchar.Transfer.build(m, v, dt, opts=graph, stream=side)
        side.synchronize()
        bchar.profile_kernel_sampled("k_zsmooth", 3)
        try:
            d = bchar.Transfer.build(m, v, dt, opts=graph)
            torch.cuda.synchronize()
            launches, ms = bchar.profile_read()
        finally:
            bchar.profile_kernel(None)
        assert a.stats["qp_cg"] > 0
        assert launches > 0 and ms > 0.0
        for t in (b, c, d):
            _same(bchar, a, t)
        # a rebuild (warm start) through the graphs too
        a.rebuild(v, dt, opts=eager)
        b.rebuild(v, dt, opts=graph)
        _same(bchar, a, b)
        for t in (a, b, c, d):
            t.close()


def test_cg_graph_replay_at_small_iteration_caps(env):
    """Where the cap on CG iterations cuts a replay short (caps 3, 6, 8: no
    replay, the first replay then single iterations, both replays) the
    graph path takes the same iterations as the eager loop: the same
    transfer bit for bit, or the same error."""
    torch, bchar = env
    w = inputs.swirl_hex(8)
    M = bchar.Mesh(w["mesh"], "subcell")
    U = bchar.VelocityLattice(w["vel_fn"](2))
    for cap in (3, 6, 8):
        _say(f"[gpu] cg cap {cap}")
        got = []
        for graphs in (0, 1):
            o = bchar.opts_default(cg_graphs=graphs, qp_max_cg=cap, qp_max_newton=60)
            try:
                got.append(("ok", bchar.Transfer.build(M, U, 0.05, opts=o)))
            except bchar.BcharError as e:
                st = e.stats or {}
                got.append(("err", (e.status, st.get("qp_cg"), st.get("qp_ipm"),
                                    st.get("qp_newton"), st.get("qp_level"))))
        assert got[0][0] == got[1][0], cap
        if got[0][0] == "ok":
            _same(bchar, got[0][1], got[1][1])
            for _, t in got:
                t.close()
        else:
            assert got[0][1] == got[1][1], cap


def test_tuner_picks_a_working_candidate(env):
    """bchar_tune_options times every candidate on the same jobs and never
    picks one whose builds fail; the transfers it builds are its own."""
    torch, bchar = env
    # a step too long for this mesh meets a void column: without halving the
    # build fails, with it the build succeeds
    q = inputs.mixed_problem(2, 400.0, 400.0)
    M = bchar.Mesh(q["mesh"], q["layout"])
    U = bchar.VelocityLattice(q["vel"])
    jobs = [(M, U, q["dt"])] + [(m, v, dt) for m, v, dt in _problems(bchar)[:1]]
    failing = bchar.opts_default()
    cands = [failing, bchar.opts_default(max_halvings=3),
             bchar.opts_default(max_halvings=3, cycle_skip=1)]
    streams = [torch.cuda.Stream() for _ in range(2)]
    _say("[gpu] tuner over 3 candidates")
    best, secs = bchar.tune_options(jobs, cands, streams, rounds=2)
    _say(f"    best {best}, seconds {secs}")
    assert best in (1, 2)
    assert secs[0] == float("inf")
    assert all(0.0 < s < float("inf") for s in secs[1:])
    assert secs[best] == min(secs)


def test_halving_when_negative_volumes_are_needed(env):
    """A request of the served workload (a 55^3 hexahedral cube, CFL 2.15)
    whose least-change problem needs level 2 -- the equalities alone, so
    volumes turn negative and 44 updates grow without bound (the porous mass
    drifts by 200 %).  With opts.halve_on_level2 the library builds half
    steps instead: a level with non-negative volumes, the same bits as the
    half-step transfer built directly and applied twice, and the mass kept
    to 1e-12 over the 44 updates."""
    torch, bchar = env
    _say("[gpu] halving when the box needs level 2")
    q = inputs.mixed_problem(1000, n_hi=2e6)
    M = bchar.Mesh(q["mesh"], q["layout"])
    U = bchar.VelocityLattice(q["vel"])
    T = bchar.Transfer.build(M, U, q["dt"], bchar.opts_default(max_halvings=4,
                                                                halve_on_level2=1))
    st = T.stats
    _say(f"    stats {st}")
    h = st["dt_halvings"]
    assert h >= 1 and st["qp_level"] <= 1
    Th = bchar.Transfer.build(M, U, q["dt"] / 2 ** h)
    assert Th.stats["qp_level"] == st["qp_level"]
    c0 = torch.as_tensor(q["c0"], device="cuda")
    a, b = c0.clone(), torch.empty_like(c0)
    T.step(a, b)
    x, y = c0.clone(), torch.empty_like(c0)
    for _ in range(2 ** h):
        Th.step(x, y)
        x, y = y, x
    assert torch.equal(b, x)
    m0 = M.mass(c0)
    for _ in range(44):
        T.step(a, b)
        a, b = b, a
    assert abs(M.mass(a) - m0) <= 1e-12 * abs(m0)
