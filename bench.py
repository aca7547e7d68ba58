"""Benchmark of the B-char transfer build and apply on one MI355X.

Workload (default): the 3D swirl on the unit cube, 64^3 hexahedra
(262,144 cells), 8 balls per cell (sub-cell layout), phi = 1, dt = 1/128,
the divergence-free swirl sampled at the middle of each step, FP64, the
transfer rebuilt every step (the field depends on time).  One step = the
whole hot path: tracking, overlap search, lens volumes, V, the N = 10
scaling sweeps, the bounded least-change problem, the update of c, and the
porous mass (checked against the initial mass at every step).

The velocity of every interval is prescribed (it does not depend on c), so
the transfers of successive intervals are independent: the run first
builds them one after another (per-step latency, reported under
"sequential"), then ``--inflight`` of them at once, each on its own stream
and host worker (bchar_build_transfer_batch), applying them in order.

Prints one JSON line.  ``value`` counts cell updates per second over the
timed steps of the second run; a run whose relative mass error exceeds
1e-12 at any step is reported with ``"mass_ok": false``.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 64] [--precision fp64|fp32]
                    [--inflight D]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
SRC = os.path.join(ROOT, "paper_1908_05834_amd", "csrc")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, n_cells, nnz, n_balls, stats):
    """Bytes a launch of ``kernel`` must move at least (each array read or
    written once; gathers of vector entries counted once per cell)."""
    if kernel == "k_smooth":
        # one Jacobi sweep of a launched multigrid level (row pointers,
        # neighbours and weights, diagonal, smoother step, right-hand side
        # and iterate in, iterate out), mean over the sweeps of one cycle,
        # as counted by the library for the last solve
        return stats["qp_smooth_bytes"]
    if kernel == "k_fused_cycle":
        # the coarsest levels of the preconditioner, one workgroup: their
        # graphs, diagonals, right-hand sides, aggregation and the dense
        # inverse, as counted by the library for the last solve
        return stats["qp_coarse_bytes"]
    if kernel == "k_zsmooth":
        # per cell: s,g in (16), rhs (16), block inverse (24), shifts (16),
        # row_ptr and col_ptr (8), diagonal position (4), out (16); per
        # entry, once in the CSR pass and once in the CSC pass: index (4) and
        # weight (8)
        return n_cells * (16 + 16 + 24 + 16 + 8 + 4 + 16) + 2 * nnz * 12
    if kernel == "k_zop":
        return n_cells * (16 + 16 + 8 + 4 + 16) + 2 * nnz * 12
    if kernel == "k_assemble":
        # one launch per build: the build stage's 385 bytes per cell less
        # the velocity (read by the trace) -- the residing balls through the
        # hash (32 per ball), the bucket offsets (32 per cell), phi, |K| and
        # rho (16 per cell), the CSR rows (12 per entry, 4 per cell) -- plus
        # the tracked centres and radii the separate trace kernel wrote (32
        # per ball)
        return n_balls * 32 + n_cells * (32 + 16 + 4) + nnz * 12 + n_balls * 32
    if kernel == "k_trace":
        # ball centre in (24 per ball), tracked centre and radius out (32
        # per ball), the velocity lattice (24 per node, about one node per
        # cell)
        return n_balls * (24 + 32) + n_cells * 24
    raise KeyError(kernel)


# the sources each measured kernel's device code comes from (its file and
# the header of device helpers; the other headers declare host code only)
KERNEL_SOURCES = {"k_assemble": "build.hip", "k_trace": "build.hip"}


def source_digest(kernel):
    """Digest of the code of ``kernel``'s sources (comments and layout left
    out): a measured traffic figure is valid only for the code it was
    measured on."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES[kernel], "device_util.hpp"):
        with open(os.path.join(SRC, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        text = re.sub(r"\s+", " ", text)
        h.update((f + text).encode())
    return h.hexdigest()[:16]


CSWIRL_SQUEEZE = 0.1   # compression amplitude of the non-solenoidal workload


def workload_key(workload, n, precision):
    """The configuration a traffic figure belongs to: workload, size and
    precision (the kernels measured are those of the build, which the
    solver's options do not touch)."""
    return f"{workload}-{n}-{precision}"


def measured_traffic(kernel, workload_key):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 --pmc
    measurement (profiles/traffic_<kernel>.json), or None when there is
    none, it was taken on another workload, or the sources changed since
    it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("workload_key") != workload_key:
        return None
    if rec.get("source_digest") != source_digest(kernel):
        return None
    return rec.get("bytes_per_launch")


def copy_calibration(mib):
    """A plain device copy of ``mib`` MiB, for scaling the FETCH_SIZE and
    WRITE_SIZE counters against a kernel of known traffic."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "bytes_read": n * 8, "bytes_written": n * 8,
                      "launches": 3}))


TRAFFIC_KERNELS = ("k_assemble", "k_trace")


def kernel_base_name(name):
    """'void bchar::k_assemble<3, double, true>(bchar::AsmParams)' -> 'k_assemble'."""
    base = name.split("(")[0].split("<")[0].strip()
    return base.split("::")[-1].split(" ")[-1]


def pmc_summary(prof_dir, counter, out):
    """Sum one rocprofv3 --pmc counter (CSV output under ``prof_dir``) per
    dispatch of the kernels whose traffic bench.py reports and of the
    device copy used for calibration; write the per-dispatch means (KiB)."""
    import csv
    import glob
    files = glob.glob(os.path.join(prof_dir, "**", "*counter_collection*.csv"), recursive=True)
    tot = {}
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                name = r.get("Kernel_Name", "")
                base = kernel_base_name(name)
                key = base if base in TRAFFIC_KERNELS else None
                if key is None and "copy" in name.lower():
                    key = "copy: " + name[:80]
                if key is None:
                    continue
                d = tot.setdefault(key, {"dispatches": set(), "sum": 0.0})
                d["dispatches"].add(r.get("Dispatch_Id"))
                d["sum"] += float(r["Counter_Value"])
    res = {k: {"dispatches": len(v["dispatches"]),
               "kib_per_dispatch": v["sum"] / max(1, len(v["dispatches"]))} for k, v in tot.items()}
    with open(out, "w") as fh:
        json.dump({"counter": counter, "kernels": res}, fh, indent=1)
    print(json.dumps(res))


def write_traffic(fetch, write, copy_fetch, copy_write, copy_mib, commands, workload, key):
    """profiles/traffic_<kernel>.json from the four counter summaries: the
    kernel's FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    same counter reads for a plain device copy of copy_mib MiB (read once,
    written once)."""
    def load(p):
        with open(p) as fh:
            return json.load(fh)["kernels"]
    f, w, cf, cw = load(fetch), load(write), load(copy_fetch), load(copy_write)
    copy_kib = copy_mib * 1024.0

    def copy_of(d):
        # the device copy: the copy kernel moving the most data
        return max((v for k, v in d.items() if k.startswith("copy")),
                   key=lambda v: v["kib_per_dispatch"])
    ccf, ccw = copy_of(cf), copy_of(cw)
    ff = copy_kib / ccf["kib_per_dispatch"]
    wf = copy_kib / ccw["kib_per_dispatch"]
    for k in TRAFFIC_KERNELS:
        if k not in f or k not in w:
            continue
        rec = {"kernel": k, "workload": workload, "workload_key": key,
               "commands": commands,
               "dispatches": f[k]["dispatches"],
               "fetch_kib_per_dispatch": f[k]["kib_per_dispatch"],
               "write_kib_per_dispatch": w[k]["kib_per_dispatch"],
               "copy_calibration": {"copy_kib": copy_kib,
                                    "fetch_kib_per_dispatch": ccf["kib_per_dispatch"],
                                    "write_kib_per_dispatch": ccw["kib_per_dispatch"],
                                    "fetch_factor": ff, "write_factor": wf},
               "bytes_per_launch": 1024.0 * (f[k]["kib_per_dispatch"] * ff +
                                             w[k]["kib_per_dispatch"] * wf),
               "source_digest": source_digest(k)}
        with open(os.path.join(ROOT, "profiles", f"traffic_{k}.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        print(k, rec["bytes_per_launch"])


def cpu_baseline(sample_n=16, workload="swirl"):
    """The oracle timed on the host: one full time step (build + apply) of
    the same workload on a reduced mesh (sample_n^3 hexahedra, or
    sample_n^3 cubes of 6 tetrahedra), one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import transfer as otr
    from paper_1908_05834_amd import inputs

    solenoidal = True
    if workload == "tets":
        w = inputs.jittered_tets(sample_n, steps=1)
        layout, prec, what = "equal_measure", "fp32", "jittered tetrahedra"
        n_cells = 6 * sample_n ** 3
    elif workload == "cswirl":
        w = inputs.compressible_swirl_hex(sample_n, squeeze=CSWIRL_SQUEEZE)
        layout, prec, what = "subcell", "fp64", "hexahedra, 8 balls per cell, non-solenoidal u"
        n_cells = sample_n ** 3
        solenoidal = False
    else:
        w = inputs.swirl_hex(sample_n)
        layout, prec, what = "subcell", "fp64", "hexahedra, 8 balls per cell"
        n_cells = sample_n ** 3
    with threadpool_limits(1):
        t0 = time.perf_counter()
        T = otr.build_transfer(w["mesh"], w["vel_fn"](0), w["dt"], layout=layout,
                               precision=prec, solenoidal=solenoidal)
        c1 = otr.apply(T["row_ptr"], T["col"], T["A"], T["b"], w["c0"])
        t1 = time.perf_counter()
    assert np.all(np.isfinite(c1))
    model, ncpu = host_cpu()
    return {"value": n_cells / (t1 - t0), "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle", "cpu_model": model, "host_cores": ncpu,
            "sample": f"one step (build + apply) of the {workload} workload on a "
                      f"{sample_n}^3 grid ({n_cells} cells, {what}, {prec.upper()}), "
                      f"{t1 - t0:.2f} s single-threaded"}


def host_cpu():
    """Model name of the host CPU and the number of cores the OS reports."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline_swirl64():
    """The oracle on the host cores, one thread, on the headline workload
    itself (64^3 hexahedra, 8 balls per cell, FP64): one step through the
    tracking, candidate pairs, V and the N = 10 scaling sweeps.  Its
    least-change solve does not finish in practical time at this size (a
    full step takes about 80 s at 24^3 and more than 20 minutes at 32^3),
    so the rate counts these stages only: an upper bound on the oracle's
    full-step rate.  A full oracle step at 16^3 is given beside it."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import transfer as otr
    from paper_1908_05834_amd import inputs

    model, ncpu = host_cpu()
    w = inputs.swirl_hex(64)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        T = otr.build_transfer(w["mesh"], w["vel_fn"](0), w["dt"], layout="subcell",
                               stop_after="sinkhorn")
        t1 = time.perf_counter()
        w16 = inputs.swirl_hex(16)
        t2 = time.perf_counter()
        T16 = otr.build_transfer(w16["mesh"], w16["vel_fn"](0), w16["dt"], layout="subcell")
        c16 = otr.apply(T16["row_ptr"], T16["col"], T16["A"], T16["b"], w16["c0"])
        t3 = time.perf_counter()
    assert np.all(np.isfinite(T["AN"])) and np.all(np.isfinite(c16))
    nc = 64 ** 3
    return {"value": nc / (t1 - t0), "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one step of the 64^3 swirl (262,144 cells, 8 balls per cell, FP64) "
                      f"through tracking, candidate pairs, V and the 10 scaling sweeps, "
                      f"{t1 - t0:.1f} s single-threaded (the least-change solve left out: "
                      f"an upper bound on the oracle's full-step rate)",
            "full_step_16": {"value": 16 ** 3 / (t3 - t2), "seconds": t3 - t2,
                             "cells": 16 ** 3},
            "cpu_model": model, "host_cores": ncpu}


def bench_mixed(args):
    """A batch of independent small problems (inputs.mixed_problem, seeds
    0 .. problems-1): every transfer built once and applied 10 times, first
    one problem after another, then with ``inflight`` workers taking the
    next build whenever they are free (up to 64 builds a call).  Meshes,
    velocity lattices and c^0 are resident on the device before timing;
    transfers are released once applied.  ``value`` counts 10 updates of
    every cell of every problem (the simulated time span), also where a
    void made the time step halve."""
    import numpy as np
    import torch

    from paper_1908_05834_amd import bchar, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    D = max(1, args.inflight)
    # a void makes the library repeat the build with half the step
    opts = bchar.opts_default(max_halvings=4)
    probs = []
    for p in range(args.problems):
        q = inputs.mixed_problem(p)
        log(f"problem {p}: {q['name']}, {inputs.n_cells(q['mesh'])} cells, CFL {q['cfl']:.2f}")
        q["M"] = bchar.Mesh(q["mesh"], q["layout"])
        q["U"] = bchar.VelocityLattice(q["vel"])
        q["c0_dev"] = torch.as_tensor(q["c0"], device="cuda")
        q["m0"] = q["M"].mass(q["c0_dev"])
        probs.append(q)
    cells = sum(q["M"].n_cells for q in probs)
    steps = probs[0]["steps"]
    mass_err = 0.0

    def finish(q, T):
        nonlocal mass_err
        c = q["c0_dev"].clone()
        nxt = torch.empty_like(c)
        for _ in range(steps):
            T.step(c, nxt)
            c, nxt = nxt, c
        m = q["M"].mass(c)
        mass_err = max(mass_err, abs(m - q["m0"]) / abs(q["m0"]))
        T.close()

    def run(depth):
        streams = [torch.cuda.Stream() for _ in range(depth)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cg = []
        levels = [0, 0, 0]
        halvings = 0
        per_call = 64 if depth > 1 else 1
        for b0 in range(0, len(probs), per_call):
            chunk = probs[b0:b0 + per_call]
            Ts = bchar.build_batch([(None, q["M"], q["U"], q["dt"]) for q in chunk], opts, streams)
            for q, T in zip(chunk, Ts):
                cg.append(T.stats["qp_cg"])
                levels[T.stats["qp_level"]] += 1
                halvings += T.stats["dt_halvings"]
                finish(q, T)
            if depth > 1 or b0 % 16 == 15:
                log(f"  depth {depth}: problems up to {min(b0 + per_call, len(probs)) - 1} done "
                    f"at {time.perf_counter() - t0:.2f} s")
        torch.cuda.synchronize()
        return time.perf_counter() - t0, cg, halvings, levels

    run(D)   # warm-up pass (code objects, allocator)
    t_seq, cg_seq, _, _ = run(1)
    log(f"mixed, one at a time: {t_seq:.3f} s")
    t_par, cg_par, halvings, levels = run(D)
    log(f"mixed, {D} in flight: {t_par:.3f} s, {halvings} time steps halved")
    assert cg_seq == cg_par
    out = {
        "metric": "B-char cell-updates/s, batch of independent problems (build once + 10 applies)",
        "value": cells * steps / t_par,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": t_par / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(probs)} independent problems (seeds 0..{len(probs) - 1}): "
                               "2D triangulated squares or 3D hexahedral cubes, N ~ "
                               "logU[4e3, 2e5] cells, four Fourier modes, CFL ~ U[0.5, 4]",
                   "problems": len(probs), "cells_total": cells, "inflight_builds": D,
                   "dt_halvings": halvings,
                   "qp_cg_mean": float(np.mean(cg_par)),
                   "qp_levels": {"paper_box": levels[0], "nonnegative": levels[1],
                                 "equalities_only": levels[2]}},
        "mass_ok": bool(mass_err <= 1e-12),
        "max_rel_mass_err": mass_err,
        "sequential": {"value": cells * steps / t_seq, "seconds": t_seq},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def serve_run(requests, rate, seed, problems, workers, mem_budget_gib, per_request_mesh,
              serial, n_hi=2.0e5):
    """Requests arriving as a Poisson process (seeded) at ``rate`` per
    second; each builds the transfer of one step and applies it U{1..50}
    times.  With resident meshes the problem is drawn from a pool of
    ``problems`` (inputs.mixed_problem); with ``per_request_mesh`` every
    request draws its own problem (mixed_problem of seed 1000 + i, up to
    ``n_hi`` cells) and creates its mesh on arrival, destroyed once its
    result is in.  The server (bchar_server_*) runs them with ``workers``
    workers (and again with one when ``serial``).  Latency is arrival to
    result."""
    import threading

    import numpy as np
    import torch

    from paper_1908_05834_amd import bchar, inputs

    torch.cuda.set_device(0)
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    nsteps = rng.integers(1, 51, size=requests)
    pool = []
    if per_request_mesh:
        descs = [inputs.mixed_problem(1000 + i, n_hi=n_hi) for i in range(requests)]
        which = np.arange(requests)
    else:
        for p in range(problems):
            q = inputs.mixed_problem(p)
            M = bchar.Mesh(q["mesh"], q["layout"])
            c0 = torch.as_tensor(q["c0"], device="cuda")
            pool.append({"M": M, "U": bchar.VelocityLattice(q["vel"]), "dt": q["dt"],
                         "c0": c0, "m0": M.mass(c0)})
        which = rng.integers(0, len(pool), size=requests)

    def run(nw, label):
        # a void makes the library repeat the build with half the step
        srv = bchar.Server(nw, mem_budget=int(mem_budget_gib * (1 << 30)),
                           opts=bchar.opts_default(max_halvings=4))
        if pool:
            # warm-up: every pool problem once (worker buffers reach their size)
            for q in pool:
                out, tmp = torch.empty_like(q["c0"]), torch.empty_like(q["c0"])
                srv.wait(srv.submit(q["M"], q["U"], q["dt"], 1, q["c0"], out, tmp))
        results = [None] * requests
        tickets = [None] * requests
        held = [None] * requests
        pre = [0.0] * requests   # arrival to submission (mesh creation), seconds
        ready = threading.Semaphore(0)

        def collect():
            for i in range(requests):
                ready.acquire()
                results[i] = srv.wait(tickets[i])
                q = held[i]["q"]
                m = q["M"].mass(held[i]["out"])
                results[i]["mass_err"] = abs(m - q["m0"]) / abs(q["m0"])
                results[i]["t_arrival"] = results[i]["t_submit"] - pre[i]
                results[i]["cells"] = q["M"].n_cells
                if per_request_mesh:
                    q["M"].close()
                held[i] = None
                r = results[i]
                log(f"  {label}: request {i} done, {r['cells']} cells, status {r['status']}, "
                    f"halvings {r['stats']['dt_halvings']}, build+updates "
                    f"{r['t_done'] - r['t_start']:.2f} s, latency "
                    f"{r['t_done'] - r['t_arrival']:.2f} s")
        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for i in range(requests):
            dly = t0 + arrivals[i] - time.perf_counter()
            if dly > 0:
                time.sleep(dly)
            ta = time.perf_counter()
            if per_request_mesh:
                d = descs[i]
                M = bchar.Mesh(d["mesh"], d["layout"])
                c0 = torch.as_tensor(d["c0"], device="cuda")
                q = {"M": M, "U": bchar.VelocityLattice(d["vel"]), "dt": d["dt"], "c0": c0,
                     "m0": M.mass(c0)}
            else:
                q = pool[which[i]]
            out, tmp = torch.empty_like(q["c0"]), torch.empty_like(q["c0"])
            held[i] = {"q": q, "out": out, "tmp": tmp}
            pre[i] = time.perf_counter() - ta
            tickets[i] = srv.submit(q["M"], q["U"], q["dt"], int(nsteps[i]), q["c0"], out, tmp)
            ready.release()
            if i % 20 == 19:
                log(f"  {label}: {i + 1} requests submitted at {time.perf_counter() - t0:.1f} s")
        th.join()
        srv.close()
        ok = all(r["status"] == bchar.OK for r in results)
        lat = np.array([r["t_done"] - r["t_arrival"] for r in results])
        span = max(r["t_done"] for r in results) - min(r["t_arrival"] for r in results)
        cu = sum(r["cells"] * int(nsteps[i]) for i, r in enumerate(results))
        # requests whose least-change problem needed level 2 (the equalities
        # alone) carry negative volumes: their updates conserve the mass in
        # exact arithmetic but grow, and rounding then shows in the mass;
        # they are counted apart
        l2 = [r for r in results if r["stats"]["qp_level"] == 2]
        merr = max([r["mass_err"] for r in results if r["stats"]["qp_level"] < 2], default=0.0)
        log(f"{label}: {span:.2f} s, p50 {np.percentile(lat, 50) * 1e3:.0f} ms, "
            f"p99 {np.percentile(lat, 99) * 1e3:.0f} ms")
        return {"value": cu / span, "unit": "cell-updates/s", "seconds": span, "ok": ok,
                "max_rel_mass_err": merr, "requests": requests, "rate_per_s": rate,
                "workers": nw, "cells_mean": float(np.mean([r["cells"] for r in results])),
                "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
                "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
                "mass_ok": bool(ok and merr <= 1e-12),
                "level2_requests": len(l2),
                "level2_max_rel_mass_err": max([r["mass_err"] for r in l2], default=None)}

    out = run(workers, f"{workers} workers")
    if serial:
        out["serial"] = run(1, "1 worker")
    out["per_request_mesh"] = bool(per_request_mesh)
    return out


def bench_serve(args):
    """The served workload alone: ``--requests`` Poisson arrivals at
    ``--rate`` per second, served with ``--inflight`` workers and then by
    one (the serial path) on the same arrivals."""
    D = max(1, args.inflight)
    r = serve_run(args.requests, args.rate, args.seed, args.problems, D, args.mem_budget_gib,
                  bool(args.per_request_mesh), True, args.n_hi)
    where = ("a mesh created per request (mixed problems up to "
             f"{args.n_hi:.0f} cells)" if args.per_request_mesh else
             f"problems drawn from {args.problems} resident meshes")
    out = {
        "metric": "B-char served cell-updates/s and p99 latency (arrival to result)",
        "value": r["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": 0 if args.per_request_mesh else args.problems,
        "ms_per_step": r["seconds"] / args.requests * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.requests} requests, Poisson arrivals at {args.rate}/s "
                               f"(seed {args.seed}), {where}, U{{1..50}} updates each",
                   "workers": D, "mem_budget_gib": args.mem_budget_gib,
                   "latency_ms_p50": r["latency_ms_p50"],
                   "latency_ms_p99": r["latency_ms_p99"]},
        "mass_ok": bool(r["mass_ok"] and r["serial"]["mass_ok"]),
        "max_rel_mass_err": max(r["max_rel_mass_err"], r["serial"]["max_rel_mass_err"]),
        "serial": r["serial"],
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--n", type=int, default=None,
                    help="cells per axis (swirl: 64; tets: 96 cubes of 6 tetrahedra)")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default=None,
                    help="swirl: fp64 by default; tets: fp32 (binary32 volumes)")
    ap.add_argument("--inflight", type=int, default=4,
                    help="transfers built at once on separate streams (1: one after another)")
    ap.add_argument("--build-kernel", default="k_assemble")
    ap.add_argument("--trace-kernel", default="k_trace")
    ap.add_argument("--legs", type=int, choices=[0, 1], default=1,
                    help="swirl: also run the FP32-volume leg and the served leg")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="served leg: requests")
    ap.add_argument("--serve-rate", type=float, default=3.0,
                    help="served leg: Poisson arrivals per second")
    ap.add_argument("--serve-problems", type=int, default=16,
                    help="served leg: resident problems the requests draw from")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a device copy of this many MiB (counter calibration)")
    ap.add_argument("--cg-graphs", type=int, choices=[0, 1], default=1,
                    help="replay the CG iterations from captured HIP graphs (1) or launch "
                         "every kernel from the host (0)")
    ap.add_argument("--cycle-skip", type=int, choices=[0, 1], default=0,
                    help="multigrid cycle visiting every other level (opts.cycle_skip), "
                         "with --tune 0")
    ap.add_argument("--tune", type=int, choices=[0, 1], default=1,
                    help="swirl/tets: choose cycle_skip by measuring both (bchar_tune_options)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--workload", choices=["swirl", "cswirl", "tets", "mixed", "serve"],
                    default="swirl")
    ap.add_argument("--rate", type=float, default=4.0, help="serve: arrivals per second")
    ap.add_argument("--requests", type=int, default=120, help="serve: number of requests")
    ap.add_argument("--seed", type=int, default=0, help="serve: arrival seed")
    ap.add_argument("--mem-budget-gib", type=float, default=64.0,
                    help="serve: device memory the workers may hold")
    ap.add_argument("--per-request-mesh", type=int, choices=[0, 1], default=0,
                    help="serve: create each request's mesh on arrival (and destroy it "
                         "after), instead of drawing from resident meshes")
    ap.add_argument("--n-hi", type=float, default=2.0e5,
                    help="serve with --per-request-mesh: largest mesh (cells)")
    ap.add_argument("--problems", type=int, default=32,
                    help="mixed workload: number of problems (seeds 0 .. problems-1)")
    ap.add_argument("--pmc-sum", nargs=3, metavar=("PROF_DIR", "COUNTER", "OUT"),
                    help="only summarise a rocprofv3 --pmc run (no device work)")
    ap.add_argument("--traffic-json", nargs=5,
                    metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE", "COPY_MIB"),
                    help="only write profiles/traffic_<kernel>.json from four summaries")
    args = ap.parse_args()

    if args.pmc_sum:
        pmc_summary(*args.pmc_sum)
        return
    if args.traffic_json:
        fe, wr, cfe, cwr, mib = args.traffic_json
        cmd = "rocprofv3 --pmc {c} --output-format csv -d /tmp/pmc_{t} -o p -- python3 bench.py {a}"
        run = "--steps 1 --warmup 1 --inflight 1 --legs 0 --no-cpu-baseline --tune 0"
        write_traffic(fe, wr, cfe, cwr, int(mib),
                      [cmd.format(c="FETCH_SIZE", t="f", a=run),
                       cmd.format(c="WRITE_SIZE", t="w", a=run),
                       cmd.format(c="FETCH_SIZE", t="cf", a=f"--copy-calibration {mib}"),
                       cmd.format(c="WRITE_SIZE", t="cw", a=f"--copy-calibration {mib}")],
                      "3D swirl, 64^3 hexahedra, 8 balls per cell, FP64",
                      workload_key("swirl", 64, "fp64"))
        return

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    D = max(1, args.inflight)
    if D > 1:
        # one hardware queue per build stream, plus the default stream (set
        # before the HIP runtime starts)
        q = max(int(os.environ.get("GPU_MAX_HW_QUEUES", "4")), D + 2)
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(q, 32))
    if args.workload == "mixed":
        bench_mixed(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(torch.device("cuda:0"))
    args.precision = args.precision or ("fp32" if args.workload == "tets" else "fp64")
    args.n = args.n or (96 if args.workload == "tets" else 64)
    res = run_transport(args, args.workload, args.precision, args.steps, args.warmup, D,
                        bool(args.tune))
    out = {
        "metric": res["metric"],
        "value": res["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": res["steps_timed"],
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": res["dtype"],
        "data": "synthetic",
        "config": res["config"],
        "mass_ok": res["mass_ok"],
        "max_rel_mass_err": res["max_rel_mass_err"],
        "sequential": res["sequential"],
        "roofline": res["roofline"],
        "roofline_build_stage": res["roofline_build_stage"],
        "roofline_step": res["roofline_step"],
        "cpu_baseline": None,
    }
    if args.workload == "swirl" and args.legs:
        # the FP32-volume mode on the same workload (binary32 tracking and
        # lenses, binary64 adjustment), fewer steps
        log("FP32-volume leg")
        r32 = run_transport(args, "swirl", "fp32", max(4, args.steps // 2), args.warmup, D,
                            False)
        out["fp32_volume"] = {"value": r32["value"], "ms_per_step": r32["ms_per_step"],
                              "steps": r32["steps_timed"], "mass_ok": r32["mass_ok"],
                              "max_rel_mass_err": r32["max_rel_mass_err"],
                              "sequential": r32["sequential"],
                              "qp_cg_mean": r32["config"]["qp_cg_mean"],
                              "trace_precision": r32["config"]["trace_precision"]}
        # served requests: continuous batching with p50 / p99 latency
        log("served leg")
        sv = serve_run(requests=args.serve_requests, rate=args.serve_rate, seed=0,
                       problems=args.serve_problems, workers=D, mem_budget_gib=64.0,
                       per_request_mesh=False, serial=False)
        out["served"] = sv
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = (cpu_baseline_swirl64() if args.workload == "swirl" and args.n == 64
                               else cpu_baseline(args.cpu_sample if args.workload in ("swirl", "cswirl")
                                                 else 6, args.workload))
    print(json.dumps(out))


def step_bytes_per_cell(cg_iterations):
    """Algorithmic bytes of one whole step per cell (the build 385, the
    transposed pattern 35, the N = 10 scaling sweeps 1,500, 150 per CG
    iteration of the least-change solve, the update 73 and the mass 24)."""
    return 385 + 35 + 1500 + 150 * cg_iterations + 73 + 24


def run_transport(args, workload, precision, steps, warmup, D, tune):
    """The transfer of every step rebuilt and applied: first one build after
    another (per-step latency; the build kernel timed with HIP events on
    these steps), then D builds at once on their own streams (throughput).
    Returns the measured figures."""
    import numpy as np
    import torch

    from paper_1908_05834_amd import bchar, inputs

    dev = torch.device("cuda:0")
    if workload == "tets":
        n = args.n or 96
        w = inputs.jittered_tets(n, steps=max(warmup + steps, 3))
        layout = "equal_measure"
        desc = (f"3D jittered Kuhn tetrahedra, {n}^3 cubes x 6 = {6 * n ** 3} "
                f"cells, lognormal phi, swirl at CFL 4, one centroid ball per cell, "
                f"dt = 1/128, transfer rebuilt every step")
        metric = (f"B-char cell-updates/s (3D tets {6 * n ** 3}) at 1e-12 mass err; "
                  "served p99 latency")
    elif workload == "cswirl":
        n = args.n or 64
        w = inputs.compressible_swirl_hex(n, squeeze=CSWIRL_SQUEEZE)
        layout = "subcell"
        desc = (f"3D swirl plus a sine compression of amplitude {CSWIRL_SQUEEZE} per axis "
                f"(non-solenoidal),"
                f" unit cube, {n}^3 hexahedra, 8 balls per cell, phi = 1, dt = 1/128, "
                f"transfer rebuilt every step")
        metric = (f"B-char cell-updates/s (3D hex {n}^3, non-solenoidal u) at 1e-12 mass err; "
                  "served p99 latency")
    else:
        n = args.n or 64
        w = inputs.swirl_hex(n)
        layout = "subcell"
        desc = (f"3D swirl, unit cube, {n}^3 hexahedra, 8 balls per cell, "
                f"phi = 1, dt = 1/128, transfer rebuilt every step")
        metric = "B-char cell-updates/s (3D hex 64^3) at 1e-12 mass err; served p99 latency"
    # binary32 tracking (FP32_VOLUME) needs a constant porosity; the porous
    # unstructured workload tracks in binary64 with binary32 lenses
    prec = bchar.FP64 if precision == "fp64" else (
        bchar.FP32_LENS if workload in ("tets", "cswirl") else bchar.FP32_VOLUME)
    div = bchar.DIV_GENERAL if workload == "cswirl" else bchar.DIV_FREE
    opts = bchar.opts_default(precision=prec, cg_graphs=args.cg_graphs,
                              cycle_skip=args.cycle_skip, divergence=div)
    M = bchar.Mesh(w["mesh"], layout)
    seq_total = warmup + steps
    warm_batches = max(1, math.ceil(warmup / D))
    timed_batches = max(1, math.ceil(steps / D))
    steps_timed = timed_batches * D if D > 1 else steps
    pipe_first = max(0, warmup - warm_batches * D)
    pipe_total = pipe_first + (warm_batches + timed_batches) * D if D > 1 else 0
    vels = [bchar.VelocityLattice(w["vel_fn"](s % w["steps"]))
            for s in range(max(seq_total, pipe_total, 3))]
    c0 = torch.as_tensor(w["c0"], device=dev)
    m0 = M.mass(c0)
    mass_err = 0.0

    def apply(T, c, nxt):
        nonlocal mass_err
        T.step(c, nxt)
        m = M.mass(nxt)
        e = abs(m - m0) / abs(m0)
        mass_err = max(mass_err, e)
        return nxt, c, e

    streams = [torch.cuda.Stream() for _ in range(D)]
    tuned = None
    if tune:
        # the bucket side of the spatial hash (a mesh option: the same
        # pairs whichever is chosen), timed on builds that stop after V in
        # alternating rounds; another side only when it beats the default
        # by 3 %
        hscales = [1.0, 0.5, 2.0]
        hmeshes = [M] + [bchar.Mesh(w["mesh"], layout, hash_scale=h) for h in hscales[1:]]
        vopt = bchar.opts_default(precision=prec, stop_after=bchar.STAGE_V, divergence=div)
        htimes = [[] for _ in hscales]
        for _ in range(6):
            for i, Mi in enumerate(hmeshes):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                built = bchar.build_batch([(None, Mi, vels[j % len(vels)], w["dt"])
                                           for j in range(D)], vopt, streams)
                torch.cuda.synchronize()
                htimes[i].append(time.perf_counter() - t0)
                for Tb in built:
                    Tb.close()
        hsecs = [float(np.median(x)) for x in htimes]
        hb = int(np.argmin(hsecs))
        if not hsecs[hb] < 0.97 * hsecs[0]:
            hb = 0
        for i, Mi in enumerate(hmeshes):
            if i != hb:
                Mi.close()
        M = hmeshes[hb]
        log(f"tuned: hash_scale {hscales[hb]} ({', '.join(f'{x:.4f}' for x in hsecs)} s)")
        jobs = [(M, vels[j % len(vels)], w["dt"]) for j in range(D)]
        # the assembly's tile shape and LDS staging, timed on builds that
        # stop after V (the same transfer bit for bit whichever is chosen)
        shapes = [(a, l) for a in (0, 1, -1) for l in (0, 1)]
        kc = [bchar.opts_default(precision=prec, stop_after=bchar.STAGE_V, tile_aspect=a,
                                 lds_stage=l, divergence=div) for a, l in shapes]
        kb, ksecs = bchar.tune_options(jobs, kc, streams, rounds=6)
        # these builds are short and their times close: another shape is
        # taken only when it beats the default by 3 %
        if not ksecs[kb] < 0.97 * ksecs[0]:
            kb = 0
        aspect, lds = shapes[kb]
        log(f"tuned: tile_aspect {aspect}, lds_stage {lds} "
            f"({', '.join(f'{x:.4f}' for x in ksecs)} s)")
        # the multigrid cycle, timed on whole builds
        cands = [bchar.opts_default(precision=prec, cg_graphs=args.cg_graphs, cycle_skip=v,
                                    tile_aspect=aspect, lds_stage=lds, divergence=div)
                 for v in (0, 1)]
        best, secs = bchar.tune_options(jobs, cands, streams, rounds=2)
        opts = cands[best]
        tuned = {"option": "cycle_skip", "values": [0, 1], "seconds": secs, "chosen": best,
                 "assembly": {"options": ["tile_aspect", "lds_stage"],
                              "values": [list(x) for x in shapes], "seconds": ksecs,
                              "chosen": [aspect, lds]},
                 "hash_scale": {"values": hscales, "seconds": hsecs,
                                "chosen": hscales[hb]}}
        log(f"tuned: cycle_skip {best} ({secs[0]:.3f} s against {secs[1]:.3f} s)")

    # ---- phase 1: one build after another; the build kernel (one launch a
    # step) timed with HIP events over the timed steps
    c, nxt = c0.clone(), torch.empty_like(c0)
    T = None
    lat = []
    seq_stats = []
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    for s in range(seq_total):
        if s == warmup:
            bchar.profile_kernel(args.build_kernel)
        tw = time.perf_counter()
        if T is None:
            T = bchar.Transfer.build(M, vels[s], w["dt"], opts)
        else:
            T.rebuild(vels[s], w["dt"], opts)
        c, nxt, e = apply(T, c, nxt)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - tw
        if s == warmup - 1 or (warmup == 0 and s == 0):
            ts0 = time.perf_counter()
        if s >= warmup:
            lat.append(dt_s)
            seq_stats.append(T.stats)
        log(f"sequential step {s}: {dt_s:.3f} s, ipm {T.stats['qp_ipm']}, cg {T.stats['qp_cg']}, "
            f"mass err {e:.2e}")
    seq_elapsed = time.perf_counter() - ts0
    b_launches, b_ms = bchar.profile_read()
    bchar.profile_kernel(args.trace_kernel)
    T.rebuild(vels[0], w["dt"], opts)
    torch.cuda.synchronize()
    t_launches, t_ms = bchar.profile_read()
    bchar.profile_kernel(None)

    # ---- phase 2: D transfers built at once (D = 1: the sequential run)
    if D > 1:
        c, nxt = c0.clone(), torch.empty_like(c0)
        Ts = [None] * D
        last = None
        stats = []
        k = pipe_first

        def batch(timed):
            nonlocal Ts, last, k, c, nxt
            jobs = [(Ts[j], M, vels[k + j], w["dt"], last) for j in range(D)]
            Ts = bchar.build_batch(jobs, opts, streams)
            for j in range(D):
                c, nxt, e = apply(Ts[j], c, nxt)
                if timed:
                    stats.append(Ts[j].stats)
            last = Ts[D - 1]
            k += D

        for _ in range(warm_batches):
            batch(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(timed_batches):
            batch(True)
            log(f"batch {b}: t = {time.perf_counter() - t0:.3f} s, cg "
                f"{[s_['qp_cg'] for s_ in stats[-D:]]}, mass err {mass_err:.2e}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    else:
        stats = seq_stats
        elapsed = seq_elapsed

    n_cells = M.n_cells
    value = n_cells * steps_timed / elapsed
    nnz = stats[-1]["nnz"]
    cg_mean = float(np.mean([s_["qp_cg"] for s_ in stats]))

    def roof(kernel, n_launch, total_ms, alg):
        if n_launch <= 0:
            return None
        avg_s = total_ms / 1e3 / n_launch
        achieved = alg / avg_s / 1e9
        traffic = measured_traffic(kernel, workload_key(workload, n, precision))
        return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "launches": n_launch, "avg_us": avg_s * 1e6,
                "algorithmic_bytes_per_launch": alg,
                "timing": "HIP events around each launch, sequential phase"}

    st = seq_stats[-1]
    roof_build = roof(args.build_kernel, b_launches, b_ms,
                      algorithmic_bytes(args.build_kernel, n_cells, st["nnz"], M.n_balls, st))
    roof_trace = roof(args.trace_kernel, t_launches, t_ms,
                      algorithmic_bytes(args.trace_kernel, n_cells, st["nnz"], M.n_balls, st))
    # the build stage a1-a4 (tracking and assembly) against its 385 bytes
    # per cell
    stage = None
    if roof_build and roof_trace:
        t_stage = (roof_build["avg_us"] + roof_trace["avg_us"]) * 1e-6
        ach = 385.0 * n_cells / t_stage / 1e9
        stage = {"bound": "hbm", "kernels": [args.trace_kernel, args.build_kernel],
                 "bytes_per_cell": 385, "seconds": t_stage, "achieved": ach,
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
    # the whole step (every stage, the least-change solve by its CG count)
    bpc = step_bytes_per_cell(cg_mean)
    ach_step = bpc * n_cells * steps_timed / elapsed / 1e9
    step_roof = {"bound": "hbm", "bytes_per_cell": bpc, "qp_cg_mean": cg_mean,
                 "bytes_per_step": bpc * n_cells, "achieved": ach_step, "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": ach_step / HBM_PEAK_GBS,
                 "timing": "host clock over the timed steps of the reported run"}
    lat_ms = np.array(lat) * 1e3
    return {
        "metric": metric,
        "value": value,
        "steps_timed": steps_timed,
        "ms_per_step": elapsed / steps_timed * 1e3,
        "dtype": "f64" if precision == "fp64" else "f32 geometry + f64 adjustment",
        "config": {"workload": desc, "n_cells": n_cells, "precision": precision, "nnz": nnz,
                   "inflight_builds": D, "cg_graphs": args.cg_graphs,
                   "cycle_skip": int(opts.cycle_skip), "tuned": tuned,
                   "trace_precision": int(st["trace_precision"]),
                   "qp_ipm_mean": float(np.mean([s_["qp_ipm"] for s_ in stats])),
                   "qp_cg_mean": cg_mean,
                   "qp_levels": sorted({s_["qp_level"] for s_ in stats}),
                   "device_bytes_per_transfer": int(st["device_bytes"])},
        "mass_ok": bool(mass_err <= 1e-12),
        "max_rel_mass_err": mass_err,
        "sequential": {"value": n_cells * steps / seq_elapsed,
                       "step_latency_ms_p50": float(np.percentile(lat_ms, 50)),
                       "step_latency_ms_p99": float(np.percentile(lat_ms, 99)),
                       "qp_cg_mean": float(np.mean([s_["qp_cg"] for s_ in seq_stats]))},
        "roofline": roof_build,
        "roofline_trace": roof_trace,
        "roofline_build_stage": stage,
        "roofline_step": step_roof,
    }


if __name__ == "__main__":
    main()
