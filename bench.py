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
        # two launches per build, a counting pass and a filling pass, both
        # reading the tracked centre and radius (32 per ball), the residing
        # balls through the hash (32 per ball) and phi (8 per cell); the
        # filling pass writes the CSR entries (12 each): per launch, the
        # inputs and half the output
        return n_balls * (32 + 32) + n_cells * 8 + nnz * 12 // 2
    if kernel == "k_trace":
        # centre in, tracked centre and radius out, velocity lattice (24 B
        # per node, about one node per cell)
        return n_balls * (24 + 32) + n_cells * 24
    raise KeyError(kernel)


# the sources each measured kernel's device code comes from (its file and
# the header of device helpers; the other headers declare host code only)
KERNEL_SOURCES = {"k_smooth": "qp.hip", "k_zsmooth": "qp.hip", "k_fused_cycle": "qp.hip",
                  "k_assemble": "build.hip"}


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


def workload_key(workload, n, precision, cycle_skip):
    """The configuration a traffic figure belongs to: workload, size,
    precision and multigrid cycle (the cycle changes the launched levels)."""
    return f"{workload}-{n}-{precision}-skip{int(cycle_skip)}"


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


TRAFFIC_KERNELS = ("k_smooth", "k_fused_cycle", "k_zsmooth", "k_assemble")


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

    if workload == "tets":
        w = inputs.jittered_tets(sample_n, steps=1)
        layout, prec, what = "equal_measure", "fp32", "jittered tetrahedra"
        n_cells = 6 * sample_n ** 3
    else:
        w = inputs.swirl_hex(sample_n)
        layout, prec, what = "subcell", "fp64", "hexahedra, 8 balls per cell"
        n_cells = sample_n ** 3
    with threadpool_limits(1):
        t0 = time.perf_counter()
        T = otr.build_transfer(w["mesh"], w["vel_fn"](0), w["dt"], layout=layout,
                               precision=prec)
        c1 = otr.apply(T["row_ptr"], T["col"], T["A"], T["b"], w["c0"])
        t1 = time.perf_counter()
    assert np.all(np.isfinite(c1))
    return {"value": n_cells / (t1 - t0), "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"one step (build + apply) of the {workload} workload on a "
                      f"{sample_n}^3 grid ({n_cells} cells, {what}, {prec.upper()}), "
                      f"{t1 - t0:.2f} s single-threaded"}


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
        halvings = 0
        per_call = 64 if depth > 1 else 1
        for b0 in range(0, len(probs), per_call):
            chunk = probs[b0:b0 + per_call]
            Ts = bchar.build_batch([(None, q["M"], q["U"], q["dt"]) for q in chunk], opts, streams)
            for q, T in zip(chunk, Ts):
                cg.append(T.stats["qp_cg"])
                halvings += T.stats["dt_halvings"]
                finish(q, T)
            if depth > 1 or b0 % 16 == 15:
                log(f"  depth {depth}: problems up to {min(b0 + per_call, len(probs)) - 1} done "
                    f"at {time.perf_counter() - t0:.2f} s")
        torch.cuda.synchronize()
        return time.perf_counter() - t0, cg, halvings

    run(D)   # warm-up pass (code objects, allocator)
    t_seq, cg_seq, _ = run(1)
    log(f"mixed, one at a time: {t_seq:.3f} s")
    t_par, cg_par, halvings = run(D)
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
                   "qp_cg_mean": float(np.mean(cg_par))},
        "mass_ok": bool(mass_err <= 1e-12),
        "max_rel_mass_err": mass_err,
        "sequential": {"value": cells * steps / t_seq, "seconds": t_seq},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def bench_serve(args):
    """Requests arriving as a Poisson process (seeded) at ``--rate`` per
    second: each takes a problem from a pool of ``--problems`` resident
    meshes (inputs.mixed_problem), builds its transfer and applies it a
    number of times drawn from U{1..50}; the server (bchar_server_*) runs
    them with ``--inflight`` workers, then with one (the serial path) on the
    same arrivals.  Reports cell-updates/s and the latency from arrival to
    result (p50, p99)."""
    import threading

    import numpy as np
    import torch

    from paper_1908_05834_amd import bchar, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    D = max(1, args.inflight)
    pool = []
    for p in range(args.problems):
        q = inputs.mixed_problem(p)
        M = bchar.Mesh(q["mesh"], q["layout"])
        c0 = torch.as_tensor(q["c0"], device="cuda")
        pool.append({"M": M, "U": bchar.VelocityLattice(q["vel"]), "dt": q["dt"], "c0": c0,
                     "m0": M.mass(c0), "name": q["name"]})
    rng = np.random.default_rng(args.seed)
    gaps = rng.exponential(1.0 / args.rate, size=args.requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    which = rng.integers(0, len(pool), size=args.requests)
    nsteps = rng.integers(1, 51, size=args.requests)

    def run(workers, label):
        srv = bchar.Server(workers, mem_budget=int(args.mem_budget_gib * (1 << 30)))
        # warm-up: every pool problem once (worker buffers reach their size)
        for q in pool:
            out, tmp = torch.empty_like(q["c0"]), torch.empty_like(q["c0"])
            srv.wait(srv.submit(q["M"], q["U"], q["dt"], 1, q["c0"], out, tmp))
        results = [None] * args.requests
        tickets = [None] * args.requests
        bufs = [None] * args.requests
        ready = threading.Semaphore(0)

        def collect():
            for i in range(args.requests):
                ready.acquire()
                results[i] = srv.wait(tickets[i])
                q = pool[which[i]]
                m = q["M"].mass(bufs[i][0])
                results[i]["mass_err"] = abs(m - q["m0"]) / abs(q["m0"])
                bufs[i] = None
        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for i in range(args.requests):
            dly = t0 + arrivals[i] - time.perf_counter()
            if dly > 0:
                time.sleep(dly)
            q = pool[which[i]]
            out, tmp = torch.empty_like(q["c0"]), torch.empty_like(q["c0"])
            bufs[i] = (out, tmp)
            tickets[i] = srv.submit(q["M"], q["U"], q["dt"], int(nsteps[i]), q["c0"], out, tmp)
            ready.release()
            if i % 25 == 24:
                log(f"  {label}: {i + 1} requests submitted at {time.perf_counter() - t0:.1f} s")
        th.join()
        srv.close()
        ok = all(r["status"] == bchar.OK for r in results)
        lat = np.array([r["t_done"] - r["t_submit"] for r in results])
        span = max(r["t_done"] for r in results) - min(r["t_submit"] for r in results)
        cu = sum(pool[which[i]]["M"].n_cells * int(nsteps[i]) for i in range(args.requests))
        merr = max(r["mass_err"] for r in results)
        log(f"{label}: {span:.2f} s, p50 {np.percentile(lat, 50) * 1e3:.0f} ms, "
            f"p99 {np.percentile(lat, 99) * 1e3:.0f} ms")
        return {"value": cu / span, "seconds": span, "ok": ok, "mass_err": merr,
                "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
                "latency_ms_p99": float(np.percentile(lat, 99) * 1e3)}

    par = run(D, f"{D} workers")
    ser = run(1, "1 worker")
    out = {
        "metric": "B-char served cell-updates/s and p99 latency (arrival to result)",
        "value": par["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": len(pool),
        "ms_per_step": par["seconds"] / args.requests * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.requests} requests, Poisson arrivals at {args.rate}/s "
                               f"(seed {args.seed}), problems drawn from {len(pool)} resident "
                               "meshes of the batch of independent problems, U{1..50} "
                               "updates each",
                   "workers": D, "mem_budget_gib": args.mem_budget_gib,
                   "latency_ms_p50": par["latency_ms_p50"],
                   "latency_ms_p99": par["latency_ms_p99"]},
        "mass_ok": bool(par["ok"] and ser["ok"] and max(par["mass_err"], ser["mass_err"]) <= 1e-12),
        "max_rel_mass_err": max(par["mass_err"], ser["mass_err"]),
        "serial": ser,
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
    ap.add_argument("--roofline-kernel", default="k_smooth")
    ap.add_argument("--build-kernel", default="k_assemble")
    ap.add_argument("--smoother-kernel", default="k_zsmooth")
    ap.add_argument("--coarse-kernel", default="k_fused_cycle")
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
    ap.add_argument("--workload", choices=["swirl", "tets", "mixed", "serve"], default="swirl")
    ap.add_argument("--rate", type=float, default=4.0, help="serve: arrivals per second")
    ap.add_argument("--requests", type=int, default=120, help="serve: number of requests")
    ap.add_argument("--seed", type=int, default=0, help="serve: arrival seed")
    ap.add_argument("--mem-budget-gib", type=float, default=64.0,
                    help="serve: device memory the requests in progress may take")
    ap.add_argument("--problems", type=int, default=32,
                    help="mixed workload: number of problems (seeds 0 .. problems-1)")
    ap.add_argument("--pmc-sum", nargs=3, metavar=("PROF_DIR", "COUNTER", "OUT"),
                    help="only summarise a rocprofv3 --pmc run (no device work)")
    ap.add_argument("--traffic-json", nargs=5,
                    metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE", "COPY_MIB"),
                    help="only write profiles/traffic_<kernel>.json from four summaries")
    ap.add_argument("--traffic-cycle-skip", type=int, choices=[0, 1], default=0,
                    help="with --traffic-json: the cycle the counter runs used")
    args = ap.parse_args()

    if args.pmc_sum:
        pmc_summary(*args.pmc_sum)
        return
    if args.traffic_json:
        fe, wr, cfe, cwr, mib = args.traffic_json
        cmd = "rocprofv3 --pmc {c} --output-format csv -d /tmp/pmc_{t} -o p -- python3 bench.py {a}"
        sk = args.traffic_cycle_skip
        run = f"--steps 1 --warmup 1 --inflight 1 --no-cpu-baseline --tune 0 --cycle-skip {sk}"
        write_traffic(fe, wr, cfe, cwr, int(mib),
                      [cmd.format(c="FETCH_SIZE", t="f", a=run),
                       cmd.format(c="WRITE_SIZE", t="w", a=run),
                       cmd.format(c="FETCH_SIZE", t="cf", a=f"--copy-calibration {mib}"),
                       cmd.format(c="WRITE_SIZE", t="cw", a=f"--copy-calibration {mib}")],
                      "3D swirl, 64^3 hexahedra, 8 balls per cell, FP64"
                      + (", cycle visiting every other level" if sk else ""),
                      workload_key("swirl", 64, "fp64", sk))
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

    import numpy as np
    import torch

    from paper_1908_05834_amd import bchar, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.workload == "tets":
        args.n = args.n or 96
        args.precision = args.precision or "fp32"
        w = inputs.jittered_tets(args.n, steps=max(args.warmup + args.steps, 3))
        layout = "equal_measure"
        workload = (f"3D jittered Kuhn tetrahedra, {args.n}^3 cubes x 6 = {6 * args.n ** 3} "
                    f"cells, lognormal phi, swirl at CFL 4, one centroid ball per cell, "
                    f"dt = 1/128, transfer rebuilt every step")
        metric = (f"B-char cell-updates/s (3D tets {6 * args.n ** 3}) at 1e-12 mass err; "
                  "served p99 latency")
    else:
        args.n = args.n or 64
        args.precision = args.precision or "fp64"
        w = inputs.swirl_hex(args.n)
        layout = "subcell"
        workload = (f"3D swirl, unit cube, {args.n}^3 hexahedra, 8 balls per cell, "
                    f"phi = 1, dt = 1/128, transfer rebuilt every step")
        metric = "B-char cell-updates/s (3D hex 64^3) at 1e-12 mass err; served p99 latency"
    # binary32 tracking (FP32_VOLUME) needs a constant porosity; the porous
    # unstructured workload tracks in binary64 with binary32 lenses
    prec = bchar.FP64 if args.precision == "fp64" else (
        bchar.FP32_LENS if args.workload == "tets" else bchar.FP32_VOLUME)
    opts = bchar.opts_default(precision=prec, cg_graphs=args.cg_graphs,
                              cycle_skip=args.cycle_skip)
    M = bchar.Mesh(w["mesh"], layout)
    # phase 1: one build after another (per-step latency); phase 2: D builds
    # at once (throughput, the reported value).  Every interval's velocity
    # lattice is resident on the device before timing.
    # Both runs time the same intervals (warmup .. warmup + steps - 1) when
    # the warm-up spans whole batches.
    seq_total = args.warmup + args.steps
    warm_batches = max(1, math.ceil(args.warmup / D))
    timed_batches = max(1, math.ceil(args.steps / D))
    steps_timed = timed_batches * D if D > 1 else args.steps
    pipe_first = max(0, args.warmup - warm_batches * D)
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

    # ---- autotuning (untimed): which multigrid cycle builds D transfers in
    # flight fastest on this workload, measured by the library on the first
    # intervals (bchar_tune_options), unless --tune 0 fixes it
    # one stream per build in flight, created once: the tuning and the
    # in-flight phase share them (more streams than hardware queues would
    # put two builds on one queue)
    streams = [torch.cuda.Stream() for _ in range(D)]
    tuned = None
    if args.tune:
        cands = [bchar.opts_default(precision=prec, cg_graphs=args.cg_graphs, cycle_skip=v)
                 for v in (0, 1)]
        best, secs = bchar.tune_options([(M, vels[j % len(vels)], w["dt"]) for j in range(D)],
                                        cands, streams, rounds=2)
        opts = cands[best]
        tuned = {"option": "cycle_skip", "values": [0, 1], "seconds": secs, "chosen": best}
        log(f"tuned: cycle_skip {best} ({secs[0]:.3f} s against {secs[1]:.3f} s)")

    # ---- phase 1: sequential
    c, nxt = c0.clone(), torch.empty_like(c0)
    T = None
    lat = []
    seq_stats = []
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    for s in range(seq_total):
        tw = time.perf_counter()
        if T is None:
            T = bchar.Transfer.build(M, vels[s], w["dt"], opts)
        else:
            T.rebuild(vels[s], w["dt"], opts)
        c, nxt, e = apply(T, c, nxt)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - tw
        if s == args.warmup - 1 or (args.warmup == 0 and s == 0):
            ts0 = time.perf_counter()
        if s >= args.warmup:
            lat.append(dt_s)
            seq_stats.append(T.stats)
        log(f"sequential step {s}: {dt_s:.3f} s, ipm {T.stats['qp_ipm']}, cg {T.stats['qp_cg']}, "
            f"mass err {e:.2e}")
    seq_elapsed = time.perf_counter() - ts0

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
        # every 17th launch: the events barely disturb the run, and as 17 is
        # prime the sample runs through the levels of a cycle (unless a cycle
        # launches the kernel a multiple of 17 times)
        bchar.profile_kernel_sampled(args.roofline_kernel, 17)
        t0 = time.perf_counter()
        for b in range(timed_batches):
            batch(True)
            log(f"batch {b}: t = {time.perf_counter() - t0:.3f} s, cg "
                f"{[s_['qp_cg'] for s_ in stats[-D:]]}, mass err {mass_err:.2e}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        launches, kms = bchar.profile_read()
        bchar.profile_kernel(None)
        T_last = Ts[0]
    else:
        # the sequential run is the timed one; time the roofline kernel over
        # one more pass of the same steps
        stats = seq_stats
        elapsed = seq_elapsed
        bchar.profile_kernel(args.roofline_kernel)
        for s in range(args.warmup, seq_total):
            T.rebuild(vels[s], w["dt"], opts)
        torch.cuda.synchronize()
        launches, kms = bchar.profile_read()
        bchar.profile_kernel(None)
        T_last = T
    # the build kernel and the fine-level smoother, timed the same way over
    # one more (untimed) build each
    bchar.profile_kernel(args.build_kernel)
    T_last.rebuild(vels[0], w["dt"], opts)
    torch.cuda.synchronize()
    b_launches, b_kms = bchar.profile_read()
    bchar.profile_kernel(args.smoother_kernel)
    T_last.rebuild(vels[1], w["dt"], opts)
    torch.cuda.synchronize()
    z_launches, z_kms = bchar.profile_read()
    z_stats = T_last.stats
    bchar.profile_kernel(args.coarse_kernel)
    T_last.rebuild(vels[2], w["dt"], opts)
    torch.cuda.synchronize()
    c_launches, c_kms = bchar.profile_read()
    bchar.profile_kernel(None)

    n_cells = M.n_cells
    value = n_cells * steps_timed / elapsed
    nnz = stats[-1]["nnz"]

    def roofline(kernel, n_launch, total_ms, st):
        if n_launch <= 0:
            return None
        avg_s = total_ms / 1e3 / n_launch
        alg = algorithmic_bytes(kernel, n_cells, st["nnz"], M.n_balls, st)
        achieved = alg / avg_s / 1e9
        traffic = measured_traffic(kernel, workload_key(args.workload, args.n, args.precision,
                                                        opts.cycle_skip))
        return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "launches": n_launch, "avg_us": avg_s * 1e6,
                "algorithmic_bytes_per_launch": alg}

    roof = roofline(args.roofline_kernel, launches, kms, stats[-1])
    roof_build = roofline(args.build_kernel, b_launches, b_kms, T_last.stats)
    roof_smoother = roofline(args.smoother_kernel, z_launches, z_kms, z_stats)
    roof_coarse = roofline(args.coarse_kernel, c_launches, c_kms, T_last.stats)
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": metric,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps_timed,
        "warmup": args.warmup,
        "ms_per_step": elapsed / steps_timed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 geometry + f64 adjustment",
        "data": "synthetic",
        "config": {"workload": workload,
                   "n_cells": n_cells, "precision": args.precision, "nnz": nnz,
                   "inflight_builds": D, "cg_graphs": args.cg_graphs,
                   "cycle_skip": int(opts.cycle_skip), "tuned": tuned,
                   "qp_ipm_mean": float(np.mean([s_["qp_ipm"] for s_ in stats])),
                   "qp_cg_mean": float(np.mean([s_["qp_cg"] for s_ in stats])),
                   "qp_levels": sorted({s_["qp_level"] for s_ in stats})},
        "mass_ok": bool(mass_err <= 1e-12),
        "max_rel_mass_err": mass_err,
        "sequential": {"value": n_cells * args.steps / seq_elapsed,
                       "step_latency_ms_p50": float(np.percentile(lat_ms, 50)),
                       "step_latency_ms_p99": float(np.percentile(lat_ms, 99)),
                       "qp_cg_mean": float(np.mean([s_["qp_cg"] for s_ in seq_stats]))},
        "roofline": roof,
        "roofline_build": roof_build,
        "roofline_smoother": roof_smoother,
        "roofline_coarse": roof_coarse,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the oracle's cost grows faster than linearly on tetrahedra: a
        # 6^3-cube sample (1,296 cells) keeps it to seconds
        out["cpu_baseline"] = cpu_baseline(
            args.cpu_sample if args.workload == "swirl" else 6, args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
