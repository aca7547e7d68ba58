"""CPU-side checks of the C ABI: the library loads and exports every entry
point declared in include/bchar.h (no device work is done here)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bchar.h")
LIB = os.path.join(ROOT, "paper_1908_05834_amd", "libbchar.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(bchar_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for core in ("bchar_mesh_create", "bchar_build_transfer", "bchar_step", "bchar_mass"):
        assert core in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_1908_05834_amd import bchar
    assert sorted(bchar.EXPORTED) == declared()


def test_status_strings_and_defaults_without_device():
    from paper_1908_05834_amd import bchar
    assert bchar.status_string(bchar.E_VOID_ROW) == "void row"
    o = bchar.opts_default()
    assert o.n_sweeps == 10 and o.qp_tol == 1e-13 and o.precision == bchar.FP64


def test_batch_build_rejects_bad_arguments_without_device():
    import ctypes as C

    from paper_1908_05834_amd import bchar
    o = bchar.opts_default()
    streams = (C.c_void_p * 1)(None)
    jobs = (bchar.BuildJob * 2)()
    # NULL job array, no streams, a job with neither transfer nor mesh, one
    # transfer in two jobs: all refused before any device work
    assert bchar._build_batch(None, 1, C.byref(o), streams, 1) == bchar.E_INVALID_ARG
    assert bchar._build_batch(jobs, 1, C.byref(o), streams, 0) == bchar.E_INVALID_ARG
    assert bchar._build_batch(jobs, 1, C.byref(o), streams, 1) == bchar.E_INVALID_ARG
    jobs[0].transfer = jobs[1].transfer = 0x1000
    assert bchar._build_batch(jobs, 2, C.byref(o), streams, 1) == bchar.E_INVALID_ARG
    assert b"two jobs" in bchar._last_error()


def test_server_rejects_bad_arguments_without_device():
    import ctypes as C

    from paper_1908_05834_amd import bchar
    h = C.c_void_p()
    streams = (C.c_void_p * 1)(None)
    # no streams, no workers, negative budget: refused before any device work
    assert bchar._server_create(1, None, 0, None, C.byref(h)) == bchar.E_INVALID_ARG
    assert bchar._server_create(0, streams, 0, None, C.byref(h)) == bchar.E_INVALID_ARG
    assert bchar._server_create(1, streams, -1, None, C.byref(h)) == bchar.E_INVALID_ARG
    t = C.c_int64()
    assert bchar._server_submit(None, None, C.byref(t)) == bchar.E_INVALID_ARG
    assert bchar._server_destroy(None) == bchar.OK


def _struct_fields(name):
    """Member names of `typedef struct { ... } name;` in the header, in order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"typedef struct\s*\{((?:(?!typedef).)*?)\}\s*" + name + r"\s*;", text,
                  flags=re.S)
    assert m, name
    out = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if decl:
            # every declarator of the line: `double a, b, c`, `int64_t n[3]`
            out.extend(re.findall(r"(\w+)\s*(?:\[[^\]]*\])?\s*(?:,|$)", decl))
    return out


def test_binding_structs_mirror_the_header():
    from paper_1908_05834_amd import bchar
    pairs = [("bchar_mesh_desc", bchar.MeshDesc), ("bchar_velocity", bchar.Velocity),
             ("bchar_opts", bchar.Opts), ("bchar_stats", bchar.Stats),
             ("bchar_build_job", bchar.BuildJob), ("bchar_request", bchar.Request),
             ("bchar_request_result", bchar.RequestResult)]
    for cname, py in pairs:
        assert [f for f, _ in py._fields_] == _struct_fields(cname), cname


def test_option_defaults_of_the_solver():
    from paper_1908_05834_amd import bchar
    o = bchar.opts_default()
    # CG iterations replayed from graphs, every multigrid level visited,
    # voids reported rather than remedied
    assert o.cg_graphs == 1 and o.cycle_skip == 0 and o.max_halvings == 0
    assert o.warm_start == 1 and o.qp_max_cg == 400


def test_binding_struct_offsets_match_the_c_compiler(tmp_path):
    """sizeof and every member offset of the ctypes mirrors against what gcc
    lays out for the header's structs."""
    import shutil
    import subprocess

    import pytest

    from paper_1908_05834_amd import bchar
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = [("bchar_mesh_desc", bchar.MeshDesc), ("bchar_velocity", bchar.Velocity),
             ("bchar_opts", bchar.Opts), ("bchar_stats", bchar.Stats),
             ("bchar_build_job", bchar.BuildJob), ("bchar_request", bchar.Request),
             ("bchar_request_result", bchar.RequestResult)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bchar.h"', "int main(void) {"]
    for cname, _ in pairs:
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f in _struct_fields(cname):
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for cname, py in pairs:
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_tuner_rejects_bad_arguments_without_device():
    import ctypes as C

    from paper_1908_05834_amd import bchar
    cands = (bchar.Opts * 2)(bchar.opts_default(), bchar.opts_default(cycle_skip=1))
    streams = (C.c_void_p * 1)(None)
    jobs = (bchar.BuildJob * 1)()
    best = C.c_int(-1)
    secs = (C.c_double * 2)()
    # NULL jobs, no candidates, zero rounds, a job without a mesh, a job
    # naming a transfer, an invalid candidate: refused before device work
    assert bchar._tune_options(None, 1, cands, 2, 1, streams, 1, C.byref(best), secs) == \
        bchar.E_INVALID_ARG
    jobs[0].mesh = 0x1000
    jobs[0].u = C.cast(C.c_void_p(0x2000), C.POINTER(bchar.Velocity))
    assert bchar._tune_options(jobs, 1, cands, 0, 1, streams, 1, C.byref(best), secs) == \
        bchar.E_INVALID_ARG
    assert bchar._tune_options(jobs, 1, cands, 2, 0, streams, 1, C.byref(best), secs) == \
        bchar.E_INVALID_ARG
    jobs[0].mesh = None
    assert bchar._tune_options(jobs, 1, cands, 2, 1, streams, 1, C.byref(best), secs) == \
        bchar.E_INVALID_ARG
    jobs[0].mesh = 0x1000
    jobs[0].transfer = 0x3000
    assert bchar._tune_options(jobs, 1, cands, 2, 1, streams, 1, C.byref(best), secs) == \
        bchar.E_INVALID_ARG
    jobs[0].transfer = None
    bad = (bchar.Opts * 1)(bchar.opts_default(n_sweeps=-1))
    assert bchar._tune_options(jobs, 1, bad, 1, 1, streams, 1, C.byref(best), secs) == \
        bchar.E_INVALID_ARG
    assert best.value == -1
