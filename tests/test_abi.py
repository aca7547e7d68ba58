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
