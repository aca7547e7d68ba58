"""Host-side logic of bench.py (no device work): when a committed traffic
figure is attached to a bench line, and the counter summaries it is made
from."""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_source_digest_ignores_comments_and_layout(tmp_path, monkeypatch):
    src = tmp_path / "src"
    src.mkdir()
    (src / "device_util.hpp").write_text("int helper();\n")
    (src / "k.hip").write_text("// a kernel\n__global__ void k() { int a = 1; }\n")
    monkeypatch.setattr(bench, "SRC", str(src))
    monkeypatch.setitem(bench.KERNEL_SOURCES, "k_test", "k.hip")
    d0 = bench.source_digest("k_test")
    (src / "k.hip").write_text("/* the kernel,\n   reworded */\n__global__ void k() {\n"
                               "  int a = 1;  // one\n}\n")
    assert bench.source_digest("k_test") == d0
    (src / "k.hip").write_text("__global__ void k() { int a = 2; }\n")
    assert bench.source_digest("k_test") != d0
    (src / "k.hip").write_text("// a kernel\n__global__ void k() { int a = 1; }\n")
    (src / "device_util.hpp").write_text("int helper(int);\n")
    assert bench.source_digest("k_test") != d0


def test_traffic_attached_only_to_its_workload_and_code(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    key = bench.workload_key("swirl", 64, "fp64")
    rec = {"kernel": "k_assemble", "workload_key": key,
           "source_digest": bench.source_digest("k_assemble"), "bytes_per_launch": 123.0}
    (prof / "traffic_k_assemble.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("k_assemble", key) == 123.0
    # another precision, size or workload: not this figure
    assert bench.measured_traffic("k_assemble", bench.workload_key("swirl", 64, "fp32")) is None
    assert bench.measured_traffic("k_assemble", bench.workload_key("tets", 96, "fp32")) is None
    # code changed since the counters were taken
    rec["source_digest"] = "0" * 16
    (prof / "traffic_k_assemble.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("k_assemble", key) is None
    # no figure at all
    assert bench.measured_traffic("k_trace", key) is None
