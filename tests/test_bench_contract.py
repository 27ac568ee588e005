"""Host-side parts of the measurement contract of bench.py (no GPU).

The roofline's `traffic` comes from the committed counter summaries and must be
reported only for the kernel sources and run mode they were taken on; a run on
more than one GPU is refused with a message, as this build measures one GPU.
"""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _records():
    with open(os.path.join(ROOT, "profiles", "traffic_combined-p4-1024.json")) as fh:
        return json.load(fh)["records"]


def test_traffic_records_name_their_run():
    # each record names the kernel, the run mode, the calibration and the sources it was taken on
    recs = _records()
    kinds = {(r["kernel"], r["precision"], r["precond"], bool(r.get("matrix_free"))) for r in recs}
    assert ("factor", "bf16", "learned-fp8", False) in kinds
    for r in recs:
        assert len(r["kernel_source_hash"]) == 16 and r["bytes_per_launch"] > 0
        assert r["fetch_scale"] > 0 and r["write_scale"] > 0 and r["source"].startswith("profiles/")


def test_traffic_lookup_follows_the_run_mode():
    if not any(r["kernel_source_hash"] == bench.kernel_source_hash() for r in _records()):
        pytest.skip("the kernel sources changed since the counters were taken (traffic is null)")
    got = bench.measured_traffic("combined-p4-1024", "factor", "bf16", "learned-fp8")
    assert got is not None and 4.0e9 < got < 7.0e9   # bytes per preconditioner apply
    # another kernel, precision, preconditioner or mode has no record: null, not a guess
    assert bench.measured_traffic("combined-p4-1024", "factor", "fp32", "learned-fp8") is None
    assert bench.measured_traffic("combined-p4-1024", "div", "bf16", "bj") is None
    assert bench.measured_traffic("combined-p4-1024", "div", "fp64", "bj", matrix_free=True) is None
    assert bench.measured_traffic("mixed-p4-512", "factor", "bf16", "learned-fp8") is None


def test_traffic_is_null_once_the_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.measured_traffic("combined-p4-1024", "factor", "bf16", "learned-fp8") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "gpus 1" in r.stderr
    assert r.stdout.strip() == ""
