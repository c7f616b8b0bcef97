"""Host logic of the benchmark's counter record (CPU only).

The roofline's HBM traffic comes from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
of the benchmark.  Each counter is scaled by what it reads for a device copy
of known size made in the same run, and the record is trusted only while
the kernel sources and the configuration match.  These tests feed
synthetic counter files in rocprofv3's CSV layout through that path.
"""
import csv
import json
import os
import re

import pytest

import bench

HEADER = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]
FORCE = "void nb6::regf_kernel<0, 1, 6>(nb6::RegfArgs, int)"


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEADER)
        for k, (name, value) in enumerate(rows):
            w.writerow([k, k, "Agent 1", 1, 1, 1, 256, 1, name, 256, 0, 0, 8, 0, 16,
                        counter, value, 100 * k, 100 * k + 50])


def _files(tmp_path, copy_kib_read, copy_kib_write, force_read, force_write):
    fetch, write, valu = (str(tmp_path / n) for n in ("fetch.csv", "write.csv", "valu.csv"))
    _write(fetch, "FETCH_SIZE", [("fill", 3.0), ("__amd_rocclr_copyBuffer", copy_kib_read)] +
           [(FORCE, v) for v in force_read] + [("__amd_rocclr_copyBuffer", 2.5)])
    _write(write, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", copy_kib_write)] +
           [(FORCE, v) for v in force_write])
    rows = []
    for c, v in zip(bench.VALU_COUNTERS, (350, 120, 70, 130, 10, 5, 4, 64)):
        rows += [(FORCE, v), ("fill", 1.0)]
    with open(valu, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEADER)
        for k, ((name, value), c) in enumerate(zip(rows, [c for c in bench.VALU_COUNTERS
                                                         for _ in range(2)])):
            w.writerow([k, k, "Agent 1", 1, 1, 1, 256, 1, name, 256, 0, 0, 8, 0, 16,
                        c, value, 0, 1])
    return fetch, write, valu


def _record(text):
    m = re.search(r"^counter-record: (\{.*\})$", text, re.M)
    assert m, text
    return json.loads(m.group(1))


def test_traffic_is_scaled_by_the_calibration_copy(tmp_path):
    # a 512 MiB copy read as 262144 KiB (factor 2) and written as 524288 KiB
    # (factor 1); three force launches each: the median is taken
    files = _files(tmp_path, 262144.0, 524288.0, [100.0, 140000.0, 150000.0],
                   [600000.0, 610000.0, 5.0])
    text = bench.counter_summary(*files, 512, "cfg", 1.0e10)
    rec = _record(text)
    assert rec["kernel"] == FORCE
    assert rec["read_bytes"] == 140000 * 1024 * 2
    assert rec["write_bytes"] == 600000 * 1024
    assert rec["config"] == "cfg"
    assert rec["source_sha256"] == bench.kernel_source_hash()
    # FP32 flop from the VALU counts: 64 lanes x (add + mul + 2 fma + trans)
    assert rec["fp32_flop"] == 64.0 * (120 + 70 + 2 * 130 + 10)
    assert "| FETCH_SIZE | 262144 | 2.0 |" in text


def test_missing_copy_or_force_dispatch_is_an_error(tmp_path):
    fetch, write, valu = _files(tmp_path, 262144.0, 524288.0, [1.0], [1.0])
    _write(fetch, "FETCH_SIZE", [(FORCE, 10.0)])  # no calibration copy
    with pytest.raises(SystemExit):
        bench.counter_summary(fetch, write, valu, 512, "cfg", 1.0)


def test_record_is_used_only_for_matching_sources_and_config(tmp_path, monkeypatch):
    files = _files(tmp_path, 262144.0, 524288.0, [1000.0], [2000.0])
    text = bench.counter_summary(*files, 512, "cfg A", 1.0e10)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "rec.md").write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "COUNTER_FILE", os.path.join("profiles", "rec.md"))
    real_hash = _record(text)["source_sha256"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: real_hash)
    assert bench.counters_from_profile("cfg A")["read_bytes"] == 1000 * 1024 * 2
    assert bench.counters_from_profile("cfg B") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.counters_from_profile("cfg A") is None


def test_committed_record_matches_the_sources():
    """The committed counter record belongs to the current kernel sources and
    the benchmark's default configuration, so the benchmark reports its
    traffic (skipped, with the reason, while the kernels have changed since
    the counters were taken: the benchmark then reports null)."""
    args = bench.argparse.Namespace(config=3, block="all", mode="local", cap=256, ipl=0,
                                    slices=0, lanes=0)
    rec = bench.counters_from_profile(bench.traffic_config(args))
    if rec is None:
        pytest.skip("the counter record predates the current kernel sources")
    assert rec["read_bytes"] > 0 and rec["write_bytes"] > 0
