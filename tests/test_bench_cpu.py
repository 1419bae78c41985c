"""Host logic of bench.py (no GPU): the one-GPU guard, the conversion of two
rocprofv3 --pmc counter files into HBM bytes per launch, and the hash that
voids a traffic record once the kernel sources change."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for k, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": k + 1, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""                  # no JSON line for a refused run


def test_traffic_from_counters_and_the_source_hash(tmp_path, monkeypatch):
    # a stand-in tree: the kernel's sources and the profiles folder
    (tmp_path / "profiles").mkdir()
    (tmp_path / "k.hip").write_text("kernel v1\n")
    (tmp_path / "k.h").write_text("header\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    spec = {"kernel": "step_kernel", "kernel_label": "step_kernel<4,2>", "sources": ["k.hip", "k.h"],
            "traffic": "t.json"}
    copy_mib = 64
    # FETCH_SIZE reads half the copy's bytes, WRITE_SIZE all of them; a table fill
    # and a smaller copy must not be taken for the calibration copy
    fetch_rows = [("__amd_rocclr_fillBufferAligned", 900000.0), ("__amd_rocclr_copyBuffer", 100.0),
                  ("void step_kernel<4, 2, false>(StepArgs)", 1000.0),
                  ("void step_kernel<4, 2, false>(StepArgs)", 3000.0),
                  ("void plan_kernel<4>(PlanArgs)", 50.0),
                  ("__amd_rocclr_copyBuffer", copy_mib * 1024.0 / 2)]
    write_rows = [("__amd_rocclr_fillBufferAligned", 900000.0), ("__amd_rocclr_copyBuffer", 10.0),
                  ("void step_kernel<4, 2, false>(StepArgs)", 500.0),
                  ("void step_kernel<4, 2, false>(StepArgs)", 700.0),
                  ("void plan_kernel<4>(PlanArgs)", 5.0),
                  ("__amd_rocclr_copyBuffer", copy_mib * 1024.0)]
    _write_counters(tmp_path / "fetch.csv", "FETCH_SIZE", fetch_rows)
    _write_counters(tmp_path / "write.csv", "WRITE_SIZE", write_rows)
    rec = bench.traffic_from_counters(str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv"), spec, copy_mib)
    assert rec["launches"] == 2
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == pytest.approx(600.0 * 1024)
    assert rec["bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0 + 600.0 * 1024)
    on_disk = json.load(open(tmp_path / "profiles" / "t.json"))
    assert on_disk == rec
    # the record counts while the sources are the measured ones ...
    assert bench.measured_traffic(spec) == pytest.approx(rec["bytes_per_launch"])
    # ... and not once any of them changes
    (tmp_path / "k.h").write_text("header, edited\n")
    assert bench.measured_traffic(spec) is None
    # a missing record is no traffic either
    assert bench.measured_traffic(dict(spec, traffic="absent.json")) is None


def test_every_workload_names_existing_sources():
    for name in bench.WORKLOADS:
        for prec, store in (("fp64", "bucketed"), ("fp64", "direct"), ("fp64", "hash"), ("fp32", "hash")):
            spec = bench.workload_spec(name, prec, store)
            for f in spec["sources"]:
                assert os.path.exists(os.path.join(ROOT, f)), (name, prec, f)
            assert len(bench.kernel_source_hash(spec)) == 64
