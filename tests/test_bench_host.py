"""Host-side logic of the benchmark: the HBM-traffic record (counter
summary keyed to the kernel source) and the GPU-count contract.  No GPU."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_counter_summary_scales_by_the_calibration_copies(tmp_path, monkeypatch):
    """Two counter runs: the roofline kernel's FETCH_SIZE / WRITE_SIZE are
    averaged over its dispatches and scaled by what the counters read for the
    1 GiB copies (here FETCH_SIZE reads half of the copy, WRITE_SIZE all of
    it, as on the MI355X): (1000 x 2 + 500 x 1) KiB per launch."""
    kern = bench.ROOF_KERNEL["mixed"] + ", false, true>(...)"
    half = bench.COPY_KIB // 2
    fetch = [(1, kern, "FETCH_SIZE", 900.0), (2, kern, "FETCH_SIZE", 1100.0),
             (3, "__amd_rocclr_copyBuffer", "FETCH_SIZE", half),
             (4, "other_kernel", "FETCH_SIZE", 7.0)]
    write = [(1, kern, "WRITE_SIZE", 500.0), (2, kern, "WRITE_SIZE", 500.0),
             (3, "__amd_rocclr_copyBuffer", "WRITE_SIZE", bench.COPY_KIB),
             (5, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 3.0)]   # a small copy: not a calibration
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", write)
    out = str(tmp_path / "rec.md")
    bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), "medium", "mixed", out)
    monkeypatch.setattr(bench, "traffic_path", lambda w, p: out)
    assert bench.recorded_traffic("medium", "mixed") == pytest.approx((1000 * 2 + 500 * 1) * 1024)


def test_traffic_record_is_dropped_when_the_kernel_source_changes(tmp_path, monkeypatch):
    rec = tmp_path / "rec.md"
    rec.write_text(f"source_sha256: {bench._kernel_sha()}\nbytes_per_launch: 123\n")
    monkeypatch.setattr(bench, "traffic_path", lambda w, p: str(rec))
    assert bench.recorded_traffic("medium", "mixed") == 123.0
    rec.write_text("source_sha256: " + "0" * 64 + "\nbytes_per_launch: 123\n")
    assert bench.recorded_traffic("medium", "mixed") is None
    monkeypatch.setattr(bench, "traffic_path", lambda w, p: str(tmp_path / "absent.md"))
    assert bench.recorded_traffic("medium", "mixed") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
