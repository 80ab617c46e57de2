"""Host logic of bench.py that needs no GPU: the one-GPU guard, the
copy-calibrated traffic summary written from the two rocprofv3 counter runs,
and the staleness check that drops stored counter figures once the kernel
sources change."""

import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, grid, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter, "Counter_Value": value})


def _rows(copy_kib, dominant_kib):
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::BinaryFunctor<Mul> >(int)"
    small_copy = (copy, 1024, 1.0)  # a smaller launch of the same kernel: not the calibration
    dom = "void semcond::%s(semcond::ApplyArgs<float>, long)" % bench.DOMINANT
    other = ("void semcond::k_cg_step<float, true, false, 1>(float*)", 4096, 5.0e6)
    return [small_copy, (copy, 1 << 20, copy_kib), other] + [(dom, 221184, v) for v in dominant_kib]


def test_traffic_summary_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.md"))
    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    # the calibration copy moves COPY_BYTES each way; FETCH reads half of it
    # (factor 2), WRITE all of it (factor 1).  Dominant launches: two full ones
    # and one that left at once (below a tenth of the median: excluded).
    copy_kib = bench.COPY_BYTES / 1024.0
    _counter_csv(fetch, "FETCH_SIZE", _rows(copy_kib / 2, [1000.0, 1200.0, 3.0]))
    _counter_csv(write, "WRITE_SIZE", _rows(copy_kib, [500.0, 700.0, 1.0]))
    bench.pmc_summary(str(fetch), str(write), ["rocprofv3 --pmc FETCH_SIZE -- python3 bench.py --pmc-workload"])
    text = open(bench.TRAFFIC_FILE).read()
    assert "rocprofv3 --pmc FETCH_SIZE" in text
    assert "(2 of 3 dispatches)" in text
    expect = 1100.0 * 1024 * 2.0 + 600.0 * 1024 * 1.0
    assert bench.stored_traffic() == pytest.approx(expect, rel=1e-12)
    assert "kernel_sources_sha256: %s" % bench.kernel_sources_hash() in text


def test_stored_figures_are_dropped_for_other_kernel_sources(tmp_path, monkeypatch):
    traffic, counters = tmp_path / "traffic.md", tmp_path / "counters.md"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(counters))
    assert bench.stored_traffic() is None and bench.stored_valu_busy() is None  # absent
    h = bench.kernel_sources_hash()
    traffic.write_text("traffic_bytes_per_launch: 123\nkernel_sources_sha256: %s\n" % h)
    counters.write_text("valu_busy: 0.5\nkernel_sources_sha256: %s\n" % h)
    assert bench.stored_traffic() == 123.0 and bench.stored_valu_busy() == 0.5
    other = "0" * 16 if h != "0" * 16 else "1" * 16
    traffic.write_text("traffic_bytes_per_launch: 123\nkernel_sources_sha256: %s\n" % other)
    counters.write_text("valu_busy: 0.5\nkernel_sources_sha256: %s\n" % other)
    assert bench.stored_traffic() is None and bench.stored_valu_busy() is None


def test_committed_summaries_match_the_current_kernel_sources():
    """The traffic and counter figures the bench line reports come from the
    kernel sources in the tree (re-measure after changing them)."""
    assert bench.stored_traffic() is not None
    assert bench.stored_valu_busy() is not None
