"""Measurement tooling on the CPU: the counter summary's arithmetic, its link to
the kernel source, and the bench's roofline arithmetic."""
import csv
import os

import pytest

import bench
from paper_1711_05075_amd import rocprof_summary as rs


def _counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], r)))


def test_traffic_summary_scales_counters_by_the_copy_calibration(tmp_path):
    k = "void corr::k_spread_fftx<256>(int const*)"
    # two dispatches, each counter split over two rows (summed per dispatch), and
    # a kernel the regex must not pick up
    _counters(tmp_path / "f.csv", [(1, k, "FETCH_SIZE", 100), (1, k, "FETCH_SIZE", 20), (2, k, "FETCH_SIZE", 80),
                                   (2, k, "FETCH_SIZE", 40), (3, "other", "FETCH_SIZE", 1e9)])
    _counters(tmp_path / "w.csv", [(1, k, "WRITE_SIZE", 1000), (2, k, "WRITE_SIZE", 3000)])
    _counters(tmp_path / "cf.csv", [(7, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512)])
    _counters(tmp_path / "cw.csv", [(7, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024)])
    out = tmp_path / "t.txt"
    rs.traffic("k_spread_fftx", tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "cf.csv", tmp_path / "cw.csv",
               1 << 20, out, "cmd a;;cmd b")
    fields = dict(l.split(": ", 1) for l in out.read_text().splitlines() if ": " in l and not l.startswith("#"))
    # copy of 1 MiB: FETCH reads 512 KiB (scale 2), WRITE 1024 KiB (scale 1);
    # the kernel's means are 120 KiB fetched and 2000 KiB written per dispatch
    assert float(fields["fetch_scale"]) == pytest.approx(2.0)
    assert float(fields["write_scale"]) == pytest.approx(1.0)
    assert int(fields["dispatches_fetch"]) == 2
    assert float(fields["hbm_bytes_per_launch"]) == pytest.approx(2 * 120 * 1024 + 2000 * 1024)
    assert fields["kernel_source_sha256"] == rs.kernel_source_digest()
    assert "#   cmd a" in out.read_text() and "#   cmd b" in out.read_text()


def test_bench_reads_traffic_only_for_the_current_kernel_source():
    text = open(bench.TRAFFIC_SUMMARY).read()
    fields = dict(l.split(":", 1) for l in text.splitlines() if ":" in l and not l.startswith("#"))
    got = bench.measured_traffic()
    if fields["kernel_source_sha256"].strip() == rs.kernel_source_digest():
        assert got == pytest.approx(float(fields["hbm_bytes_per_launch"]))
    else:
        assert got is None
    # the digest stops before the kernels that follow the spreading kernel
    src = open(rs.KERNEL_SOURCE).read()
    cut = src.index("// Index of kept output mode")
    assert rs.kernel_source_digest(src[:cut] + src[cut:] + "\n// later kernel\n") == rs.kernel_source_digest(src)
    assert rs.kernel_source_digest(src.replace("k_spread_fftx", "k_spread_fftY", 1)) != rs.kernel_source_digest(src)


def test_roofline_from_the_spreading_work_record():
    # per-stage event times (ms summed over launches, launches) and the
    # spreading kernel's own work record: bytes per launch over mean duration
    prof = {"rotate": (1.0, 4), "spread_fft_x": (8.0, 4), "fft_y": (2.0, 4)}
    work = {"written_bytes": 3_000_000_000, "record_bytes": 1_000_000_000, "launches": 4}
    r = bench._roofline(prof, work, None)
    assert r["kernel"] == "spread_fft_x" and r["launches"] == 4
    assert r["mean_launch_ms"] == pytest.approx(2.0)
    assert r["alg_bytes_per_launch"] == pytest.approx(1e9)
    assert r["achieved"] == pytest.approx(1e9 / 2e-3 / 1e9)  # GB/s
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS)
    # a work record that does not cover the timed launches gives no figure
    r = bench._roofline(prof, dict(work, launches=3), None)
    assert r["achieved"] is None and r["frac"] is None
    # another dominant stage: timed, but with no byte record of its own
    r = bench._roofline(dict(prof, fft_y=(20.0, 4)), work, None)
    assert r["kernel"] == "fft_y" and r["achieved"] is None
