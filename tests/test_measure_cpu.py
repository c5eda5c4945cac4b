"""Measurement tooling on the CPU: the counter summary's arithmetic, its link to
the kernel source, and the bench's algorithmic byte model."""
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


def test_stage_byte_model():
    n, w = 128, 8
    info = {"n": n, "kb_width": w}
    pa = {"q": 10, "knots": 4096, "tile_rows": 8, "m": 256, "live_tiles": 883, "live_rows": 87}
    pb = dict(pa, live_tiles=903, live_rows=100)
    b = bench.stage_bytes(info, pa, pb)
    spec = 8 * n * n * (n // 2)
    rec = 4096 * (4 + 12 * w + 4 * 10)
    tile_out = lambda p: p["live_tiles"] * 8 * (256 // 4) * 8 * 10  # noqa: E731
    assert b["ifft_x"] == spec + 4 * n ** 3
    assert b["ifft_y"] == 2 * spec
    assert b["spread_fft_x"] == pytest.approx(rec + (tile_out(pa) + tile_out(pb)) / 2)
    assert b["fft_z_product"] == pb["live_rows"] * n * (n // 2) * 8 * 10 + 2 * spec
    # the spreading launch of the committed single-rotation workload: 37.2 MB
    assert b["spread_fft_x"] == pytest.approx(37.15e6, rel=1e-3)
