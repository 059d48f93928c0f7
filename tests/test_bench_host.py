"""Host logic of bench.py (no GPU): the profile summaries written from
rocprofv3 CSV output, the traffic lookup that fills the bench line's
`traffic` fields, and the mapping of timing names to kernel symbols."""
import csv
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_traffic_scales_by_the_copy(tmp_path):
    """Counters in KiB per dispatch, scaled so that the calibration copy of
    nbytes reads and writes nbytes; means over dispatches."""
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    nbytes = 1 << 20
    kern = "void fftfem::line_kernel<double, 9, 0, false, false, 0>(fftfem::LineArgs<double>)"
    _write_csv(str(tmp_path / "f" / "run_counter_collection.csv"), hdr,
               [["__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0], [kern, "FETCH_SIZE", 100.0],
                [kern, "FETCH_SIZE", 300.0]])
    _write_csv(str(tmp_path / "w" / "run_counter_collection.csv"), hdr,
               [["__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0], [kern, "WRITE_SIZE", 50.0]])
    out = str(tmp_path / "t.txt")
    bench.summarize_traffic("wl_mode", str(tmp_path / "f"), str(tmp_path / "w"), str(nbytes), "fcmd", "wcmd", out)
    text = open(out).read()
    assert f"sources_sha256: {bench.sources_sha256()}" in text
    row = [line for line in text.splitlines() if line.startswith("kernel:")][0]
    kv = dict(x.strip().split("=") for x in row.split("|")[1:])
    # fetch factor 2 (512 KiB read for 1 MiB), mean 200 KiB -> 400 KiB; write factor 1 -> 50 KiB
    assert float(kv["fetch_bytes"]) == pytest.approx(400 * 1024)
    assert float(kv["write_bytes"]) == pytest.approx(50 * 1024)
    assert float(kv["bytes"]) == pytest.approx(450 * 1024)


def test_traffic_lookup_per_mode_and_stale_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    sym = "line_kernel<double, 9, 0, false, false, 0>"
    sha = bench.sources_sha256()
    for mode, val in (("fp64", 1.5e9), ("fp64_b", 2.5e9)):
        (prof / f"traffic_w_{mode}.txt").write_text(
            f"sources_sha256: {sha}\n"
            f"kernel: void fftfem::{sym}(x) | dispatches=1 | fetch_bytes=1 | write_bytes=1 | bytes={val}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_sha256", lambda: sha)
    assert bench.measured_traffic("w", sym, "fp64") == 1.5e9
    assert bench.measured_traffic("w", sym, "fp64_b") == 2.5e9
    assert bench.measured_traffic("w", sym, "fp32") is None  # no file of that mode, none of the workload
    monkeypatch.setattr(bench, "sources_sha256", lambda: "other")
    assert bench.measured_traffic("w", sym, "fp64") is None  # counters taken on other sources


def test_profiler_kernel_names():
    assert bench.profiler_kernel_name("fwd64_ax1", 9, 2, 1024) == "line_kernel<double, 9, 0, false, false, 0>"
    assert bench.profiler_kernel_name("mid64_ax0t", 9, 2, 1024) == "line_kernel<double, 9, 2, false, false, 0>"
    assert bench.profiler_kernel_name("inv32_ax0", 5, 2, 48) == "line_kernel<float, 5, 1, false, true, 1>"
    assert bench.profiler_kernel_name("fwd32_ax1", 5, 2, 31) == "line_kernel<float, 5, 0, false, false, 2>"
    assert bench.profiler_kernel_name("inv_upd32_ax1", 9, 2, 1024) == "line_kernel<float, 9, 1, true, false, 0>"
    assert bench.profiler_kernel_name("transpose32", 9, 2, 1024) == "transpose_kernel<float>"
    assert bench.profiler_kernel_name("resid2dd", 9, 2, 1024) == "resid2_kernel<9, true>"
    assert bench.profiler_kernel_name("bandtile64_ax0", 9, 3, 64).startswith("band_tile_kernel<9, ")


def test_summarize_replay_finds_the_periodic_tail(tmp_path):
    """Three identical replays of two kernels with a 5 ns gap: busy time is
    the union of the kernels' intervals, gaps are reported."""
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows, t = [], 0
    for rep in range(4):
        for k in range(120):
            rows.append([f"fftfem::k{k}_kernel", t, t + 100])
            t += 105
    _write_csv(str(tmp_path / "tr" / "run_kernel_trace.csv"), hdr, rows)
    out = str(tmp_path / "r.txt")
    bench.summarize_replay(str(tmp_path / "tr"), "cmd", out)
    text = open(out).read()
    assert "replay -1: launches 120" in text
    line = [s for s in text.splitlines() if s.startswith("replay -1")][0]
    frac = float(line.split("(")[-1].split(" of wall")[0])
    assert frac == pytest.approx(120 * 100 / (120 * 105 - 5), rel=1e-3)
    assert "idle gaps between kernels: total 0.001 ms" in text  # 119 gaps of 5 ns


def test_summarize_counters_derives_busy_and_residency(tmp_path):
    """Means over dispatches; VALU busy and resident waves from the kernel's
    mean duration over the modes of a bench line (one symbol, two modes)."""
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    kern = "void fftfem::line_kernel<double, 9, 0, false, false, 0>(fftfem::LineArgs<double>)"
    rows = []
    for v in (100.0, 300.0):
        rows += [[kern, "SQ_WAVES", 1000.0], [kern, "SQ_INSTS_VALU", 2.0e6], [kern, "SQ_INSTS_LDS", 1.0e5],
                 [kern, "SQ_WAVE_CYCLES", 6.144e8], [kern, "SQ_WAIT_INST_LDS", v * 1e4]]
    _write_csv(str(tmp_path / "c" / "run_counter_collection.csv"), hdr, rows)
    line = {"config": {"N": 2, "n": 9, "K": [1024, 1024]},
            "modes": {"fp64": {"kernels_ms": {"fwd64_ax1": 1.5}}, "fp64_b": {"kernels_ms": {"fwd64_ax1": 0.5}}}}
    (tmp_path / "b.json").write_text("noise\n" + __import__("json").dumps(line) + "\n")
    out = str(tmp_path / "c.txt")
    bench.summarize_counters(str(tmp_path / "c"), str(tmp_path / "b.json"), "t", "cmd", out)
    row = [x for x in open(out).read().splitlines() if x.startswith("void fftfem::line_kernel")][0]
    f = [x.strip() for x in row.split("|")]
    # duration 1.0 ms (mean of the two modes) = 2.4e6 cycles
    assert f[1] == "1.000" and f[2] == "1000" and f[3] == "2000" and f[4] == "100"
    assert float(f[5]) == pytest.approx(2.0e6 * 4 / (4 * 256 * 2.4e6), abs=0.01)
    assert float(f[6]) == pytest.approx(2.0e6 / 6.144e8, abs=1e-3)
    assert float(f[7]) == pytest.approx(6.144e8 * 4 / (256 * 2.4e6), abs=0.1)
