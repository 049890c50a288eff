"""The measurement pipeline's own arithmetic, on synthetic rocprofv3 output:
the clock summary (GRBM_GUI_ACTIVE per XCD over the dispatch time), the
counter summary's calibration and traffic, and the loaders that read a
committed summary only while its source hash matches the sweep sources."""
import csv
import os

import pytest

import bench


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                    "Start_Timestamp", "End_Timestamp"])
        for r in rows:
            w.writerow(r)


SWEEP_Z = "void teno::k_sweep<3, 2, 8, false, 74, false>(teno::SweepArgs)"
ALPHA = "void teno::k_alpha<3>(double const*, long, double, double*)"


def test_clock_summary_and_roofline_fields(tmp_path, monkeypatch):
    # 8 XCDs at 2.1 GHz for 1 ms: 8 x 2.1e6 busy cycles
    rows = []
    for i in range(4):
        rows.append([i, SWEEP_Z, "GRBM_GUI_ACTIVE", 8 * 2.1e6, 1000, 1000 + 1_000_000])
        rows.append([i, SWEEP_Z, "GRBM_COUNT", 8 * 2.1e6, 1000, 1000 + 1_000_000])
        rows.append([10 + i, ALPHA, "GRBM_GUI_ACTIVE", 8 * 2.35e5, 0, 100_000])
    _write_csv(str(tmp_path / "grbm" / "x" / "g_counter_collection.csv"), rows)
    clock_file = tmp_path / "clock.txt"
    monkeypatch.setattr(bench, "CLOCK_FILE", str(clock_file))
    bench.summarize_clock(str(tmp_path))
    text = clock_file.read_text()
    assert f"source_sha256: {bench.sources_sha()}" in text
    assert bench.load_clock_ghz("k_sweep<3,2,8,false>") == pytest.approx(2.1, abs=1e-3)
    assert bench.load_clock_ghz("k_alpha<3>") == pytest.approx(2.35, abs=1e-3)
    # a summary taken from other sources is not used
    clock_file.write_text(text.replace(bench.sources_sha(), "0" * 16))
    assert bench.load_clock_ghz("k_sweep<3,2,8,false>") is None


def test_counter_summary_calibration_and_ratio(tmp_path, monkeypatch):
    # the copy reads FETCH_SIZE = COPY_BYTES / 2 KiB-units (a factor 2.0) and
    # writes WRITE_SIZE = COPY_BYTES (1.0); the z sweep fetches and writes
    # exactly its algorithmic bytes after calibration
    kib = 1024.0
    cal_f, cal_w = 2.0, 1.0
    copy = "void at::native::vectorized_elementwise_kernel<4, copy>(int)"
    alg = bench.sweep_bytes(3, [256] * 3, 2, fused_rk=True)
    fetch_b, write_b = 0.75 * alg, 0.25 * alg
    d = tmp_path
    _write_csv(str(d / "calf" / "c.csv".replace(".csv", "_counter_collection.csv")),
               [[0, copy, "FETCH_SIZE", bench.COPY_BYTES / cal_f / kib, 0, 1]])
    _write_csv(str(d / "calw" / "c_counter_collection.csv"),
               [[0, copy, "WRITE_SIZE", bench.COPY_BYTES / cal_w / kib, 0, 1]])
    _write_csv(str(d / "fetch" / "f_counter_collection.csv"),
               [[0, SWEEP_Z, "FETCH_SIZE", fetch_b / cal_f / kib, 0, 1]])
    _write_csv(str(d / "write" / "w_counter_collection.csv"),
               [[0, SWEEP_Z, "WRITE_SIZE", write_b / cal_w / kib, 0, 1]])
    _write_csv(str(d / "valu" / "v_counter_collection.csv"),
               [[0, SWEEP_Z, "SQ_INSTS_VALU_FMA_F64", 1000.0, 0, 1],
                [0, SWEEP_Z, "SQ_INSTS_VALU_ADD_F64", 500.0, 0, 1]])
    traffic_file = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic_file))
    bench.summarize_counters(str(d))
    assert bench.load_traffic("k_sweep<3,2,8,false>") == pytest.approx(alg, rel=1e-6)
    assert "ratio=1.000" in traffic_file.read_text()
    # executed FP64 flop: 64 lanes x (ADD + 2 FMA)
    assert bench.load_executed_flop("k_sweep<3,2,8,false>") == pytest.approx(64 * (500 + 2000))
