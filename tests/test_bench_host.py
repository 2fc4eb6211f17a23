"""CPU checks of bench.py's host-side helpers: the HBM traffic figure built
from two rocprofv3 counter files (FETCH_SIZE, WRITE_SIZE per dispatch),
scaled by the calibration kernel of known size, and its staleness guard."""

import csv
import json
import os

import pytest

native = pytest.importorskip("paper_2410_21607_amd.native")

HEADER = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]
CALIB = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<double, double, double>>"
COLS = "void sem::k_stage_columns<5, 4, double, false, false, 1>(sem::DevMesh)"
COLS0 = "void sem::k_stage_columns<5, 4, double, false, false, 0>(sem::DevMesh)"


def _write(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HEADER)
        for i, (name, value) in enumerate(rows):
            w.writerow([i, i, "Agent 1", 1, 1, 1, 1, 1, name, 256, 0, 0, 8, 0, 8, counter, value, 0, 1])


def test_traffic_from_counters(tmp_path):
    if not os.path.exists(native.LIB_PATH):
        pytest.skip("libsem.so not built")
    import bench
    from paper_2410_21607_amd.api import sem_mesh_plan
    from synth import cases
    info = sem_mesh_plan(cases.get("vortex_8x8x4_n4"))[0]
    calib_bytes = 5 * info["n_h"] * info["ldz"] * 8
    # the calibration reads its array through FETCH_SIZE at half its bytes
    # (a factor of 2) and writes it through WRITE_SIZE at its bytes; the
    # column kernel's medians are 300 and 100 KiB per dispatch
    fetch = [(CALIB, calib_bytes / 2048)] * 5 + [(COLS, 300.0)] * 7 + [(COLS, 1e9)] * 2
    write = [(CALIB, calib_bytes / 1024)] * 5 + [(COLS, 100.0)] * 7 + [(COLS, 0.0)] * 2
    _write(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _write(tmp_path / "w.csv", "WRITE_SIZE", write)
    out = bench.traffic_from_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                                      "vortex_8x8x4_n4", launches_per_stage=4, out_dir=str(tmp_path))
    assert out["fetch_factor"] == pytest.approx(2.0) and out["write_factor"] == pytest.approx(1.0)
    assert out["hbm_bytes_per_stage"] == pytest.approx(4 * 1024 * (300.0 * 2 + 100.0))
    assert out["kernel"] == COLS and out["dispatches"] == 9
    saved = json.load(open(tmp_path / "traffic_vortex_8x8x4_n4.json"))["records"]
    assert len(saved) == 1 and saved[0]["kernel_source_hash"] == bench.kernel_source_hash()
    # a second instance's counters join the file; the same instance replaces its record
    _write(tmp_path / "f0.csv", "FETCH_SIZE", [(CALIB, calib_bytes / 2048)] * 5 + [(COLS0, 400.0)] * 9)
    _write(tmp_path / "w0.csv", "WRITE_SIZE", [(CALIB, calib_bytes / 1024)] * 5 + [(COLS0, 100.0)] * 9)
    bench.traffic_from_counters(str(tmp_path / "f0.csv"), str(tmp_path / "w0.csv"),
                                "vortex_8x8x4_n4", out_dir=str(tmp_path))
    bench.traffic_from_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                                "vortex_8x8x4_n4", out_dir=str(tmp_path))
    saved = json.load(open(tmp_path / "traffic_vortex_8x8x4_n4.json"))["records"]
    assert sorted(r["kernel"] for r in saved) == sorted([COLS, COLS0])
    # two counter runs whose autotuners chose different instances are refused
    _write(tmp_path / "w2.csv", "WRITE_SIZE",
           [(CALIB, calib_bytes / 1024)] * 5 + [(COLS0, 100.0)] * 9 + [(COLS, 100.0)] * 2)
    with pytest.raises(ValueError):
        bench.traffic_from_counters(str(tmp_path / "f.csv"), str(tmp_path / "w2.csv"),
                                    "vortex_8x8x4_n4", out_dir=str(tmp_path))


def test_measured_traffic_is_null_for_other_sources(tmp_path, monkeypatch):
    """The committed figure is used only with the kernel sources it was taken on."""
    import bench
    h = bench.kernel_source_hash()
    d = tmp_path / "profiles"
    d.mkdir()
    json.dump({"kernel_source_hash": "0" * 16, "hbm_bytes_per_stage": 1.0}, open(d / "traffic_x.json", "w"))
    json.dump({"kernel_source_hash": h, "hbm_bytes_per_stage": 2.0}, open(d / "traffic_y.json", "w"))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("x") is None
    assert bench.measured_traffic("y") == 2.0
    assert bench.measured_traffic("z") is None


def test_measured_traffic_picks_the_record_of_the_instance(tmp_path, monkeypatch):
    import bench
    h = bench.kernel_source_hash()
    d = tmp_path / "profiles"
    d.mkdir()
    json.dump({"records": [{"kernel_source_hash": h, "hbm_bytes_per_stage": 5.0, "kernel": COLS0},
                           {"kernel_source_hash": h, "hbm_bytes_per_stage": 6.0, "kernel": COLS}]},
              open(d / "traffic_v.json", "w"))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("v", bench.column_instance(4, 4, 0, True, False)) == 5.0
    assert bench.measured_traffic("v", bench.column_instance(4, 4, 2, True, False)) == 6.0
    assert bench.measured_traffic("v", bench.column_instance(4, 4, 3, True, False)) is None


def test_measured_traffic_only_for_the_instance_timed(tmp_path, monkeypatch):
    """A figure taken on one thread order or chunk depth is not reported for another."""
    import bench
    h = bench.kernel_source_hash()
    d = tmp_path / "profiles"
    d.mkdir()
    json.dump({"kernel_source_hash": h, "hbm_bytes_per_stage": 3.0, "kernel": COLS},
              open(d / "traffic_w.json", "w"))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    timed = bench.column_instance(4, 4, 2, True, False)
    assert timed == "k_stage_columns<5, 4, double, false, false, 1>"
    assert bench.measured_traffic("w", timed) == 3.0
    assert bench.measured_traffic("w", bench.column_instance(4, 4, 0, True, False)) is None
    assert bench.measured_traffic("w", bench.column_instance(4, 2, 2, True, False)) is None
    assert bench.column_instance(4, 4, 1, True, False) is None          # block layout
    assert bench.column_instance(4, 4, 3, False, False).endswith("float, false, false, 1>")
