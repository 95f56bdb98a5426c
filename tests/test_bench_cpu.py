"""Host logic of bench.py that needs no GPU: the roofline block, the folding
of rocprofv3 counter files into the counters file, and the one-GPU guard."""
import argparse
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SURVEY_ADDS = 1024 * 503832 * 1024


def test_roofline_peak_is_the_packed_lane_rate():
    # 39.32 T 32-bit lane operations/s; eight 2-bit or two 8-bit channel-adds each
    assert bench.alu_peak_tadds(2) == pytest.approx(8 * 39.3216)
    assert bench.alu_peak_tadds(8) == pytest.approx(2 * 39.3216)
    blk = bench.roofline_block(2, SURVEY_ADDS, 4.66, None)
    assert blk["bound"] == "alu" and blk["unit"] == "Tadd/s"
    assert blk["achieved"] == pytest.approx(SURVEY_ADDS / 4.66e-3 / 1e12)
    assert blk["frac"] == pytest.approx(blk["achieved"] / blk["peak"])
    assert 0 < blk["frac"] < 1
    assert blk["traffic"] is None and blk["valu_issue"] is None


def test_roofline_reads_counters():
    ctr = {"hbm_bytes_per_launch": 3.2e9, "grbm_gui_active": 8 * 1.0e7, "sq_insts_valu": 1.0e9,
           "sq_lds_idx_active": 256 * 0.5e7, "kernel": ["k"]}
    blk = bench.roofline_block(2, SURVEY_ADDS, 4.66, ctr)
    assert blk["traffic"] == 3.2e9
    # 1e9 wave64 instructions x 4 cycles over 1024 SIMDs x 1e7 cycles
    assert blk["valu_issue"] == pytest.approx(4e9 / (1024 * 1e7))
    assert blk["lds_busy"] == pytest.approx(0.5)
    assert blk["counters_kernel_us"] == pytest.approx(1e7 / 2.4e3)


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summarize_counters_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    kern = "void dedisp::k_tiled<4, 16, 1, 3, 64, 1>(dedisp::BeamDesc)"
    other = "void dedisp::k_unpack_planes(dedisp::BeamDesc)"
    # two dispatches of the kernel (one counter row each), one of another kernel
    _write_counters(tmp_path / "p1", [
        {"Dispatch_Id": 1, "Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000.0},
        {"Dispatch_Id": 2, "Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": 3000.0},
        {"Dispatch_Id": 3, "Kernel_Name": other, "Counter_Name": "FETCH_SIZE", "Counter_Value": 9e9}])
    _write_counters(tmp_path / "p2", [
        {"Dispatch_Id": 1, "Kernel_Name": kern, "Counter_Name": "WRITE_SIZE", "Counter_Value": 500.0},
        {"Dispatch_Id": 1, "Kernel_Name": kern, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 7.0}])
    # a 1 GiB copy reads half its bytes in FETCH_SIZE and all of them in WRITE_SIZE
    _write_counters(tmp_path / "cf", [{"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer",
                                       "Counter_Name": "FETCH_SIZE", "Counter_Value": 524288.0}])
    _write_counters(tmp_path / "cw", [{"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer",
                                       "Counter_Name": "WRITE_SIZE", "Counter_Value": 1048576.0}])
    out = tmp_path / "counters.json"
    args = argparse.Namespace(summarize_counters=[str(tmp_path / "p1"), str(tmp_path / "p2")],
                              tile_key="16,1,3,64,4", kernel_filter="k_tiled<4, 16, 1, 3, 64, 1>",
                              calibration_dirs=[str(tmp_path / "cf"), str(tmp_path / "cw")],
                              workload="survey-2bit-1024ch", counters_json=str(out))
    bench.summarize_counters(args)
    doc = json.load(open(out))
    (e,) = doc["entries"]
    assert e["fetch_scale_from_copy"] == pytest.approx(2.0)
    assert e["write_scale_from_copy"] == pytest.approx(1.0)
    assert e["counters_per_dispatch"]["FETCH_SIZE"] == pytest.approx(2000.0)   # the kernel's mean only
    assert e["hbm_bytes_per_launch"] == pytest.approx((2000.0 * 2 + 500.0) * 1024)
    assert e["sq_insts_valu"] == 7.0
    tile = dict(kind=0, waves=16, dms_per_wave=1, words_per_lane=3, chunk_chans=64, sample_format=4)
    assert e["tile"] == tile
    # looked up by workload, tile and the current kernel sources
    assert bench.counters_for(str(out), "survey-2bit-1024ch", tile) == e
    assert bench.counters_for(str(out), "large-8bit-4096ch", tile) is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 64)
    assert bench.counters_for(str(out), "survey-2bit-1024ch", tile) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
