"""Host-side checks of bench.py's counter summaries (no GPU): the FP64 MFMA
flops, rate and busy fraction from rocprofv3 counter rows."""
import csv
import importlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    sys.path.insert(0, ROOT)
    return importlib.import_module("bench")


def test_mfma_summary_from_counter_rows(tmp_path, monkeypatch):
    bench = _bench()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    d = tmp_path / "run"
    d.mkdir()
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    rows = []
    # two launches of 2 ms, each 4,000 v_mfma_f64_16x16x4f64 (2,048 flops and
    # 64 busy cycles apiece) over 4.8e6 clocks of each of the 8 XCDs
    for disp in (1, 2):
        t0, t1 = 10**9 * disp, 10**9 * disp + 2_000_000
        vals = {"SQ_INSTS_VALU_MFMA_MOPS_F64": 4000 * 2048 / 512, "SQ_VALU_MFMA_BUSY_CYCLES": 4000 * 64,
                "SQ_BUSY_CYCLES": 1.0, "GRBM_GUI_ACTIVE": 8 * 4.8e6}
        for name, v in vals.items():
            rows.append({"Dispatch_Id": disp, "Kernel_Name": "void pxs::k_selinv_off<64, pxs::OnePanel>(pxs::OnePanel)",
                         "Counter_Name": name, "Counter_Value": v, "Start_Timestamp": t0, "End_Timestamp": t1})
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)
    bench.mfma_from_counters("toy", str(d), "cmd")
    out = json.load(open(tmp_path / "profiles" / "mfma_toy.json"))
    k = out["kernels"]["k_selinv_off"]
    assert k["launches"] == 2
    assert k["mfma_flops_per_launch"] == 4000 * 2048
    assert k["avg_launch_ms"] == 2.0
    assert abs(k["mfma_tflops"] - 4000 * 2048 / 2e-3 / 1e12) < 0.01
    # 256,000 busy cycles over 4.8e6 clocks x 1,024 SIMDs
    assert abs(k["mfma_busy_frac"] - round(4000 * 64 / (4.8e6 * 1024), 4)) < 1e-9
    assert abs(k["clock_ghz"] - 2.4) < 1e-9
