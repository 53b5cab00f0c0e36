"""The counter summary behind profiles/traffic.json (no GPU): bytes per
launch are the counter's KiB scaled by what the same counter reads for a
copy of 1 GiB, averaged over a class's dispatches, with the hash of the
class's kernel sources."""
import csv
import os

import pytest

from paper_2508_07610_amd import pmc_summary as PS


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_scaling_and_class_averages(tmp_path):
    out = str(tmp_path)
    gib_kib = 1024.0 * 1024.0
    # the copy reads half its bytes on FETCH_SIZE and all of them on WRITE_SIZE
    _write(f"{out}/pmc_cf/run_counter_collection.csv", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", gib_kib / 2)] * 3)
    _write(f"{out}/pmc_cw/run_counter_collection.csv", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", gib_kib)] * 3)
    g = "void mpdo::k_gemm<double, double, double, 64, 64, false>(...)"
    _write(f"{out}/pmc_fetch/run_counter_collection.csv",
           [(g, "FETCH_SIZE", 100.0), (g, "FETCH_SIZE", 300.0), ("mpdo::k_heev_global(...)", "FETCH_SIZE", 10.0),
            ("void mpdo::k_q2_chol_e<double>(...)", "FETCH_SIZE", 4.0), ("other_kernel", "FETCH_SIZE", 1e9)])
    _write(f"{out}/pmc_write/run_counter_collection.csv",
           [(g, "WRITE_SIZE", 50.0), (g, "WRITE_SIZE", 50.0), ("mpdo::k_heev_global(...)", "WRITE_SIZE", 5.0)])
    t = PS.summarize(out)
    assert t["_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert t["_calibration"]["write_scale"] == pytest.approx(1.0)
    gemm = t["k_gemm (FP64 MFMA)"]
    assert gemm["dispatches"] == 2
    assert gemm["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2.0)
    assert gemm["write_bytes_per_launch"] == pytest.approx(50.0 * 1024)
    assert gemm["bytes_per_launch"] == pytest.approx(gemm["fetch_bytes_per_launch"] + gemm["write_bytes_per_launch"])
    assert gemm["sources"] == PS.kernel_sources_hash("k_gemm (FP64 MFMA)")
    assert t["k_heev_global"]["sources"] == PS.kernel_sources_hash("k_heev_global")
    assert "k_q2_chol_e" in t and "other_kernel" not in str(t)


def test_class_names():
    assert PS.kernel_class("void mpdo::k_gemm<float, float, float, 32, 32, true>(x)") == "k_gemm (FP32 MFMA)"
    assert PS.kernel_class("void mpdo::k_gemm<double, double, float, 64, 64, false>(x)") == "k_gemm (FP64 MFMA)"
    assert PS.kernel_class("void mpdo::k_heev_reg<128, 512, 32, 4>(x)") == "k_heev_reg"
    assert PS.kernel_class("mpdo::k_transfer_prep<double>") is None

