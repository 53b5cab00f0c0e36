"""Summaries of the rocprofv3 runs of the benchmark step, for the roofline
object's `traffic` figure and the committed profile notes.

Reads, under a result folder (default ``gpurun_out``):
  pmc_fetch/, pmc_write/  FETCH_SIZE and WRITE_SIZE passes over the step,
  pmc_cf/, pmc_cw/        the same counters over a copy of 1 GiB
                          (``bench.py --copy-calibration``),
  prof_c2/                the kernel trace with --stats (optional),
  pmc_mfma/               SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE (optional),
each with ``--output-format csv -o run``.  Writes ``profiles/traffic.json``:
per kernel class, HBM bytes per launch = counter KiB x 1024 x the copy's
scale (bytes copied / counter bytes read for the copy), with the hash of the
kernel sources it was taken from; ``bench.py`` uses a class's figure only
while that hash matches.  Prints the kernel-stats table and the MFMA busy
ratio per class.

    python -m paper_2508_07610_amd.pmc_summary [result_folder]
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_07610_amd", "csrc")

# sources that decide a kernel class's code and the shapes it is launched with
KERNEL_SOURCES = {
    "k_gemm": ("gemm.hip", "common.h", "ops.hip", "ops.h", "engine.hip", "engine.h", "kernels.h"),
    "k_heev": ("eigh.hip", "common.h", "ops.hip", "engine.hip", "kernels.h"),
}

STEP = ("python3 -u bench.py --steps 1 --warmup 1 --no-cpu --no-ttf --no-crosstalk --no-maxcut --no-sampling "
        "--no-gemm-tiles --no-noise-models --no-truncation-study --no-sweep --no-mitigation")


def kernel_sources_hash(kernel: str) -> str:
    h = hashlib.sha256()
    key = "k_gemm" if kernel.startswith("k_gemm") else "k_heev"
    for f in KERNEL_SOURCES[key]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def kernel_class(name: str):
    if "k_q2_chol_e" in name:
        return "k_q2_chol_e"
    if "k_heev_global" in name:
        return "k_heev_global"
    if "k_heev_reg" in name:
        return "k_heev_reg"
    if "k_heev_band" in name:
        return "k_heev_band"
    if "k_gemm<double, double" in name:
        return "k_gemm (FP64 MFMA)"
    if "k_gemm<float" in name or "k_gemm<double, float" in name:
        return "k_gemm (FP32 MFMA)"
    return None


def _rows(path):
    with open(path) as f:
        yield from csv.DictReader(f)


def per_class(path: str, counter: str) -> dict:
    acc = collections.defaultdict(lambda: [0, 0.0])
    for r in _rows(path):
        if r["Counter_Name"] != counter:
            continue
        c = kernel_class(r["Kernel_Name"])
        if c is not None:
            acc[c][0] += 1
            acc[c][1] += float(r["Counter_Value"])
    return acc


def copy_reading(path: str, counter: str) -> float:
    vals = [float(r["Counter_Value"]) for r in _rows(path)
            if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no copy kernel with {counter} in {path}")
    return sum(vals) / len(vals)


def summarize(out: str) -> dict:
    fk = copy_reading(os.path.join(out, "pmc_cf", "run_counter_collection.csv"), "FETCH_SIZE")
    wk = copy_reading(os.path.join(out, "pmc_cw", "run_counter_collection.csv"), "WRITE_SIZE")
    gib_kib = 1024.0 * 1024.0
    fs, ws = gib_kib / fk, gib_kib / wk
    fetch = per_class(os.path.join(out, "pmc_fetch", "run_counter_collection.csv"), "FETCH_SIZE")
    write = per_class(os.path.join(out, "pmc_write", "run_counter_collection.csv"), "WRITE_SIZE")
    traffic = {}
    for c in sorted(set(fetch) | set(write)):
        nf, sf = fetch.get(c, [0, 0.0])
        nw, sw = write.get(c, [0, 0.0])
        fb = sf / max(nf, 1) * 1024 * fs
        wb = sw / max(nw, 1) * 1024 * ws
        traffic[c] = {"sources": kernel_sources_hash(c), "dispatches": nf, "fetch_bytes_per_launch": fb,
                      "write_bytes_per_launch": wb, "bytes_per_launch": fb + wb}
    traffic["_calibration"] = {"copy_bytes": 1 << 30, "fetch_kib_read": fk, "write_kib_read": wk,
                               "fetch_scale": fs, "write_scale": ws}
    traffic["_command"] = (f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o run -- {STEP} "
                           "(then WRITE_SIZE into gpurun_out/pmc_write); calibration: the same two passes over "
                           "python3 -u bench.py --copy-calibration (1 GiB copied three times)")
    return traffic


def main(argv) -> None:
    out = argv[1] if len(argv) > 1 else os.path.join(ROOT, "gpurun_out")
    traffic = summarize(out)
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(traffic, f, indent=1)
    print(json.dumps({k: v for k, v in traffic.items() if not k.startswith("_")}, indent=1))
    cal = traffic["_calibration"]
    print(f"copy scale: fetch x {cal['fetch_scale']:.3f}, write x {cal['write_scale']:.3f}")
    stats = os.path.join(out, "prof_c2", "run_kernel_stats.csv")
    if os.path.exists(stats):
        print("| kernel | calls | avg (us) | share (%) |")
        for r in list(_rows(stats))[:20]:
            print(f"| `{r['Name'].split('(')[0]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                  f"{float(r['Percentage']):.2f} |")
    busy_csv = os.path.join(out, "pmc_mfma", "run_counter_collection.csv")
    if os.path.exists(busy_csv):
        recs = collections.defaultdict(dict)
        for r in _rows(busy_csv):
            recs[r["Dispatch_Id"]][r["Counter_Name"]] = float(r["Counter_Value"])
            recs[r["Dispatch_Id"]]["name"] = r["Kernel_Name"]
        busy = collections.defaultdict(lambda: [0, 0.0, 0.0])
        for d in recs.values():
            c = kernel_class(d["name"])
            if c is not None:
                busy[c][0] += 1
                busy[c][1] += d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
                busy[c][2] += d.get("GRBM_GUI_ACTIVE", 0.0)
        for c, (n, b, g) in sorted(busy.items()):
            print(f"{c}: {n} dispatches, SQ_VALU_MFMA_BUSY_CYCLES / GRBM_GUI_ACTIVE = {b / max(g, 1.0):.1f}")


if __name__ == "__main__":
    main(sys.argv)
