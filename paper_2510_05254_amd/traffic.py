"""Reduce two rocprofv3 counter runs of bench.py to measured HBM bytes per
stage-kernel launch.

    python -m paper_2510_05254_amd.traffic --fetch F.csv --write W.csv \
        --workload euler3d_64x64x64_N4 --precision fp64 --out profiles/...json

F.csv / W.csv are the counter_collection.csv files of `rocprofv3 --pmc
FETCH_SIZE` and `rocprofv3 --pmc WRITE_SIZE` over the same bench.py command.
The raw counters are scaled by what they read for bench.py's own calibration
copies in the same run (device-to-device copies of exactly 2 GiB, the largest
copyBuffer dispatches), so bytes = counter * (2 GiB / counter of the copy).
The output records the hash of the stage kernel's source with its comments
removed (code_only), so bench.py drops the record once the code changes and
keeps it across comment edits.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 31                  # bench.py: torch.empty(1 << 28, float64)
KERNEL_SOURCES = ["paper_2510_05254_amd/csrc/dg_stage.hpp"]


def code_only(text: str) -> str:
    """C++ source without its comments, trailing blanks and empty lines: what
    the compiler reads, so that editing a comment keeps recorded counters
    valid while any change to the code itself does not."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":                       # string or character literal
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            while i < n and text[i] != "\n":
                i += 1
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = ("".join(out)).split("\n")
    return "\n".join(line.rstrip() for line in lines if line.strip())


def kernel_hash() -> str:
    """Hash of the stage-kernel sources, comments excluded (code_only)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(code_only(open(os.path.join(ROOT, f), encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def per_dispatch(path: str, counter: str):
    """[(kernel name, value)] per dispatch, summed over the counter's instances."""
    vals = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        key = (r["Dispatch_Id"], r["Kernel_Name"])
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    return [(name, v) for (_, name), v in sorted(vals.items(), key=lambda kv: int(kv[0][0]))]


def reduce(path: str, counter: str, kernel: str):
    rows = per_dispatch(path, counter)
    copies = [v for name, v in rows if "copyBuffer" in name]
    if not copies:
        raise SystemExit(f"{path}: no copyBuffer dispatch to calibrate {counter}")
    top = max(copies)
    cal = [v for v in copies if v >= 0.9 * top]
    factor = COPY_BYTES / statistics.median(cal)
    ks = [v for name, v in rows if kernel in name]
    if not ks:
        raise SystemExit(f"{path}: no dispatch of {kernel}")
    return {"counter": counter, "bytes_per_unit": factor, "calibration_dispatches": len(cal),
            "kernel_dispatches": len(ks), "kernel_mean_units": statistics.mean(ks),
            "bytes_per_launch": statistics.mean(ks) * factor}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--precision", required=True)
    ap.add_argument("--kernel", default="stage_kernel")
    ap.add_argument("--command", default="", help="the profiled command, recorded as is")
    ap.add_argument("--rk", type=int, default=4, help="RK scheme of the profiled run")
    ap.add_argument("--launch-config", default=None,
                    help="tile order, z-slab, x-block, z-march length of the profiled run "
                         "(bench.py's launch_config)")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    f = reduce(a.fetch, "FETCH_SIZE", a.kernel)
    w = reduce(a.write, "WRITE_SIZE", a.kernel)
    rec = {"workload": a.workload, "precision": a.precision, "kernel": a.kernel,
           "kernel_hash": kernel_hash(), "rk": a.rk,
           "bytes_per_launch": f["bytes_per_launch"] + w["bytes_per_launch"],
           "fetch": f, "write": w, "command": a.command}
    if a.launch_config:
        rec["launch_config"] = [int(x) for x in a.launch_config.split(",")]
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
