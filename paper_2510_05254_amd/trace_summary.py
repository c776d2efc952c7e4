"""Summarise a rocprofv3 kernel trace of bench.py over its timed launches only.

    python -m paper_2510_05254_amd.trace_summary --trace T_kernel_trace.csv \
        --kernel stage_kernel --skip 8 --take 200 [--md out.md]

T_kernel_trace.csv is the kernel_trace.csv of
`rocprofv3 --kernel-trace --output-format csv` over a bench.py run. The
dispatches of kernels whose name contains --kernel are taken in dispatch
order; the first --skip (the warm-up steps' launches: warmup x stages) are
dropped and the next --take (steps x stages x repeats: the timed region) are
summarised: count, total, mean, min and max duration per instantiation and
over all of them, in microseconds.
"""
from __future__ import annotations

import argparse
import csv
import statistics


def dispatches(path: str, kernel: str):
    rows = []
    for r in csv.DictReader(open(path)):
        name = r.get("Kernel_Name", "")
        if kernel not in name:
            continue
        t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        rows.append((int(r["Dispatch_Id"]), name, (t1 - t0) / 1e3, t0, t1))
    rows.sort()
    return rows


def summarise(rows):
    d = [r[2] for r in rows]
    return {"count": len(d), "total_us": sum(d), "mean_us": statistics.mean(d),
            "min_us": min(d), "max_us": max(d)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--kernel", default="stage_kernel")
    ap.add_argument("--skip", type=int, default=0, help="leading dispatches to drop (warm-up)")
    ap.add_argument("--take", type=int, required=True, help="dispatches of the timed region")
    ap.add_argument("--md", default=None, help="write the table as markdown here")
    a = ap.parse_args()
    rows = dispatches(a.trace, a.kernel)
    if len(rows) < a.skip + a.take:
        raise SystemExit(f"{a.trace}: {len(rows)} dispatches of {a.kernel}, need {a.skip + a.take}")
    sel = rows[a.skip:a.skip + a.take]
    span_us = (sel[-1][4] - sel[0][3]) / 1e3
    names = sorted({r[1] for r in sel})
    lines = ["| kernel | launches | total (us) | mean (us) | min (us) | max (us) |",
             "|:--|--:|--:|--:|--:|--:|"]
    for n in names:
        s = summarise([r for r in sel if r[1] == n])
        lines.append(f"| `{n}` | {s['count']} | {s['total_us']:.1f} | {s['mean_us']:.1f} | "
                     f"{s['min_us']:.1f} | {s['max_us']:.1f} |")
    s = summarise(sel)
    lines.append(f"| all timed launches | {s['count']} | {s['total_us']:.1f} | {s['mean_us']:.1f} | "
                 f"{s['min_us']:.1f} | {s['max_us']:.1f} |")
    lines.append("")
    lines.append(f"first timed launch start to last timed launch end: {span_us:.1f} us "
                 f"({span_us / len(sel):.1f} us per launch, gaps included)")
    text = "\n".join(lines)
    print(text)
    if a.md:
        with open(a.md, "w") as fh:
            fh.write(text + "\n")


if __name__ == "__main__":
    main()
