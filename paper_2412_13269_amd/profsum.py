"""Summarise a rocprofv3 kernel trace (CSV, `--kernel-trace --output-format csv`)
by kernel and grid size: launches, average and total duration.

    python -m paper_2412_13269_amd.profsum <..._kernel_trace.csv> [--top N]
"""
from __future__ import annotations

import csv
import sys
from collections import defaultdict


def summarise(path: str, top: int = 25) -> str:
    groups = defaultdict(list)
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = row.get("Kernel_Name") or row.get("kernel_name") or "?"
            grid = row.get("Grid_Size_X") or row.get("Grid_Size") or row.get("grid_size_x") or "?"
            wg = row.get("Workgroup_Size_X") or row.get("Workgroup_Size") or "?"
            t0 = int(row.get("Start_Timestamp") or row.get("start_timestamp"))
            t1 = int(row.get("End_Timestamp") or row.get("end_timestamp"))
            short = name.split("(")[0].replace("void ", "")
            groups[(short, grid, wg)].append((t1 - t0) / 1000.0)
    total = sum(sum(v) for v in groups.values())
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]
    out = ["| kernel | grid (threads) | wg | launches | avg us | total us | share |", "|---|---|---|---|---|---|---|"]
    for (name, grid, wg), d in rows:
        out.append(f"| `{name}` | {grid} | {wg} | {len(d)} | {sum(d) / len(d):.2f} | {sum(d):.1f} | {sum(d) / total:.3f} |")
    return "\n".join(out)


if __name__ == "__main__":
    top = 25
    if "--top" in sys.argv:
        top = int(sys.argv[sys.argv.index("--top") + 1])
    print(summarise(sys.argv[1], top))
