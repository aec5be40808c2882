"""Summarise rocprofv3 CSV output by kernel and grid size.

    python -m paper_2412_13269_amd.profsum <..._kernel_trace.csv> [--top N]
        launches, average and total duration (`--kernel-trace --output-format csv`)
    python -m paper_2412_13269_amd.profsum --pmc <..._counter_collection.csv> [--match REGEX]
        per-dispatch average of every collected counter (`--pmc ...`), with the
        kernel's VGPR/SGPR counts and LDS block size
    python -m paper_2412_13269_amd.profsum --traffic <FETCH_SIZE csv> <WRITE_SIZE csv>
            --kernel REGEX --copy REGEX:GRID:KIB
        HBM bytes per dispatch of the kernels matching --kernel (all their
        dispatches), each counter scaled by what it reads for the copy kernel
        of known size (dispatches of that name and grid; KIB read = KIB written)
    python -m paper_2412_13269_amd.profsum --runs R <..._kernel_trace.csv> [--top N]
        the kernels after the longest idle gap of the trace (the runs after
        the setup: `workload --query` idles 0.5 s there), grouped by kernel
        name, per run (divided by R), with the device's busy and idle time
        over that span
        with --name NAME it also prints the machine-readable line
        "traffic_bytes_per_launch: B kernel: NAME sources_sha256: H" (H over
        the sources that define the kernel, SOURCES[NAME])
    python -m paper_2412_13269_amd.profsum --valu-per-op <SQ counters csv> --after REGEX --ops K
        VALU wave instructions (SQ_INSTS_VALU) summed over every dispatch
        after the last one of the marker kernel REGEX, divided by K, and the
        line "valu_wave_instructions_per_rotation: V sources_sha256: H" (H over
        SOURCES["ks_rotation"]); for `workload --rotations-only --calibrate`
    python -m paper_2412_13269_amd.profsum --valu <SQ counters csv> <..._kernel_trace.csv> [--top N]
        per kernel and grid: VALU wave instructions per dispatch (SQ_INSTS_VALU),
        the average duration from the trace run, and the issue rate against
        the chip's peak for full-rate FP64 VALU instructions: 256 CUs x 4 SIMDs
        x 2.4 GHz / 4 cycles per wave64 instruction = 614.4 G/s
"""
from __future__ import annotations

import csv
import hashlib
import os
import sys
from collections import defaultdict

# sources that define a profiled kernel: their hash ties a committed counter
# measurement to the code it was taken on
SOURCES = {"ks_inner": ["kernels.hip", "modarith.h", "ntt_core.h", "internal.h"],
           "repack_fused": ["keyswitch.hip", "modarith.h", "ntt_core.h", "internal.h"],
           "ks_rotation": ["kernels.hip", "keyswitch.hip", "modarith.h", "ntt_core.h", "internal.h"]}


def sources_sha256(name: str) -> str:
    h = hashlib.sha256()
    for f in SOURCES[name]:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


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


def summarise_pmc(path: str, match: str | None = None) -> str:
    import re
    vals = defaultdict(lambda: defaultdict(list))
    meta = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = (row.get("Kernel_Name") or "?").split("(")[0].replace("void ", "")
            if match and not re.search(match, name):
                continue
            grid = row.get("Grid_Size") or row.get("Grid_Size_X") or "?"
            key = (name, grid)
            vals[key][row["Counter_Name"]].append(float(row["Counter_Value"]))
            meta[key] = (row.get("VGPR_Count", "?"), row.get("Accum_VGPR_Count", "?"), row.get("SGPR_Count", "?"),
                         row.get("LDS_Block_Size", "?"))
    counters = sorted({c for v in vals.values() for c in v})
    out = ["| kernel | grid (threads) | dispatches | vgpr/agpr/sgpr | lds | " + " | ".join(counters) + " |",
           "|---|---|---|---|---|" + "---|" * len(counters)]
    for key in sorted(vals):
        v = vals[key]
        n = max(len(x) for x in v.values())
        cells = [f"{sum(v[c]) / len(v[c]):.4g}" if v.get(c) else "" for c in counters]
        m = meta[key]
        out.append(f"| `{key[0]}` | {key[1]} | {n} | {m[0]}/{m[1]}/{m[2]} | {m[3]} | " + " | ".join(cells) + " |")
    return "\n".join(out)


def _per_dispatch(path: str, counter: str, match: str, grid: str | None = None) -> list:
    import re
    per = defaultdict(float)
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            name = (row.get("Kernel_Name") or "?").split("(")[0].replace("void ", "")
            if not re.search(match, name) or (grid is not None and row.get("Grid_Size") != grid):
                continue
            per[row["Dispatch_Id"]] += float(row["Counter_Value"])    # summed over instances
    return list(per.values())


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy: str, name: str | None = None) -> str:
    cname, cgrid, ckib = copy.rsplit(":", 2)
    out = []
    total = 0.0
    for path, ctr in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        cal = _per_dispatch(path, ctr, cname, cgrid)
        k = _per_dispatch(path, ctr, kernel)
        if not cal or not k:
            raise SystemExit(f"{ctr}: no dispatches of the copy or of the kernel")
        c_avg, k_avg = sum(cal) / len(cal), sum(k) / len(k)
        scale = float(ckib) / c_avg
        nbytes = k_avg * 1024.0 * scale
        total += nbytes
        out.append(f"{ctr}: copy {c_avg:.2f} KiB over {len(cal)} dispatches -> scale {scale:.5f}; "
                   f"kernel {k_avg:.2f} KiB over {len(k)} dispatches -> {nbytes:.0f} bytes")
    out.append(f"total bytes per dispatch: {total:.0f}")
    if name is not None:
        out.append(f"traffic_bytes_per_launch: {total:.0f} kernel: {name} sources_sha256: {sources_sha256(name)}")
    return "\n".join(out)


def valu_per_op(counters_csv: str, after: str, ops: int) -> str:
    """Kernels (by name and grid) dispatched a multiple of `ops` times after
    the marker are the op's own (each op launches the same sequence); any
    other dispatch (the process's tail) is listed and left out."""
    import re
    rows = []
    with open(counters_csv, newline="") as f:
        for row in csv.DictReader(f):
            name = (row.get("Kernel_Name") or "?").split("(")[0].replace("void ", "")
            if row.get("Grid_Size"):
                name += f" [{row['Grid_Size']}]"
            rows.append((int(row["Dispatch_Id"]), name, row["Counter_Name"], float(row["Counter_Value"])))
    marks = [d for d, n, _, _ in rows if re.search(after, n)]
    if not marks:
        raise SystemExit(f"no dispatch of {after}")
    last = max(marks)
    disp = defaultdict(set)
    inst = defaultdict(float)
    for d, n, c, v in rows:
        if d > last and c == "SQ_INSTS_VALU":
            disp[n].add(d)
            inst[n] += v
    out = ["| kernel | dispatches | VALU wave instr. per dispatch | per op |", "|---|---|---|---|"]
    per, left = 0.0, []
    for n in sorted(inst, key=lambda k: -inst[k]):
        k = len(disp[n])
        if k % ops:
            left.append(f"{n} x{k}")
            continue
        per += inst[n] / ops
        out.append(f"| `{n}` | {k} | {inst[n] / k:.4g} | {inst[n] / ops:.4g} |")
    out.append("")
    out.append(f"per op: {per:.6g} VALU wave instructions over {sum(len(disp[n]) for n in disp if len(disp[n]) % ops == 0) / ops:.0f} dispatches"
               + (f"; left out: {', '.join(left)}" if left else ""))
    out.append(f"valu_wave_instructions_per_rotation: {per:.6g} sources_sha256: {sources_sha256('ks_rotation')}")
    return "\n".join(out)


def per_run(path: str, runs: int, top: int = 20) -> str:
    ks = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = (row.get("Kernel_Name") or "?").split("(")[0].replace("void ", "").split("<")[0]
            ks.append((int(row["Start_Timestamp"]), int(row["End_Timestamp"]), name))
    ks.sort()
    gaps = [(ks[i + 1][0] - ks[i][1], i) for i in range(len(ks) - 1)]
    cut = max(gaps)[1] + 1 if gaps else 0
    ks = ks[cut:]
    span = (ks[-1][1] - ks[0][0]) / 1000.0
    busy = sum(e - s for s, e, _ in ks) / 1000.0
    groups = defaultdict(list)
    for s_, e, n in ks:
        groups[n].append((e - s_) / 1000.0)
    out = [f"{len(ks) / runs:.0f} launches per run; per run {span / runs:.1f} us span, "
           f"{busy / runs:.1f} us busy, {(span - busy) / runs:.1f} us idle between launches", "",
           "| kernel | launches per run | avg us | us per run | share |", "|---|---|---|---|---|"]
    for n, d in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append(f"| `{n}` | {len(d) / runs:.0f} | {sum(d) / len(d):.2f} | {sum(d) / runs:.1f} | "
                   f"{sum(d) / busy:.3f} |")
    return "\n".join(out)


VALU_PEAK = 256 * 4 * 2.4e9 / 4     # wave64 FP64 VALU instructions per second


def valu(counters_csv: str, trace_csv: str, top: int = 16) -> str:
    inst = defaultdict(lambda: defaultdict(float))     # (name, grid) -> dispatch -> SQ_INSTS_VALU
    busy = defaultdict(lambda: defaultdict(float))
    with open(counters_csv, newline="") as f:
        for row in csv.DictReader(f):
            name = (row.get("Kernel_Name") or "?").split("(")[0].replace("void ", "")
            key = (name, row.get("Grid_Size") or "?")
            if row["Counter_Name"] == "SQ_INSTS_VALU":
                inst[key][row["Dispatch_Id"]] += float(row["Counter_Value"])
            elif row["Counter_Name"] == "SQ_ACTIVE_INST_VALU":
                busy[key][row["Dispatch_Id"]] += float(row["Counter_Value"])
    dur = defaultdict(list)
    with open(trace_csv, newline="") as f:
        for row in csv.DictReader(f):
            name = (row.get("Kernel_Name") or "?").split("(")[0].replace("void ", "")
            grid = row.get("Grid_Size_X") or row.get("Grid_Size") or "?"
            wg = row.get("Workgroup_Size_X") or row.get("Workgroup_Size") or "1"
            # the counter csv's grid is in threads, the trace's in threads too
            dur[(name, grid)].append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1000.0)
    rows = []
    for key, d in inst.items():
        if key not in dur:
            continue
        n = sum(d.values()) / len(d)
        us = sum(dur[key]) / len(dur[key])
        rate = n / (us * 1e-6)
        rows.append((us * len(dur[key]), key, n, us, rate))
    rows.sort(reverse=True)
    out = ["| kernel | grid (threads) | VALU wave instr. per dispatch | avg us (trace) | G instr/s | of peak |",
           "|---|---|---|---|---|---|"]
    for _, (name, grid), n, us, rate in rows[:top]:
        out.append(f"| `{name}` | {grid} | {n:.4g} | {us:.2f} | {rate / 1e9:.1f} | {rate / VALU_PEAK:.3f} |")
    return "\n".join(out)


if __name__ == "__main__":
    if "--runs" in sys.argv:
        i = sys.argv.index("--runs")
        top = int(sys.argv[sys.argv.index("--top") + 1]) if "--top" in sys.argv else 20
        print(per_run(sys.argv[i + 2], int(sys.argv[i + 1]), top))
        sys.exit(0)
    if "--valu" in sys.argv:
        i = sys.argv.index("--valu")
        top = int(sys.argv[sys.argv.index("--top") + 1]) if "--top" in sys.argv else 16
        print(valu(sys.argv[i + 1], sys.argv[i + 2], top))
        sys.exit(0)
    if "--traffic" in sys.argv:
        i = sys.argv.index("--traffic")
        name = sys.argv[sys.argv.index("--name") + 1] if "--name" in sys.argv else None
        print(traffic(sys.argv[i + 1], sys.argv[i + 2], sys.argv[sys.argv.index("--kernel") + 1],
                      sys.argv[sys.argv.index("--copy") + 1], name))
        sys.exit(0)
    if "--valu-per-op" in sys.argv:
        i = sys.argv.index("--valu-per-op")
        print(valu_per_op(sys.argv[i + 1], sys.argv[sys.argv.index("--after") + 1],
                          int(sys.argv[sys.argv.index("--ops") + 1])))
        sys.exit(0)
    if "--pmc" in sys.argv:
        i = sys.argv.index("--pmc")
        m = sys.argv[sys.argv.index("--match") + 1] if "--match" in sys.argv else None
        print(summarise_pmc(sys.argv[i + 1], m))
        sys.exit(0)
    top = 25
    if "--top" in sys.argv:
        top = int(sys.argv[sys.argv.index("--top") + 1])
    print(summarise(sys.argv[1], top))
