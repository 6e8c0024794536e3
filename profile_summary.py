"""Summarise rocprofv3 CSV output of bench.py runs as short text.

    python profile_summary.py trace <dir>               # --kernel-trace --stats run
    python profile_summary.py counters <dir> <counter>  # --pmc run (FETCH_SIZE / WRITE_SIZE)

`trace` groups dispatches by kernel and grid (so the levels of one kernel are told
apart) and reports count and average / min / max duration in microseconds.
`counters` reports the counter per dispatch group in KiB, and the ratio of that
counter to the known bytes of the copy probe (a 256 MiB device-to-device tensor copy
that `bench.py --copy-probe` runs), which calibrates bytes per counter unit.
"""

from __future__ import annotations

import csv
import glob
import os
import re
import sys
from collections import defaultdict

COPY_PROBE_BYTES = 256 * 1024 * 1024


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[-1]


def short_name(name: str) -> str:
    name = name.strip().replace("(anonymous namespace)::", "").replace("icr::", "")
    name = re.sub(r"^void\s+", "", name)
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):       # drop the argument list: the first top-level '('
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    return name[:cut]


def _grid(row) -> str:
    g = [row.get(k) for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z")]
    if all(v is not None for v in g):
        return "x".join(g)
    return row.get("Grid_Size", "?")


def trace(d: str):
    path = _find(d, "kernel_trace.csv")
    groups = defaultdict(list)
    with open(path) as f:
        for row in csv.DictReader(f):
            dur = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3
            groups[(short_name(row["Kernel_Name"]), _grid(row))].append(dur)
    print(f"# source: {os.path.basename(path)}; durations in microseconds")
    print(f"{'kernel':70s} {'grid':>18s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s}")
    for (name, grid), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        print(f"{name[:70]:70s} {grid:>18s} {len(v):6d} {sum(v) / len(v):10.2f} {min(v):10.2f} {max(v):10.2f}")


def counters(d: str, counter: str):
    path = _find(d, "counter_collection.csv")
    groups = defaultdict(list)
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            grid = row.get("Grid_Size", "?")
            groups[(short_name(row["Kernel_Name"]), grid)].append(float(row["Counter_Value"]))
    probe = [sum(v) / len(v) for (n, g), v in groups.items() if "copy" in n.lower()]
    print(f"# source: {os.path.basename(path)}; {counter} per dispatch (KiB as reported)")
    if probe:
        kib = max(probe)
        print(f"# copy probe: {kib:.0f} KiB for {COPY_PROBE_BYTES} B read + {COPY_PROBE_BYTES} B written "
              f"-> {COPY_PROBE_BYTES / (kib * 1024):.4f} bytes moved per reported byte (one direction)")
    print(f"{'kernel':70s} {'grid':>12s} {'calls':>6s} {'avg_KiB':>14s}")
    for (name, grid), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        print(f"{name[:70]:70s} {grid:>12s} {len(v):6d} {sum(v) / len(v):14.1f}")


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "trace":
        trace(sys.argv[2])
    elif len(sys.argv) >= 4 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3])
    else:
        raise SystemExit(__doc__)
