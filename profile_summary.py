"""Summarise rocprofv3 CSV output of bench.py runs as short text.

    python profile_summary.py trace <dir>               # --kernel-trace --stats run
    python profile_summary.py counters <dir> <counter>  # --pmc run (FETCH_SIZE / WRITE_SIZE)
    python profile_summary.py traffic <fetch_dir> <write_dir> <workload> <precision>
    python profile_summary.py pmc <dir> [<dir> ...]           # --pmc runs, any counters

`trace` groups dispatches by kernel and grid (so the levels of one kernel are told
apart) and reports count and average / min / max duration in microseconds.
`counters` reports the counter per dispatch group in KiB, and the ratio of that
counter to the known bytes of the copy probe (a 256 MiB device-to-device tensor copy
that `bench.py --copy-probe` runs), which calibrates bytes per counter unit.
`pmc` merges --pmc runs of the same command (one counter group each) per dispatch group
and prints, for the groups with the most wave cycles, the per-launch averages and
ratios: L2 (TCC) hit rate; bytes the L2 read from and wrote to memory from its request
counters (32-, 64- and 128-byte read requests, 32- and 64-byte write requests); VALU,
vector-memory and LDS instructions per wave; waiting and LDS bank-conflict cycles
against wave cycles.
`traffic` combines a FETCH_SIZE run and a WRITE_SIZE run of `bench.py --copy-probe`
into HBM bytes per launch of the last-level forward and adjoint sweep kernels (the
largest dispatch group of each), prints the summary and records it in
profiles/traffic.json under the current kernel-source digest, where bench.py reads it.
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


def _counter_groups(d: str, counter: str):
    path = _find(d, "counter_collection.csv")
    groups = defaultdict(list)
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            groups[(short_name(row["Kernel_Name"]), row.get("Grid_Size", "?"))].append(float(row["Counter_Value"]))
    return path, {k: sum(v) / len(v) for k, v in groups.items()}, {k: len(v) for k, v in groups.items()}


def traffic(fetch_dir: str, write_dir: str, workload: str, precision: str):
    import json
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from bench import PROFILES, kernel_source_digest
    from workloads import WORKLOADS
    wl = WORKLOADS[workload]
    n = [int(v) for v in wl["shape0"]]
    shapes = [n]
    for _ in range(wl["depth"]):
        n = [2 * (v - 2) for v in n]
        shapes.append(n)
    el = {"f32": 4, "bf16": 2}[precision]
    prod = lambda v: int(__import__("math").prod(v))
    # algorithmic bytes of one launch: the fine level read and written; the coarse level
    # (read by the forward, written by the adjoint) apart
    alg = wl.get("batch", 1) * 2 * prod(shapes[-1]) * el
    coarse = wl.get("batch", 1) * prod(shapes[-2]) * el
    _, fetch, _ = _counter_groups(fetch_dir, "FETCH_SIZE")
    _, write, calls = _counter_groups(write_dir, "WRITE_SIZE")
    f_probe = max(v for (nm, g), v in fetch.items() if "copy" in nm.lower())
    w_probe = max(v for (nm, g), v in write.items() if "copy" in nm.lower())
    f_scale = COPY_PROBE_BYTES / f_probe          # bytes read per reported unit
    w_scale = COPY_PROBE_BYTES / w_probe          # bytes written per reported unit
    digest = kernel_source_digest()
    path = os.path.join(PROFILES, "traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    print(f"# kernel sources digest: {digest}")
    print(f"# Calibration: the 256 MiB copy probe reads {f_probe:.0f} (FETCH_SIZE) for {COPY_PROBE_BYTES} bytes "
          f"read (factor {f_scale / 1024:.3f}) and {w_probe:.0f} (WRITE_SIZE) for {COPY_PROBE_BYTES} bytes written "
          f"(factor {w_scale / 1024:.3f}); the kernels' counters are scaled by these factors.")
    for tag, kname in (("refine_adj_last", "refine3_adj_sector"), ("refine_fwd_last", "refine3_fwd_sector")):
        cands = [(v, k) for k, v in fetch.items() if k[0].startswith(kname) and k in write]
        if not cands:
            continue
        _, key = max(cands)
        rd, wr = fetch[key] * f_scale, write[key] * w_scale
        print(f"{tag:16s} {key[0]} grid {key[1]:>8s} ({calls[key]} launches): FETCH {fetch[key]:9.0f} KiB -> "
              f"{rd / 1e6:6.1f} MB read; WRITE {write[key]:9.0f} KiB -> {wr / 1e6:6.1f} MB written; total "
              f"{(rd + wr) / 1e6:6.1f} MB vs algorithmic {alg / 1e6:.1f} MB ({(rd + wr) / alg:.2f}x; "
              f"{(rd + wr) / (alg + coarse):.2f}x of {(alg + coarse) / 1e6:.1f} MB with the coarse level)")
        rec[f"{tag}:{workload}:{precision}"] = {"source_digest": digest, "hbm_bytes_per_launch": rd + wr,
                                               "read_bytes": rd, "write_bytes": wr, "alg_bytes": alg,
                                               "coarse_bytes": coarse}
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


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


def pmc(dirs):
    vals = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        with open(_find(d, "counter_collection.csv")) as f:
            for row in csv.DictReader(f):
                key = (short_name(row["Kernel_Name"]), row.get("Grid_Size", "?"))
                vals[key][row["Counter_Name"]].append(float(row["Counter_Value"]))
    avg = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in vals.items()}
    calls = {k: max(len(v) for v in cs.values()) for k, cs in vals.items()}
    order = sorted(avg, key=lambda k: -avg[k].get("SQ_WAVE_CYCLES", 0.0) * calls[k])
    print(f"# sources: {', '.join(dirs)}; per-launch averages of each dispatch group")
    for key in order[:12]:
        c = avg[key]
        g = lambda n: c.get(n, c.get(n + "_sum"))
        parts = [f"{key[0]} grid {key[1]} ({calls[key]} launches)"]
        hit, miss = g("TCC_HIT"), g("TCC_MISS")
        if hit is not None and miss is not None and hit + miss > 0:
            parts.append(f"L2 hit {hit / (hit + miss):.3f}")
        rd, rd32, rd128 = g("TCC_EA0_RDREQ"), g("TCC_EA0_RDREQ_32B"), g("TCC_EA0_RDREQ_128B")
        if rd is not None and rd32 is not None and rd128 is not None:
            parts.append(f"read {(32 * rd32 + 128 * rd128 + 64 * (rd - rd32 - rd128)) / 1e6:.1f} MB "
                         f"({rd128 / max(rd, 1):.2f} of requests 128 B)")
        wr, wr64 = g("TCC_EA0_WRREQ"), g("TCC_EA0_WRREQ_64B")
        if wr is not None and wr64 is not None:
            parts.append(f"written {(64 * wr64 + 32 * (wr - wr64)) / 1e6:.1f} MB")
        waves = g("SQ_WAVES")
        if waves:
            for n, label in (("SQ_INSTS_VALU", "VALU"), ("SQ_INSTS_VMEM", "VMEM"), ("SQ_INSTS_LDS", "LDS"),
                             ("SQ_INSTS_SALU", "SALU")):
                if g(n) is not None:
                    parts.append(f"{label}/wave {g(n) / waves:.0f}")
        cyc = g("SQ_WAVE_CYCLES")
        if cyc:
            if g("SQ_WAIT_INST_ANY") is not None:
                parts.append(f"waiting {g('SQ_WAIT_INST_ANY') / cyc:.2f} of wave cycles")
            if g("SQ_ACTIVE_INST_VALU") is not None:
                parts.append(f"VALU issue {g('SQ_ACTIVE_INST_VALU') / cyc:.3f} of wave cycles")
        if g("SQ_LDS_BANK_CONFLICT") is not None and g("SQ_INSTS_LDS"):
            parts.append(f"LDS bank-conflict cycles/LDS instruction {g('SQ_LDS_BANK_CONFLICT') / g('SQ_INSTS_LDS'):.2f}")
        print("; ".join(parts))


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "trace":
        trace(sys.argv[2])
    elif len(sys.argv) >= 4 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3])
    elif len(sys.argv) >= 3 and sys.argv[1] == "pmc":
        pmc(sys.argv[2:])
    elif len(sys.argv) >= 6 and sys.argv[1] == "traffic":
        traffic(*sys.argv[2:6])
    else:
        raise SystemExit(__doc__)
