"""Summaries of rocprofv3 output for this library's kernels.

    python -m paper_2005_05371_amd.profiling stats DIR [--match SUBSTR]
    python -m paper_2005_05371_amd.profiling traffic --fetch DIR --write DIR --kernel-match SUBSTR
        --name NAME --workload WORKLOAD --copy-mib N [--out FILE]
    python -m paper_2005_05371_amd.profiling valu --dir DIR --kernel-match SUBSTR --name NAME
        --workload WORKLOAD [--out FILE]

`stats` prints the kernel-trace statistics (`*_kernel_stats.csv`) as a markdown table.

`traffic` turns two counter runs of the same command (one with `--pmc FETCH_SIZE`, one with
`--pmc WRITE_SIZE`; both counters in KiB per dispatch) into HBM bytes per launch of the
matching kernel. Each counter is scaled by what it reads for a plain elementwise kernel of
known traffic that the command also ran (`bench.py --copy-calib N`: a bitwise not over N
MiB, N MiB read and N MiB written per pass): scale = N MiB / counter value of that pass.
The record, tagged with a hash of the kernel sources, is written into FILE (one HTML
comment line per kernel and workload, plus a table row); the benchmark reports it only
while the sources still hash the same.

`valu` turns one counter run (`--pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS`)
into the medians per dispatch of the matching kernel, stored the same way; the benchmark
derives the VALU busy fraction from them and its own measured duration (a wave64
instruction holds a 16-lane SIMD for 4 cycles).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
from typing import Dict, List, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.md")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_counters.md")
KERNEL_SOURCES = ["amf.hip", "tile_io.h", "hd_internal.h", "wiener.hip"]
COPY_KERNEL = "bitwise_not"


def code_text(src: str) -> str:
    """C++ source with comments removed and runs of whitespace folded to one space, so
    that an edit of a comment or of the layout leaves the hash of the code alone.
    String and character literals are kept as written."""
    out = []
    i, n = 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Short hash of the code (comments and layout aside) of the stage kernels' sources."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, path: str = TRAFFIC_FILE) -> Optional[Dict]:
    """The traffic record for (kernel, workload), or None when there is none or the kernel
    sources changed since the counters were taken."""
    return _measured("traffic", kernel, workload, path)


def measured_valu(kernel: str, workload: str, path: str = VALU_FILE) -> Optional[Dict]:
    """The instruction-count record for (kernel, workload), guarded like the traffic."""
    return _measured("valu", kernel, workload, path)


def _measured(kind: str, kernel: str, workload: str, path: str) -> Optional[Dict]:
    if not os.path.exists(path):
        return None
    want = kernel_source_hash()
    found = None
    tag = f"<!-- {kind} "
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line.startswith(tag):
                continue
            rec = json.loads(line[len(tag):-len(" -->")])
            if rec["kernel"] == kernel and rec["workload"] == workload and rec["source_sha256"] == want:
                found = rec
    return found


def _csv(dirname: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(dirname, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {dirname}")
    return hits[0]


def counter_per_dispatch(dirname: str, counter: str) -> Dict[str, List[float]]:
    """Kernel name -> per-dispatch values of `counter` (summed over the rows of a dispatch)."""
    per: Dict[tuple, float] = {}
    names: Dict[tuple, str] = {}
    with open(_csv(dirname, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            key = (r.get("Dispatch_Id"), r.get("Agent_Id"))
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
            names[key] = r["Kernel_Name"]
    out: Dict[str, List[float]] = {}
    for k, v in per.items():
        out.setdefault(names[k], []).append(v)
    return out


def _pick(per: Dict[str, List[float]], match: str) -> List[float]:
    vals = [v for name, vs in per.items() if match in name for v in vs]
    if not vals:
        raise KeyError(f"no dispatch of a kernel matching {match!r}")
    return vals


def counters_table(dirname: str, match: str = "") -> str:
    """Markdown table of a counter run: one row per (kernel, workgroups per dispatch), the
    dispatch count, the median kernel time (under counter collection, so an upper bound)
    and every counter's median per dispatch; the per-wave SQ counters (instructions, waits,
    cycles) divided by SQ_WAVES when that was collected."""
    per: Dict[tuple, Dict[str, float]] = {}
    info: Dict[tuple, tuple] = {}
    with open(_csv(dirname, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if match not in r["Kernel_Name"]:
                continue
            key = (r.get("Dispatch_Id"), r.get("Agent_Id"))
            d = per.setdefault(key, {})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            groups = int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"]))
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0
            info[key] = (r["Kernel_Name"], groups, us)
    rows: Dict[tuple, List[tuple]] = {}
    for key, d in per.items():
        name, groups, us = info[key]
        rows.setdefault((name, groups), []).append((us, d))
    names = sorted({c for d in per.values() for c in d})
    waves = "SQ_WAVES" in names

    def per_wave(c: str) -> bool:
        return waves and c.startswith("SQ_") and c not in ("SQ_WAVES", "SQ_BUSY_CYCLES")

    head = ["kernel", "workgroups", "dispatches", "median us"] + \
           [c + (" / wave" if per_wave(c) else "") for c in names]
    out = ["| " + " | ".join(head) + " |", "|" + "---|" * len(head)]
    for (name, groups), items in sorted(rows.items(), key=lambda kv: -len(kv[1])):
        cells = [f"`{name[:80]}`", str(groups), str(len(items)),
                 f"{statistics.median(u for u, _ in items):.1f}"]
        for c in names:
            vals = [d.get(c, 0.0) / d["SQ_WAVES"] if per_wave(c) and d.get("SQ_WAVES") else d.get(c, 0.0)
                    for _, d in items]
            v = statistics.median(vals)
            cells.append(f"{v:.0f}" if v >= 100 else f"{v:.2f}")
        out.append("| " + " | ".join(cells) + " |")
    return "\n".join(out)


def traffic(fetch_dir: str, write_dir: str, kernel_match: str, copy_mib: int) -> Dict:
    fetch = counter_per_dispatch(fetch_dir, "FETCH_SIZE")
    write = counter_per_dispatch(write_dir, "WRITE_SIZE")
    copy_bytes = float(copy_mib) * (1 << 20)
    cf = statistics.median(_pick(fetch, COPY_KERNEL)) * 1024.0
    cw = statistics.median(_pick(write, COPY_KERNEL)) * 1024.0
    sf, sw = copy_bytes / cf, copy_bytes / cw
    kf = statistics.median(_pick(fetch, kernel_match)) * 1024.0
    kw = statistics.median(_pick(write, kernel_match)) * 1024.0
    return {"fetch_bytes": round(kf * sf), "write_bytes": round(kw * sw),
            "copy_scale": [round(sf, 4), round(sw, 4)],
            "raw_kib": [round(kf / 1024.0, 1), round(kw / 1024.0, 1)],
            "copy_raw_kib": [round(cf / 1024.0, 1), round(cw / 1024.0, 1)],
            "dispatches": [len(_pick(fetch, kernel_match)), len(_pick(write, kernel_match))]}


def valu(dirname: str, kernel_match: str) -> Dict:
    """Medians per dispatch of the instruction counters of the matching kernel."""
    out = {}
    n = 0
    for counter, key in (("SQ_WAVES", "waves"), ("SQ_INSTS_VALU", "valu_insts"),
                         ("SQ_INSTS_SALU", "salu_insts"), ("SQ_INSTS_LDS", "lds_insts")):
        vals = _pick(counter_per_dispatch(dirname, counter), kernel_match)
        out[key] = round(statistics.median(vals))
        n = len(vals)
    out["dispatches"] = n
    return out


_HEADERS = {
    "traffic": ["# HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-kernel scaled)", "",
                "| kernel | workload | fetch bytes | write bytes | copy scale (fetch, write) | sources |",
                "|---|---|---|---|---|---|"],
    "valu": ["# Instruction counts per launch (rocprofv3 SQ_WAVES / SQ_INSTS_*, median over dispatches)", "",
             "| kernel | workload | waves | VALU | SALU | LDS | sources |",
             "|---|---|---|---|---|---|---|"],
}


def write_record(path: str, name: str, workload: str, rec: Dict, command: str, kind: str = "traffic") -> None:
    rec = dict(rec, kernel=name, workload=workload, source_sha256=kernel_source_hash())
    lines = open(path).read().splitlines() if os.path.exists(path) else list(_HEADERS[kind])
    keep = []
    for line in lines:
        if line.startswith(f"<!-- {kind} ") and f'"kernel": "{name}"' in line and f'"workload": "{workload}"' in line:
            continue
        if line.startswith(f"| {name} | {workload} |"):
            continue
        if line.startswith(f"<!-- command for {name} / {workload}:"):
            continue
        keep.append(line)
    if kind == "traffic":
        keep.append(f"| {name} | {workload} | {rec['fetch_bytes']} | {rec['write_bytes']} | "
                    f"{rec['copy_scale'][0]}, {rec['copy_scale'][1]} | {rec['source_sha256']} |")
    else:
        keep.append(f"| {name} | {workload} | {rec['waves']} | {rec['valu_insts']} | {rec['salu_insts']} | "
                    f"{rec['lds_insts']} | {rec['source_sha256']} |")
    keep.append(f"<!-- {kind} " + json.dumps(rec) + " -->")
    keep.append(f"<!-- command for {name} / {workload}: {command} -->")
    with open(path, "w") as f:
        f.write("\n".join(keep) + "\n")


def stats_table(dirname: str, match: str = "") -> str:
    rows = []
    with open(_csv(dirname, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            if match and match not in r["Name"]:
                continue
            rows.append(r)
    out = ["| kernel | calls | average us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        nm = r["Name"]
        nm = nm if len(nm) <= 90 else nm[:87] + "..."
        out.append(f"| `{nm}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['Percentage']):.1f} |")
    return "\n".join(out)


def grid_table(dirname: str, match: str = "") -> str:
    """Markdown table of a kernel trace split by launch size: one row per (kernel,
    workgroups per dispatch) with the dispatch count and the median / min / max duration,
    so that one workload's launches stand apart from other sizes of the same kernel."""
    groups: Dict[tuple, List[float]] = {}
    with open(_csv(dirname, "kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            if match and match not in r["Kernel_Name"]:
                continue
            wg = 1
            for d in "XYZ":
                wg *= -(-int(r.get(f"Grid_Size_{d}") or 1) // max(1, int(r.get(f"Workgroup_Size_{d}") or 1)))
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0
            groups.setdefault((r["Kernel_Name"], wg), []).append(us)
    out = ["| kernel | workgroups | dispatches | median us | min us | max us |", "|---|---|---|---|---|---|"]
    for (name, wg), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        nm = name if len(name) <= 80 else name[:77] + "..."
        out.append(f"| `{nm}` | {wg} | {len(v)} | {statistics.median(v):.1f} | {min(v):.1f} | {max(v):.1f} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2005_05371_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s1 = sub.add_parser("stats")
    s1.add_argument("dir")
    s1.add_argument("--match", default="")
    s5 = sub.add_parser("grid")
    s5.add_argument("dir")
    s5.add_argument("--match", default="")
    s4 = sub.add_parser("counters")
    s4.add_argument("dir")
    s4.add_argument("--match", default="")
    s2 = sub.add_parser("traffic")
    s2.add_argument("--fetch", required=True)
    s2.add_argument("--write", required=True)
    s2.add_argument("--kernel-match", required=True)
    s2.add_argument("--name", required=True)
    s2.add_argument("--workload", required=True)
    s2.add_argument("--copy-mib", type=int, required=True)
    s2.add_argument("--command", default="")
    s2.add_argument("--out", default=TRAFFIC_FILE)
    s3 = sub.add_parser("valu")
    s3.add_argument("--dir", required=True)
    s3.add_argument("--kernel-match", required=True)
    s3.add_argument("--name", required=True)
    s3.add_argument("--workload", required=True)
    s3.add_argument("--command", default="")
    s3.add_argument("--out", default=VALU_FILE)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_table(a.dir, a.match))
    elif a.cmd == "grid":
        print(grid_table(a.dir, a.match))
    elif a.cmd == "counters":
        print(counters_table(a.dir, a.match))
    elif a.cmd == "valu":
        rec = valu(a.dir, a.kernel_match)
        write_record(a.out, a.name, a.workload, rec, a.command, kind="valu")
        print(json.dumps(rec))
    else:
        rec = traffic(a.fetch, a.write, a.kernel_match, a.copy_mib)
        write_record(a.out, a.name, a.workload, rec, a.command)
        print(json.dumps(rec))


if __name__ == "__main__":
    main()
