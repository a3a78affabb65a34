"""Summaries of rocprofv3 output for the library's kernels (host tooling,
no GPU work): kernel durations from a kernel trace and per-dispatch hardware
counters, written as the short text summaries kept beside the results.

    python -m paper_2605_07612_amd.profiling trace RUN_kernel_trace.csv OUT.md \\
        --title "..." --command "rocprofv3 ..." [--match REGEX] [--top 16] [--window REGEX:FIRST:COUNT]
    python -m paper_2605_07612_amd.profiling counters OUT.json --kernel REGEX \\
        --csv FETCH_SIZE=RUN1_counter_collection.csv --csv WRITE_SIZE=RUN2_counter_collection.csv \\
        [--csv SQ_INSTS_VALU,SQ_WAVES=RUN3_counter_collection.csv] --command "..." \\
        [--calibrate KERNEL_REGEX:BYTES] [--source FILE ...] [--algorithmic-bytes N]

Counter values are per dispatch as rocprofv3 reports them (FETCH_SIZE and
WRITE_SIZE in KiB).  With --calibrate, FETCH_SIZE and WRITE_SIZE are scaled
by the factor that makes them read BYTES for the calibration kernel (a plain
device copy of known size), as the counters of different passes need not
count whole lines the same way.  --source records a SHA-256 of the kernel's
source files (their code without comments), so that a reader can tell whether
the counters still describe the code.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import re
import sys
from collections import OrderedDict


def _short(name: str) -> str:
    """Kernel name without its parameter list and return type."""
    n = name
    if n.startswith("void "):
        n = n[5:]
    depth = 0
    for k, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:k]
    return n


def read_trace(path):
    """Kernel dispatches of a rocprofv3 --kernel-trace CSV in start order:
    (name, grid threads, workgroup, duration in ns, start in ns)."""
    out = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            wg = int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"])
            t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            out.append((_short(r["Kernel_Name"]), grid, wg, t1 - t0, t0))
    out.sort(key=lambda x: x[4])
    return out


def window_table(rows, regex, first, count):
    """Launches first .. first + count - 1 (in start order) of every kernel
    whose name matches `regex`, e.g. the steps of a timed region that follow
    a known number of untimed ones: per kernel the mean duration, and the
    span from the window's first start to its last end per launch index."""
    rx = re.compile(regex)
    per = OrderedDict()
    for name, grid, wg, ns, t0 in rows:
        if rx.search(name):
            per.setdefault(name, []).append((t0, ns))
    stats, starts, ends = [], [], []
    for name, v in per.items():
        w = v[first:first + count]
        if not w:
            continue
        stats.append(dict(kernel=name, launches=len(w), avg_us=sum(ns for _, ns in w) / len(w) / 1e3))
        starts.append(w[0][0])
        ends.append(max(t0 + ns for t0, ns in w))
    span = (max(ends) - min(starts)) / count / 1e3 if stats else 0.0
    return stats, span


def trace_table(rows, match=None, top=16):
    """Per (kernel, grid) statistics, largest total first: the `top` largest
    and every other row whose name matches `match`."""
    groups = OrderedDict()
    for name, grid, wg, ns, _ in rows:
        groups.setdefault((name, grid, wg), []).append(ns)
    total = sum(r[3] for r in rows) or 1
    stats = []
    for (name, grid, wg), v in groups.items():
        stats.append(dict(kernel=name, grid=grid, workgroup=wg, calls=len(v), avg_us=sum(v) / len(v) / 1e3,
                          min_us=min(v) / 1e3, max_us=max(v) / 1e3, share=sum(v) / total))
    stats.sort(key=lambda s: -s["avg_us"] * s["calls"])
    keep = stats[:top]
    if match:
        rx = re.compile(match)
        keep += [s for s in stats[top:] if rx.search(s["kernel"])]
    return keep


def trace_markdown(stats, title, command, note="", window=None):
    lines = [f"# {title}", "", "Command (committed files only):", "", f"    {command}", ""]
    if note:
        lines += [note, ""]
    lines += ["| kernel | grid (threads) | workgroup | calls | average (us) | min (us) | max (us) | share of the run |",
              "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for s in stats:
        lines.append(f"| {s['kernel']} | {s['grid']} | {s['workgroup']} | {s['calls']} | {s['avg_us']:.1f} | "
                     f"{s['min_us']:.1f} | {s['max_us']:.1f} | {100 * s['share']:.1f} % |")
    if window:
        (wstats, span), (regex, first, count) = window
        lines += ["", f"Window: launches {first} .. {first + count - 1} of each kernel matching `{regex}`", "",
                  "| kernel | launches | average (us) |", "|---|---:|---:|"]
        for s in wstats:
            lines.append(f"| {s['kernel']} | {s['launches']} | {s['avg_us']:.1f} |")
        lines += ["", f"Sum of the means: {sum(s['avg_us'] for s in wstats):.1f} us; span from the window's first "
                      f"start to its last end: {span:.1f} us per launch index."]
    return "\n".join(lines) + "\n"


def read_counters(path):
    """{dispatch id: (short kernel name, grid threads, {counter: value})} of a
    rocprofv3 --pmc CSV."""
    out = OrderedDict()
    with open(path) as fh:
        for r in csv.DictReader(fh):
            d = int(r["Dispatch_Id"])
            if d not in out:
                out[d] = (_short(r["Kernel_Name"]), int(r["Grid_Size"]), {})
            out[d][2][r["Counter_Name"]] = out[d][2].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def counter_summary(csvs, kernel, calibrate=None):
    """Per matched kernel (short name, grid): the mean of each counter over
    its dispatches; FETCH_SIZE / WRITE_SIZE scaled by the calibration."""
    rx = re.compile(kernel)
    scale = {}
    per = OrderedDict()
    for names, path in csvs:
        disp = read_counters(path)
        if calibrate:
            crx, cbytes = calibrate
            for cname in names:
                if cname in ("FETCH_SIZE", "WRITE_SIZE"):
                    vals = [c[cname] for n, g, c in disp.values() if re.search(crx, n) and cname in c]
                    if vals:
                        kib = max(vals)  # the 1 GiB copy (the largest copy of the run)
                        scale[cname] = {"kib": kib, "bytes": cbytes, "scale": cbytes / 1024.0 / kib}
        for n, g, c in disp.values():
            if not rx.search(n):
                continue
            e = per.setdefault((n, g), {})
            for cname in names:
                if cname in c:
                    e.setdefault(cname, []).append(c[cname])
    out = []
    for (n, g), e in per.items():
        rec = {"kernel": n, "grid": g, "dispatches": max(len(v) for v in e.values())}
        for cname, v in e.items():
            mean = sum(v) / len(v)
            rec[cname] = round(mean, 3)
            if cname in scale:
                rec[cname + "_scaled"] = round(mean * scale[cname]["scale"], 3)
        out.append(rec)
    return out, scale


def code_text(src: str) -> str:
    """C/C++ source without comments and with whitespace runs collapsed: two
    sources that differ only in comments or layout give the same text.  One
    pass in source order, so a quote inside a comment starts nothing and a
    comment marker inside a string or character literal is kept."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c == "/" and src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif c == "/" and src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c and src[j] != "\n":
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def sources_sha256(paths):
    """SHA-256 over the code text (code_text) of the given source files, in
    order: it changes when the code changes, not when a comment does."""
    h = hashlib.sha256()
    for p in paths:
        with open(p, encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
        h.update(b"\0")
    return h.hexdigest()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("out")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--note", default="")
    t.add_argument("--match", default=None)
    t.add_argument("--top", type=int, default=16)
    t.add_argument("--window", default=None, help="KERNEL_REGEX:FIRST:COUNT")
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("--kernel", required=True)
    c.add_argument("--csv", action="append", required=True, help="NAME[,NAME..]=counter_collection.csv")
    c.add_argument("--command", action="append", default=[])
    c.add_argument("--calibrate", default=None, help="KERNEL_REGEX:BYTES")
    c.add_argument("--source", action="append", default=[])
    c.add_argument("--describe", default="")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        rows = read_trace(a.csv)
        stats = trace_table(rows, a.match, a.top)
        window = None
        if a.window:
            regex, first, count = a.window.rsplit(":", 2)
            window = (window_table(rows, regex, int(first), int(count)), (regex, int(first), int(count)))
        with open(a.out, "w") as fh:
            fh.write(trace_markdown(stats, a.title, a.command, a.note, window))
        return 0
    csvs = []
    for spec in a.csv:
        names, path = spec.split("=", 1)
        csvs.append((names.split(","), path))
    cal = None
    if a.calibrate:
        rx, b = a.calibrate.rsplit(":", 1)
        cal = (rx, int(b))
    recs, scale = counter_summary(csvs, a.kernel, cal)
    doc = {"kernels": a.describe, "commands": a.command, "calibration": scale, "dispatch_means": recs}
    if a.source:
        doc["source_files"] = a.source
        doc["source_sha256"] = sources_sha256(a.source)
    with open(a.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
