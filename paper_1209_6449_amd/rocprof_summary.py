"""Summaries of rocprofv3 runs for the profiles/ directory.

    # a device copy of known size, to calibrate FETCH_SIZE / WRITE_SIZE
    python -m paper_1209_6449_amd.rocprof_summary calibrate --bytes 1073741824
    # kernel statistics of a --kernel-trace --stats run
    python -m paper_1209_6449_amd.rocprof_summary stats DIR --command "..." --out FILE
    # HBM traffic per dispatch of a kernel from two --pmc runs (FETCH_SIZE,
    # WRITE_SIZE), scaled by the same counters on the calibration copy
    # shader-sequencer counters per 1 KiB of text of each scan dispatch
    python -m paper_1209_6449_amd.rocprof_summary sq DIR --bytes-per-dispatch N --command "..." --out FILE
    # L2 read requests by size (what FETCH_SIZE's formula assumes about them)
    python -m paper_1209_6449_amd.rocprof_summary requests DIR --command "..." --out FILE
    python -m paper_1209_6449_amd.rocprof_summary traffic --fetch DIR --write DIR \
        --calib-fetch DIR --calib-write DIR --calib-bytes N --kernel scan_kernel \
        --workload sweep1g --command "..." --out-json FILE --out-txt FILE
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import re
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# what decides the traffic of a search: the kernels, the host's choice of
# tile and write strategy, and the packaged tune table
KERNEL_SOURCES = sorted(os.path.relpath(p, ROOT) for p in glob.glob(os.path.join(ROOT, "paper_1209_6449_amd", "csrc", "*"))
                        if p.endswith((".hip", ".h"))) + ["paper_1209_6449_amd/tuned/gfx950_256cu.json"]


def _code_only(text: str) -> str:
    """C++ source without comments and with whitespace collapsed, so that a
    documentation edit does not invalidate measured traffic (string
    literals holding comment markers are not expected in these files)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash() -> str:
    """Hash of the code the measured kernels are built from (comments and
    whitespace ignored in C++ sources) and of the tune table."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "r", encoding="utf-8") as f:
            text = f.read()
        h.update((_code_only(text) if rel.endswith((".hip", ".h")) else text).encode())
    return h.hexdigest()[:16]


def _find(directory: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    return hits[0]


def counter_per_dispatch(directory: str, counter: str, kernel_sub: str) -> list[float]:
    """Counter value of every dispatch whose kernel name contains kernel_sub."""
    rows = csv.DictReader(open(_find(directory, "counter_collection.csv")))
    vals = {}
    for r in rows:
        if r["Counter_Name"] != counter or kernel_sub not in r["Kernel_Name"]:
            continue
        d = r["Dispatch_Id"]
        vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
    return [vals[k] for k in sorted(vals, key=int)]


def cmd_calibrate(args):
    import torch
    n = args.bytes
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": n, "reps": args.reps}), flush=True)


def cmd_stats(args):
    rows = list(csv.DictReader(open(_find(args.dir, "kernel_stats.csv"))))
    lines = [f"# rocprofv3 kernel statistics", f"command: {args.command}", "",
             f"{'calls':>7} {'avg_us':>10} {'total_ms':>10} {'pct':>6}  kernel"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"]
        if len(name) > 110:
            name = name[:107] + "..."
        lines.append(f"{int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}  {name}")
    if args.kernel:
        names = args.kernel.split(",")
        per_unit = 0.0
        units = None
        lines.append("")
        for k in names:
            sel = [r for r in rows if k in r["Name"]]
            calls = sum(int(r["Calls"]) for r in sel)
            total = sum(float(r["TotalDurationNs"]) for r in sel)
            if units is None:
                units = calls  # the first kernel counts the units (one dispatch each)
            if calls:
                lines.append(f"all instances of {k}: {calls} calls, {total / 1e6:.3f} ms, "
                             f"average {total / calls / 1e3:.2f} us per dispatch")
                per_unit += total / max(units, 1)
        if len(names) > 1 and units:
            lines.append(f"per {names[0]} dispatch, {' + '.join(names)}: {per_unit / 1e3:.2f} us")
    text = "\n".join(lines) + "\n"
    with open(args.out, "w") as f:
        f.write(text)
    print(text)


def cmd_sq(args):
    """Shader-sequencer counters of each dispatch of a kernel, per 1 KiB of
    text (one wave's piece): the instruction mix that bounds a scan."""
    rows = list(csv.DictReader(open(_find(args.dir, "counter_collection.csv"))))
    disp = {}
    for r in rows:
        if args.kernel not in r["Kernel_Name"]:
            continue
        d = disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"],
                                                    "us": (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    labels = args.labels.split(",") if args.labels else []
    counters = sorted({k for d in disp.values() for k in d if k.startswith("SQ_")})
    pieces = args.bytes_per_dispatch / 1024
    lines = [f"# {args.title}", f"command: {args.command}",
             f"counts per 1 KiB of text ({pieces:.0f} pieces per dispatch); kernel duration under counters",
             "", f"{'search':>14} {'us':>9} " + " ".join(f"{c[3:]:>16}" for c in counters) + "  kernel"]
    per = args.per_label
    for i, (k, d) in enumerate(sorted(disp.items())[args.skip:]):
        lab = labels[i // per] if i // per < len(labels) else str(k)
        if args.last_only and (i % per) != per - 1:
            continue
        tmpl = d["name"].split("scan_kernel")[-1][:40] if "scan_kernel" in d["name"] else d["name"][:40]
        lines.append(f"{lab:>14} {d['us']:9.1f} " + " ".join(f"{d.get(c, 0) / pieces:16.1f}" for c in counters)
                     + f"  {tmpl}")
    text = "\n".join(lines) + "\n"
    with open(args.out, "w") as f:
        f.write(text)
    print(text)


def cmd_requests(args):
    """Read requests the L2 sends to memory, by size, for each dispatch of a
    kernel (from a run with TCC_EA0_RDREQ_sum, TCC_EA0_RDREQ_32B_sum,
    TCC_EA0_RDREQ_128B_sum and TCC_BUBBLE_sum)."""
    rows = list(csv.DictReader(open(_find(args.dir, "counter_collection.csv"))))
    disp = {}
    for r in rows:
        if args.kernel not in r["Kernel_Name"]:
            continue
        disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"]})[r["Counter_Name"]] = float(r["Counter_Value"])
    labels = args.labels.split(",") if args.labels else []
    items = sorted(disp.items())
    if labels:  # only the labelled dispatches, the first ones of the run
        items = items[:len(labels)]
    ratio = f" {'text / fetched':>15}" if args.text_bytes else ""
    lines = [f"# {args.title}", f"command: {args.command}", "",
             f"{'dispatch':>14} {'RDREQ':>12} {'RDREQ_128B':>12} {'RDREQ_32B':>10} {'BUBBLE':>8} "
             f"{'128B x 128 (MB)':>16} {'FETCH_SIZE formula (MB)':>24}{ratio}  kernel"]
    for i, (k, d) in enumerate(items):
        rq, r128 = d.get("TCC_EA0_RDREQ_sum", 0), d.get("TCC_EA0_RDREQ_128B_sum", 0)
        r32, bub = d.get("TCC_EA0_RDREQ_32B_sum", 0), d.get("TCC_BUBBLE_sum", 0)
        formula = (bub * 128 + (rq - bub - r32) * 64 + r32 * 32) / 1e6
        lab = labels[i] if labels else str(k)
        r = f" {args.text_bytes / max(r128 * 128, 1):15.2f}" if args.text_bytes else ""
        lines.append(f"{lab:>14} {rq:12.0f} {r128:12.0f} {r32:10.0f} {bub:8.0f} {r128 * 128 / 1e6:16.1f} "
                     f"{formula:24.1f}{r}  {d['name'][:50]}")
    text = "\n".join(lines) + "\n"
    with open(args.out, "w") as f:
        f.write(text)
    print(text)


def cmd_traffic(args):
    # calibration: what each counter reads for a copy of calib_bytes (KiB units)
    cf = counter_per_dispatch(args.calib_fetch, "FETCH_SIZE", args.calib_kernel)
    cw = counter_per_dispatch(args.calib_write, "WRITE_SIZE", args.calib_kernel)
    if not cf or not cw:
        raise SystemExit("calibration dispatches not found")
    fetch_factor = args.calib_bytes / (statistics.median(cf) * 1024.0)
    write_factor = args.calib_bytes / (statistics.median(cw) * 1024.0)
    # per unit: all dispatches of the listed kernels over the number of
    # dispatches of the first one (e.g. per scan: scan + expand + zero);
    # with --sum-means, the sum of each kernel's mean per dispatch (a unit
    # runs each listed kernel once, e.g. one batch replay)
    names = args.kernel.split(",")
    f_all, w_all, units = 0.0, 0.0, None
    for k in names:
        f = counter_per_dispatch(args.fetch, "FETCH_SIZE", k)
        w = counter_per_dispatch(args.write, "WRITE_SIZE", k)
        if len(f) != len(w):
            raise SystemExit(f"{k}: unequal dispatch counts ({len(f)} vs {len(w)})")
        if not f:
            raise SystemExit(f"no dispatches of {k}")
        if units is None:
            units = len(f)
        if args.sum_means:
            f_all += statistics.mean(f) * units
            w_all += statistics.mean(w) * units
        else:
            f_all += sum(f)
            w_all += sum(w)
    f = [f_all / units]
    w = [w_all / units]
    fetch_b = [x * 1024.0 * fetch_factor for x in f]
    write_b = [x * 1024.0 * write_factor for x in w]
    per = statistics.mean(a + b for a, b in zip(fetch_b, write_b))
    out = {
        "workload": args.workload,
        "kernel": args.kernel,
        "kernel_hash": kernel_hash(),
        "dispatches": units,
        "fetch_bytes_per_launch": round(statistics.mean(fetch_b)),
        "write_bytes_per_launch": round(statistics.mean(write_b)),
        "bytes_per_launch": round(per),
        "calibration": {"copy_bytes": args.calib_bytes, "fetch_factor": round(fetch_factor, 4),
                        "write_factor": round(write_factor, 4),
                        "copy_fetch_kib": statistics.median(cf), "copy_write_kib": statistics.median(cw)},
        "command": args.command,
    }
    with open(args.out_json, "w") as fh:
        json.dump(out, fh, indent=1)
    text = (f"# HBM traffic of {args.kernel} ({args.workload})\n"
            f"command: {args.command}\n\n"
            f"units (dispatches of {names[0]}): {units}\n"
            f"FETCH_SIZE mean per dispatch: {statistics.mean(f):.0f} KiB raw -> "
            f"{out['fetch_bytes_per_launch']} B after calibration\n"
            f"WRITE_SIZE mean per dispatch: {statistics.mean(w):.0f} KiB raw -> "
            f"{out['write_bytes_per_launch']} B after calibration\n"
            f"traffic per dispatch: {out['bytes_per_launch']} B\n"
            f"calibration: a {args.calib_bytes}-byte device copy reads FETCH_SIZE "
            f"{statistics.median(cf):.0f} KiB and WRITE_SIZE {statistics.median(cw):.0f} KiB "
            f"(factors {fetch_factor:.4f}, {write_factor:.4f})\n"
            f"kernel source hash: {out['kernel_hash']}\n")
    with open(args.out_txt, "w") as fh:
        fh.write(text)
    print(text)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("calibrate")
    c.add_argument("--bytes", type=int, default=1 << 30)
    c.add_argument("--reps", type=int, default=3)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--kernel", default="",
                   help="also aggregate the kernels whose names contain these (comma separated; "
                        "the first counts the units)")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--calib-bytes", type=int, default=1 << 30)
    t.add_argument("--calib-kernel", default="copy")
    t.add_argument("--kernel", default="scan_kernel,expand_kernel,zero_u64,tile_offsets_kernel",
                   help="comma-separated kernel names; the first counts the units")
    t.add_argument("--sum-means", action="store_true",
                   help="traffic per unit = sum over the kernels of their mean per dispatch")
    t.add_argument("--workload", default="sweep1g")
    t.add_argument("--command", required=True)
    t.add_argument("--out-json", required=True)
    t.add_argument("--out-txt", required=True)
    q = sub.add_parser("sq")
    q.add_argument("dir")
    q.add_argument("--kernel", default="scan_kernel")
    q.add_argument("--bytes-per-dispatch", type=int, required=True)
    q.add_argument("--labels", default="", help="comma-separated names of the searches, in dispatch order")
    q.add_argument("--per-label", type=int, default=1, help="dispatches per search (steps)")
    q.add_argument("--last-only", action="store_true", help="only the last dispatch of each search")
    q.add_argument("--skip", type=int, default=0, help="leave out the first SKIP dispatches (e.g. a sizing pass)")
    q.add_argument("--title", default="shader-sequencer counters")
    q.add_argument("--command", required=True)
    q.add_argument("--out", required=True)
    r = sub.add_parser("requests")
    r.add_argument("dir")
    r.add_argument("--kernel", default="")
    r.add_argument("--title", default="L2 read requests by size")
    r.add_argument("--labels", default="", help="comma-separated names of the first dispatches; only those are listed")
    r.add_argument("--text-bytes", type=int, default=0, help="bytes of text each dispatch scans (adds text / fetched)")
    r.add_argument("--command", required=True)
    r.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    {"calibrate": cmd_calibrate, "stats": cmd_stats, "traffic": cmd_traffic, "sq": cmd_sq,
     "requests": cmd_requests}[args.cmd](args)


if __name__ == "__main__":
    main(sys.argv[1:])
