"""Short text summaries of rocprofv3 output, and the HBM traffic of one kernel from counters.

  python -m paper_1711_03836_amd.profile_summary stats DIR OUT.txt --command "..."
  python -m paper_1711_03836_amd.profile_summary traffic FETCH_DIR WRITE_DIR OUT.json --kernel k_hop \
      --launches 3 --copy-mib 1024 --command-fetch "..." --command-write "..."

`stats` turns the kernel statistics CSV of a `rocprofv3 --kernel-trace --stats --output-format csv`
run into a table (calls, total, average per kernel).

`kernels` reads the same two passes over a whole run (e.g. one solve) and tabulates the calibrated
traffic per kernel name.

`traffic` reads two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of kernel_bench (each with a
plain device copy of --copy-mib MiB before the timed launches), takes the last --launches dispatches
of the kernel whose name contains --kernel, and scales each counter by (known bytes of the copy) /
(what the counter read for the copy).  FETCH_SIZE and WRITE_SIZE are in KiB per dispatch.  The JSON
carries the digest of the stencil kernel sources it was taken on; a later change to them makes
it stale.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))


# the sources that define the stencil kernels (host-side library code does not change them)
KERNEL_SOURCES = ("bq_device.h", "bq_kernels.h", "bq_dslash_impl.h", "bq_dslash_inst.hip")


def source_digest():
    """sha256 over the stencil kernel sources (names and contents)."""
    h = hashlib.sha256()
    csrc = os.path.join(PKG, "csrc")
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _one(pattern):
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise SystemExit(f"no file matches {pattern}")
    return hits[0]


def stats(args):
    path = _one(os.path.join(args.dir, "**", "*kernel_stats.csv"))
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics: {args.title}", "", "command:", "", "    " + args.command, "",
             f"total kernel time {total / 1e6:.3f} ms over {sum(int(r['Calls']) for r in rows)} dispatches", "",
             f"{'calls':>7} {'total ms':>10} {'avg us':>10} {'min us':>10} {'max us':>10} {'%':>6}  kernel"]
    for r in rows[:args.top]:
        name = r["Name"]
        if len(name) > args.width:
            name = name[:args.width] + "..."
        lines.append(f"{int(r['Calls']):7d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:10.2f} "
                     f"{float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f}  {name}")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_rows(d, counter):
    path = _one(os.path.join(d, "**", "*counter_collection.csv"))
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    out.sort()
    return out


def _reading(d, counter, kernel, launches, copy_bytes):
    rows = _counter_rows(d, counter)
    copies = [v for (_, name, grid, v) in rows if "copyBuffer" in name and v > 0.25 * copy_bytes / 1024]
    if not copies:
        raise SystemExit(f"{counter}: no calibration copy found in {d}")
    cal = (copy_bytes / 1024) / (sum(copies) / len(copies))
    mine = [(name, v) for (_, name, _, v) in rows if kernel in name][-launches:]
    if len(mine) < launches:
        raise SystemExit(f"{counter}: {len(mine)} dispatches of {kernel} in {d}, expected {launches}")
    kib = sum(v for _, v in mine) / len(mine)
    return {"kib_per_dispatch": kib, "copy_kib_read": sum(copies) / len(copies), "factor": cal,
            "bytes_per_dispatch": kib * 1024 * cal, "kernel_name": mine[-1][0]}


def traffic(args):
    copy_bytes = args.copy_mib * (1 << 20)
    fetch = _reading(args.fetch_dir, "FETCH_SIZE", args.kernel, args.launches, copy_bytes)
    write = _reading(args.write_dir, "WRITE_SIZE", args.kernel, args.launches, copy_bytes)
    out = {"kernel": fetch["kernel_name"], "fetch": fetch, "write": write,
           "traffic_bytes": fetch["bytes_per_dispatch"] + write["bytes_per_dispatch"],
           "copy_bytes": copy_bytes, "source_digest": source_digest(),
           "tune": [int(v) for v in args.tune.split(",")] if args.tune else None,
           "workload": args.workload, "command_fetch": args.command_fetch, "command_write": args.command_write}
    if args.algorithmic_bytes:
        out["algorithmic_bytes"] = args.algorithmic_bytes
        out["ratio_to_algorithmic"] = out["traffic_bytes"] / args.algorithmic_bytes
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


def kernels(args):
    """Per-kernel HBM traffic over every dispatch of a run (e.g. one solve): FETCH_SIZE and WRITE_SIZE
    summed per kernel name, each scaled by its copy calibration, as a text table."""
    copy_bytes = args.copy_mib * (1 << 20)
    per = {}
    for counter, d in (("FETCH_SIZE", args.fetch_dir), ("WRITE_SIZE", args.write_dir)):
        rows = _counter_rows(d, counter)
        copies = [v for (_, name, _, v) in rows if "copyBuffer" in name and v > 0.25 * copy_bytes / 1024]
        if not copies:
            raise SystemExit(f"{counter}: no calibration copy found in {d}")
        cal = (copy_bytes / 1024) / (sum(copies) / len(copies))
        for _, name, _, v in rows:
            if "copyBuffer" in name or "fillBuffer" in name:
                continue
            e = per.setdefault(name, {"FETCH_SIZE": [0, 0.0], "WRITE_SIZE": [0, 0.0]})
            e[counter][0] += 1
            e[counter][1] += v * 1024 * cal
    total = sum(e["FETCH_SIZE"][1] + e["WRITE_SIZE"][1] for e in per.values())
    lines = [f"# HBM traffic per kernel (copy-calibrated FETCH_SIZE + WRITE_SIZE): {args.title}", "",
             "FETCH_SIZE pass:", "", "    " + args.command_fetch, "", "WRITE_SIZE pass:", "", "    " + args.command_write, "",
             f"total {total / 1e9:.2f} GB over the run; stencil-kernel source digest {source_digest()}", "",
             f"{'calls':>6} {'fetch GB':>9} {'write GB':>9} {'GB/call':>8} {'%':>6}  kernel"]
    for name, e in sorted(per.items(), key=lambda kv: -(kv[1]["FETCH_SIZE"][1] + kv[1]["WRITE_SIZE"][1])):
        n = max(e["FETCH_SIZE"][0], 1)
        t = e["FETCH_SIZE"][1] + e["WRITE_SIZE"][1]
        if t < args.min_fraction * total:
            continue
        short = name if len(name) <= args.width else name[:args.width] + "..."
        lines.append(f"{n:6d} {e['FETCH_SIZE'][1] / 1e9:9.2f} {e['WRITE_SIZE'][1] / 1e9:9.2f} {t / n / 1e9:8.3f} "
                     f"{100 * t / total:6.2f}  {short}")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--top", type=int, default=25)
    s.add_argument("--width", type=int, default=110)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("out")
    t.add_argument("--kernel", default="k_hop")
    t.add_argument("--launches", type=int, default=3)
    t.add_argument("--copy-mib", type=int, default=1024)
    t.add_argument("--tune", default="")
    t.add_argument("--workload", default="")
    t.add_argument("--algorithmic-bytes", type=float, default=0.0)
    t.add_argument("--command-fetch", default="")
    t.add_argument("--command-write", default="")
    k = sub.add_parser("kernels")
    k.add_argument("fetch_dir")
    k.add_argument("write_dir")
    k.add_argument("out")
    k.add_argument("--copy-mib", type=int, default=1024)
    k.add_argument("--title", default="")
    k.add_argument("--min-fraction", type=float, default=0.002)
    k.add_argument("--width", type=int, default=110)
    k.add_argument("--command-fetch", default="")
    k.add_argument("--command-write", default="")
    args = ap.parse_args(argv)
    {"stats": stats, "traffic": traffic, "kernels": kernels}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
