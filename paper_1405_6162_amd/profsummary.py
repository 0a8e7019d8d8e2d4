"""Summarise rocprofv3 CSV output into a short text profile.

    python -m paper_1405_6162_amd.profsummary stats  <kernel_stats.csv> [--title T] [--command C]
    python -m paper_1405_6162_amd.profsummary pmc    <fetch counter_collection.csv> <write counter_collection.csv>
                                                     --kernel SUBSTRING[,SUBSTRING...] [--copy-bytes B] [--title T] [--command C]

`stats` prints the per-kernel call count and average / min / max duration
from a `rocprofv3 --kernel-trace --stats --output-format csv` run.

`pmc` prints FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the kernels
whose name contains SUBSTRING, and scales each by what the same counter
reads for the largest dispatch of the library's streaming copy
(`k_stream_copy`, which moves `copy-bytes` in each direction), giving HBM
bytes per launch.
The last lines are `key: value` pairs that bench.py reads.
"""

import argparse
import csv
import hashlib
import os
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))


def _code_only(text):
    """The source with its comments and blank space removed: // comments to
    the end of the line (outside string literals), /* */ blocks, and runs of
    whitespace collapsed, so that editing a comment changes no digest."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"':                                   # string literal: copy through its end
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_digest():
    """sha256 of the kernel sources' code (comments and whitespace removed);
    a counter summary is stale once it changes."""
    h = hashlib.sha256()
    for name in ("d3q19.h", "kernels.h", "lb_api.hip"):
        with open(os.path.join(PKG, "csrc", name), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def short(name, width=90):
    return name if len(name) <= width else name[:width - 3] + "..."


def cmd_stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    print("# %s" % (args.title or "rocprofv3 kernel statistics"))
    if args.command:
        for c in args.command.split(" ;; "):
            print("# command: %s" % c)
    print("# %-90s %6s %12s %12s %12s %7s" % ("kernel", "calls", "avg_us", "min_us", "max_us", "pct"))
    for r in rows:
        print("  %-90s %6s %12.2f %12.2f %12.2f %7.2f" % (
            short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))


def _per_kernel(path):
    vals = defaultdict(list)
    grid = {}
    for r in csv.DictReader(open(path)):
        vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        grid.setdefault(r["Kernel_Name"], []).append(int(r["Grid_Size"]))
    return vals, grid


def _copy_reference(vals, grid):
    """Counter value of the probe copy: the largest dispatches of the
    library's streaming copy `k_stream_copy` (the bench's 2 GiB probe is far
    larger than any other copy in a run); dispatches within 1% of the
    largest are averaged."""
    v = [x for name, xs in vals.items() if "k_stream_copy" in name for x in xs]
    if not v:
        raise SystemExit("no k_stream_copy dispatch found for scaling")
    top = max(v)
    best = [x for x in v if x >= 0.99 * top]
    return sum(best) / len(best)


def cmd_pmc(args):
    fv, fg = _per_kernel(args.fetch)
    wv, wg = _per_kernel(args.write)
    fref, wref = _copy_reference(fv, fg), _copy_reference(wv, wg)
    fscale = args.copy_bytes / (fref * 1024.0)
    wscale = args.copy_bytes / (wref * 1024.0)
    print("# %s" % (args.title or "rocprofv3 HBM counters"))
    if args.command:
        for c in args.command.split(" ;; "):
            print("# command: %s" % c)
    print("# copy reference: %d B read and written per dispatch; FETCH_SIZE reads %.1f KiB, WRITE_SIZE %.1f KiB"
          % (args.copy_bytes, fref, wref))
    print("# %-90s %8s %14s %14s" % ("kernel", "n", "FETCH_KiB", "WRITE_KiB"))
    rows = {}
    for name in fv:
        f = sum(fv[name]) / len(fv[name])
        w = sum(wv.get(name, [0.0])) / max(len(wv.get(name, [])), 1)
        print("  %-90s %8d %14.1f %14.1f" % (short(name), len(fv[name]), f, w))
        rows[name] = (len(fv[name]), f, w)
    # --kernel a,b: a step made of several kernels; for each substring the
    # most-dispatched matching kernel, their per-dispatch counters summed
    chosen = []
    for sub in args.kernel.split(","):
        cands = [n for n in rows if sub in n]
        if not cands:
            raise SystemExit("kernel %r not found" % sub)
        chosen.append(max(cands, key=lambda n: rows[n][0]))
    f = sum(rows[n][1] for n in chosen)
    w = sum(rows[n][2] for n in chosen)
    print("kernel: %s" % " + ".join(chosen))
    print("fetch_kib_per_dispatch: %.3f" % f)
    print("write_kib_per_dispatch: %.3f" % w)
    print("fetch_scale: %.5f" % fscale)
    print("write_scale: %.5f" % wscale)
    print("traffic_bytes_per_launch: %.0f" % (f * 1024.0 * fscale + w * 1024.0 * wscale))
    print("source_digest: %s" % kernel_source_digest())


def read_traffic(path):
    """bench.py side: {key: value} of a pmc summary, or None if absent."""
    if not os.path.exists(path):
        return None
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith("#") and not line.startswith(" "):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--title")
    a.add_argument("--command")
    b = sub.add_parser("pmc")
    b.add_argument("fetch")
    b.add_argument("write")
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy-bytes", type=int, default=2 << 30)
    b.add_argument("--title")
    b.add_argument("--command")
    args = ap.parse_args(argv)
    {"stats": cmd_stats, "pmc": cmd_pmc}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
