"""Short text summaries of rocprofv3 CSV output for this library's kernels.

  python -m paper_1902_08250_amd.prof_summary trace KERNEL_STATS_CSV --command CMD
      per-kernel calls, average / total duration (from --kernel-trace --stats)
  python -m paper_1902_08250_amd.prof_summary counters COUNTER_CSV --command CMD
      per-kernel averages of the counters of one --pmc pass
  python -m paper_1902_08250_amd.prof_summary traffic FETCH_CSV WRITE_CSV COPY_FETCH_CSV COPY_WRITE_CSV \\
         --copy-bytes N --command CMD
      per-kernel HBM bytes per dispatch from two --pmc passes (FETCH_SIZE,
      WRITE_SIZE, KiB per dispatch), each scaled by the factor that maps the
      same counter to the known bytes of a plain copy kernel

The traffic summary records a hash of the kernel sources it was taken on, so
that a reader can tell when the kernels have changed since.
"""
import argparse
import collections
import csv
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1902_08250_amd/csrc/cexp_tab.h", "paper_1902_08250_amd/csrc/expand_common.h",
                  "paper_1902_08250_amd/csrc/leaf.hip", "paper_1902_08250_amd/csrc/lmfmm_internal.h",
                  "paper_1902_08250_amd/csrc/near.hip", "paper_1902_08250_amd/csrc/tables.hip",
                  "paper_1902_08250_amd/csrc/translate.hip", "paper_1902_08250_amd/csrc/tree.hip"]


def source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name):
    n = name.replace("void ", "").replace("lmfmm::(anonymous namespace)::", "").replace("lmfmm::", "")
    depth, out = 0, []
    for ch in n:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out)


def trace(args):
    rows = list(csv.DictReader(open(args.csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("# Kernel trace: %s\n" % args.title)
    print("Command (from the repository root on the GPU machine):\n\n```\n%s\n```\n" % args.command)
    print("| kernel | calls | avg us | min us | max us | total ms | % |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for r in rows:
        print("| %s | %s | %.2f | %.2f | %.2f | %.3f | %.1f |" % (
            short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))


def per_kernel(path):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return agg


def traffic(args):
    f, w = per_kernel(args.fetch), per_kernel(args.write)
    cf, cw = per_kernel(args.copy_fetch), per_kernel(args.copy_write)

    def probe(agg):
        # the copy probe: the kernel dispatched three times
        k = max(agg, key=lambda k: (len(agg[k]) == 3, sum(agg[k])))
        return k, sum(agg[k]) / len(agg[k])
    kf, vf = probe(cf)
    kw, vw = probe(cw)
    kib = args.copy_bytes / 1024.0
    sf, sw = kib / vf, kib / vw
    print("# HBM traffic per dispatch: %s\n" % args.title)
    print("source_sha256: %s (kernel sources: %s)\n" % (source_hash(), ", ".join(KERNEL_SOURCES)))
    print("Commands (from the repository root on the GPU machine):\n\n```\n%s\n```\n" % args.command)
    print("Calibration: a plain copy of %d bytes read and %d bytes written (`%s`)." % (
        args.copy_bytes, args.copy_bytes, kf))
    print("FETCH_SIZE read %.1f KiB per dispatch: scale %.4f." % (vf, sf))
    print("WRITE_SIZE read %.1f KiB per dispatch: scale %.4f.\n" % (vw, sw))
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch (scaled) |")
    print("|---|---:|---:|---:|---|")
    rows = []
    for k in f:
        if k not in w:
            continue
        a, b = sum(f[k]) / len(f[k]), sum(w[k]) / len(w[k])
        rows.append((a * sf + b * sw, k, len(f[k]), a, b))
    rows.sort(reverse=True)
    for tot, k, n, a, b in rows:
        print("| %s | %d | %.1f | %.1f | bytes_per_launch=%.0f |" % (k, n, a, b, tot * 1024.0))


def counters(args):
    """Per-kernel averages of the counters of one --pmc pass."""
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(args.csv)):
        agg[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for d in agg.values() for c in d})
    print("# Counters per dispatch: %s\n" % args.title)
    print("source_sha256: %s (kernel sources: %s)\n" % (source_hash(), ", ".join(KERNEL_SOURCES)))
    print("Command (from the repository root on the GPU machine):\n\n```\n%s\n```\n" % args.command)
    print("| kernel | dispatches | " + " | ".join(names) + " |")
    print("|---|---:|" + "---:|" * len(names))
    rows = sorted(agg.items(), key=lambda kv: -sum(kv[1][names[0]]) if kv[1][names[0]] else 0)
    for k, d in rows:
        n = max(len(v) for v in d.values())
        vals = ["%.0f" % (sum(d[c]) / len(d[c])) if d[c] else "" for c in names]
        print("| %s | %d | %s |" % (k, n, " | ".join(vals)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--command", required=True)
    t.add_argument("--title", default="")
    c = sub.add_parser("traffic")
    for a in ("fetch", "write", "copy_fetch", "copy_write"):
        c.add_argument(a)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--title", default="")
    k = sub.add_parser("counters")
    k.add_argument("csv")
    k.add_argument("--command", required=True)
    k.add_argument("--title", default="")
    args = ap.parse_args(argv)
    {"trace": trace, "traffic": traffic, "counters": counters}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
