"""Turn rocprofv3 CSV output into the short text summaries kept in profiles/.

usage: python workloads/summarize_rocprof.py stats <kernel_stats.csv> [title]
       python workloads/summarize_rocprof.py trace <kernel_trace.csv> [title]
       python workloads/summarize_rocprof.py pmc <counter_collection.csv> [title]
       python workloads/summarize_rocprof.py batch <kernel_trace.csv> <ticks>

`trace` groups dispatches by kernel and grid size, which separates the
workloads of one run (their grids differ).
"""
import collections
import csv
import sys


def stats(path):
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append("| `%s` | %s | %.2f | %.2f | %.2f | %.1f%% |" % (
            r["Name"][:70], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def trace(path):
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(list)
    for r in rows:
        grid = "x".join(r[f"Grid_Size_{a}"] for a in "XYZ")
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        agg[(r["Kernel_Name"][:70], grid, r["Workgroup_Size_X"])].append(dur)
    tot = sum(sum(v) for v in agg.values())
    out = ["| kernel | grid (threads) | block | calls | avg us | min us | max us | share |",
           "|---|---|---|---|---|---|---|---|"]
    for (k, g, b), v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        out.append("| `%s` | %s | %s | %d | %.2f | %.2f | %.2f | %.1f%% |" % (
            k, g, b, len(v), sum(v) / len(v), min(v), max(v), 100 * sum(v) / tot))
    return "\n".join(out)


def pmc(path):
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        key = "%s` grid %s `" % (r["Kernel_Name"][:70], r["Grid_Size"])
        agg[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for v in agg.values() for c in v})
    out = ["| kernel | dispatches | " + " | ".join(f"{c} (avg/dispatch)" for c in names) + " |",
           "|---|---|" + "---|" * len(names)]
    for k, v in agg.items():
        n = max(len(x) for x in v.values())
        out.append(f"| `{k}` | {n} | " + " | ".join(
            "%.4g" % (sum(v[c]) / len(v[c])) if c in v else "-" for c in names) + " |")
    return "\n".join(out)


def batch(path, ticks):
    """The batched phase kernels (kb_*) of a run of `ticks` batch steps:
    per kernel its calls, per-launch times and time per step."""
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(list)
    for r in rows:
        if "kb_" not in r["Kernel_Name"]:
            continue
        agg[r["Kernel_Name"][:70]].append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    tot = sum(sum(v) for v in agg.values())
    out = ["| kernel | calls | avg us | min us | max us | per step us | share |",
           "|---|---|---|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        out.append("| `%s` | %d | %.1f | %.1f | %.1f | %.1f | %.1f%% |" % (
            k, len(v), sum(v) / len(v), min(v), max(v), sum(v) / ticks, 100 * sum(v) / tot))
    out.append("")
    out.append("batched kernels per step: %.2f ms" % (tot / ticks / 1e3))
    return "\n".join(out)


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    if mode == "batch":
        print(batch(path, int(sys.argv[3])))
        sys.exit(0)
    title = sys.argv[3] if len(sys.argv) > 3 else ""
    if title:
        print(f"## {title}\n")
    print({"stats": stats, "trace": trace, "pmc": pmc}[mode](path))
