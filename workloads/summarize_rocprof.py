"""Turn rocprofv3 CSV output into the short text summaries kept in profiles/.

usage: python workloads/summarize_rocprof.py stats <kernel_stats.csv> [title]
       python workloads/summarize_rocprof.py pmc <counter_collection.csv> [title]
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


def pmc(path):
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        agg[r["Kernel_Name"][:70]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for v in agg.values() for c in v})
    out = ["| kernel | dispatches | " + " | ".join(f"{c} (avg/dispatch)" for c in names) + " |",
           "|---|---|" + "---|" * len(names)]
    for k, v in agg.items():
        n = max(len(x) for x in v.values())
        out.append(f"| `{k}` | {n} | " + " | ".join(
            "%.4g" % (sum(v[c]) / len(v[c])) if c in v else "-" for c in names) + " |")
    return "\n".join(out)


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    title = sys.argv[3] if len(sys.argv) > 3 else ""
    if title:
        print(f"## {title}\n")
    print(stats(path) if mode == "stats" else pmc(path))
