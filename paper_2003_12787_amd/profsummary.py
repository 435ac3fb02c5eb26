"""Summarise rocprofv3 CSV output (kernel trace stats, or one --pmc pass) into a short text table.

usage: python -m paper_2003_12787_amd.profsummary stats <kernel_stats.csv>
       python -m paper_2003_12787_amd.profsummary pmc <counter_collection.csv> [<counter_collection.csv> ...]
"""
import collections
import csv
import sys


def stats(path):
    rows = list(csv.DictReader(open(path)))
    print(f"{'kernel':<72} {'calls':>5} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}")
    for r in rows:
        print(f"{r['Name'][:72]:<72} {r['Calls']:>5} {float(r['AverageNs']) / 1e3:>10.1f} "
              f"{float(r['MinNs']) / 1e3:>10.1f} {float(r['MaxNs']) / 1e3:>10.1f} {float(r['Percentage']):>6.2f}")


def pmc(paths):
    agg = collections.defaultdict(list)
    for p in paths:
        for r in csv.DictReader(open(p)):
            k = (r["Kernel_Name"][:72], int(r["Grid_Size"]), r["Counter_Name"])
            agg[k].append(float(r["Counter_Value"]))
    print(f"{'kernel':<72} {'grid':>9} {'counter':<24} {'n':>3} {'mean per dispatch':>18}")
    for (k, g, c), v in sorted(agg.items()):
        print(f"{k:<72} {g:>9} {c:<24} {len(v):>3} {sum(v) / len(v):>18.6g}")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    else:
        pmc(sys.argv[2:])
