"""Summarise rocprofv3 CSV output (kernel trace stats, or one --pmc pass) into a short text table.

usage: python -m paper_2003_12787_amd.profsummary stats <kernel_stats.csv>
       python -m paper_2003_12787_amd.profsummary trace <kernel_trace.csv> [last_k]
       python -m paper_2003_12787_amd.profsummary pmc <counter_collection.csv> [<counter_collection.csv> ...]
       python -m paper_2003_12787_amd.profsummary issue <counter_collection.csv> [match]

`issue` reads one pass holding SQ_WAVES, SQ_WAVE_CYCLES, SQ_ACTIVE_INST_VALU, SQ_INSTS_VALU, SQ_INSTS_LDS,
SQ_WAIT_INST_LDS and SQ_WAIT_INST_ANY and gives, per kernel whose name contains `match`, the dispatch duration,
the VALU and LDS instructions per wave, and three shares: resident waves per SIMD and VALU-busy share of the
SIMDs (both from the quad-cycle counters over the dispatch's duration at 2.4 GHz on 1024 SIMDs: a lower clock
under load makes both larger), and the share of a wave's cycles spent waiting on LDS and on anything.

`trace` gives, per kernel, the dispatch count and the mean, median, min and max duration over all dispatches
and over the last `last_k` of them (the launches a benchmark times after its warm-up ones).
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


def trace(path, last_k=None):
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        per[r["Kernel_Name"]].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    hdr = f"{'kernel':<64} {'calls':>5} {'mean_us':>9} {'med_us':>9} {'min_us':>9} {'max_us':>9}"
    if last_k:
        hdr += f" | {'last':>4} {'mean_us':>9} {'med_us':>9} {'min_us':>9} {'max_us':>9}"
    print(hdr)
    rows = sorted(per.items(), key=lambda kv: -sum(e - b for b, e in kv[1]))
    for name, d in rows:
        d.sort()
        us = [(e - b) / 1e3 for b, e in d]

        def fmt(v):
            v2 = sorted(v)
            med = v2[len(v2) // 2] if len(v2) % 2 else 0.5 * (v2[len(v2) // 2 - 1] + v2[len(v2) // 2])
            return f"{sum(v) / len(v):>9.1f} {med:>9.1f} {min(v):>9.1f} {max(v):>9.1f}"
        line = f"{name[:64]:<64} {len(us):>5} {fmt(us)}"
        if last_k and len(us) >= last_k:
            line += f" | {last_k:>4} {fmt(us[-last_k:])}"
        print(line)


def pmc(paths):
    agg = collections.defaultdict(list)
    for p in paths:
        for r in csv.DictReader(open(p)):
            k = (r["Kernel_Name"][:72], int(r["Grid_Size"]), r["Counter_Name"])
            agg[k].append(float(r["Counter_Value"]))
    print(f"{'kernel':<72} {'grid':>9} {'counter':<24} {'n':>3} {'mean per dispatch':>18}")
    for (k, g, c), v in sorted(agg.items()):
        print(f"{k:<72} {g:>9} {c:<24} {len(v):>3} {sum(v) / len(v):>18.6g}")


def issue(path, match="", clock_ghz=2.4, simds=1024):
    cnt = collections.defaultdict(lambda: collections.defaultdict(list))
    dur = collections.defaultdict(dict)
    for r in csv.DictReader(open(path)):
        k = r["Kernel_Name"]
        if match not in k:
            continue
        cnt[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        dur[k][r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    print(f"{'kernel':<60} {'waves':>7} {'us':>8} {'valu/w':>7} {'lds/w':>6} {'w/simd':>6} "
          f"{'valu%':>6} {'ldsw%':>6} {'wait%':>6}")
    for k, c in cnt.items():
        m = {n: sum(v) / len(v) for n, v in c.items()}
        d = sum(dur[k].values()) / len(dur[k])
        cyc = d * clock_ghz * simds  # SIMD-cycles of the dispatch
        wv, wc = m["SQ_WAVES"], m["SQ_WAVE_CYCLES"]
        print(f"{k[:60]:<60} {wv:>7.0f} {d / 1e3:>8.1f} {m['SQ_INSTS_VALU'] / wv:>7.0f} "
              f"{m['SQ_INSTS_LDS'] / wv:>6.0f} {4 * wc / cyc:>6.2f} {100 * 4 * m['SQ_ACTIVE_INST_VALU'] / cyc:>6.1f} "
              f"{100 * m['SQ_WAIT_INST_LDS'] / wc:>6.1f} {100 * m['SQ_WAIT_INST_ANY'] / wc:>6.1f}")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif sys.argv[1] == "issue":
        issue(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "")
    elif sys.argv[1] == "trace":
        trace(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else None)
    else:
        pmc(sys.argv[2:])
