"""Summarise rocprofv3 CSV output into the short text records kept in profiles/.

  python -m paper_0912_4230_amd.prof_summary stats <kernel_stats.csv>
  python -m paper_0912_4230_amd.prof_summary tail <kernel_trace.csv> N
  python -m paper_0912_4230_amd.prof_summary pmc <counter_collection.csv> [<more.csv> ...]
  python -m paper_0912_4230_amd.prof_summary source-sha

`stats` prints the per-kernel table (calls, average / min / max duration);
`tail` prints the same over the last N dispatches of each kernel of a trace
(the steady state, without the start-up transient);
`pmc` prints, per kernel and counter, the per-dispatch values; `source-sha`
prints the SHA-256 of the kernel sources, which ties a counter record to the
code it was taken from.
"""
import csv
import hashlib
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


def source_sha() -> str:
    """SHA-256 of the lattice library's kernel sources (the probe library's
    source is not part of it)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hpp", ".hip", ".h", ".cpp")) and name != "probe.hip":
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()


def stats(path):
    rows = list(csv.DictReader(open(path)))
    print(f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}")
    for r in rows:
        print(f"{r['Name'][:70]:70s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.1f} "
              f"{float(r['MinNs']) / 1e3:10.1f} {float(r['MaxNs']) / 1e3:10.1f} {float(r['Percentage']):6.2f}")


def tail(path, n):
    per = defaultdict(list)
    for r in csv.DictReader(open(path)):
        per[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print(f"{'kernel (last ' + str(n) + ' dispatches)':70s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s}")
    for k, v in per.items():
        w = v[-n:]
        print(f"{k[:70]:70s} {len(w):6d} {sum(w) / len(w):10.1f} {min(w):10.1f} {max(w):10.1f}")


def pmc(paths):
    agg = defaultdict(list)
    for p in paths:
        for r in csv.DictReader(open(p)):
            agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    for (k, c), v in sorted(agg.items()):
        vals = ", ".join(f"{x:.0f}" for x in v)
        print(f"{k[:70]:70s} {c:12s} n={len(v)} values(KiB)=[{vals}]")


def main():
    if len(sys.argv) < 2:
        raise SystemExit(__doc__)
    what = sys.argv[1]
    if what == "stats":
        stats(sys.argv[2])
    elif what == "tail":
        tail(sys.argv[2], int(sys.argv[3]))
    elif what == "pmc":
        pmc(sys.argv[2:])
    elif what == "source-sha":
        print(source_sha())
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main()
