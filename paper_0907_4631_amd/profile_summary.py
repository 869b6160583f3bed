"""Summarise a rocprofv3 results database (the rocpd SQLite file that
`rocprofv3 --kernel-trace` or `--pmc` writes) as a short text table: per
kernel the calls, total, average, minimum and maximum duration, and for
counter runs the per-dispatch counter values.  Reads only the database file.

    python -m paper_0907_4631_amd.profile_summary RESULTS.db [--counters]
"""
from __future__ import annotations

import argparse
import sqlite3


def kernel_stats(db):
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                     "max(duration) from kernels group by name order by sum(duration) desc")
    return [(n, k, tot, avg, mn, mx) for n, k, tot, avg, mn, mx in rows]


def counters(db):
    c = sqlite3.connect(db)
    cols = [r[1] for r in c.execute("pragma table_info(counters_collection)")]
    want = [x for x in ("kernel_name", "dispatch_id", "counter_name", "value") if x in cols]
    if len(want) < 4:
        return cols, []
    rows = c.execute(f"select {', '.join(want)} from counters_collection order by dispatch_id")
    return want, list(rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--counters", action="store_true")
    a = ap.parse_args()
    print("| kernel | calls | total ms | average us | min us | max us |")
    print("|---|---|---|---|---|---|")
    for n, k, tot, avg, mn, mx in kernel_stats(a.db):
        name = n if len(n) < 90 else n[:87] + "..."
        print(f"| {name} | {k} | {tot / 1e6:.3f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | "
              f"{mx / 1e3:.2f} |")
    if a.counters:
        cols, rows = counters(a.db)
        print()
        print("| kernel | dispatch | counter | value |")
        print("|---|---|---|---|")
        for r in rows:
            name = r[0] if len(r[0]) < 60 else r[0][:57] + "..."
            print(f"| {name} | {r[1]} | {r[2]} | {r[3]:.6g} |")


if __name__ == "__main__":
    main()
