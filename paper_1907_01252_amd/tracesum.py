"""Summarise a rocprofv3 kernel trace or counter collection (CSV) by kernel and launch grid.

    python -m paper_1907_01252_amd.tracesum <run_kernel_trace.csv | run_counter_collection.csv> [--top N]
        [--match REGEX]

Kernel trace: one line per (kernel, grid) with the launch count, mean and total
duration.  Counter collection: one line per (kernel, grid, counter) with the
dispatch count and the mean, min and max of the counter value.  The grid is the
trace's total thread count per axis (threads in x, y, z), which separates the
launches of one kernel over different batch sizes and mesh levels.
"""
from __future__ import annotations

import argparse
import collections
import csv
import re


def _short(name: str) -> str:
    name = name.replace("void ", "")
    m = re.match(r"(?:fsi::)?([A-Za-z_0-9:]+(?:<[^(]*>)?)", name)
    return m.group(1) if m else name[:100]


def _grid(d: dict) -> str:
    g = [d.get(k) for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z")]
    g = [int(x) for x in g if x not in (None, "")]
    if not g and d.get("Grid_Size") not in (None, ""):
        g = [int(d["Grid_Size"])]   # counter collection: total threads of the launch
    while len(g) > 1 and g[-1] == 1:
        g.pop()
    return "x".join(str(x) for x in g)


def summarise(path: str, top: int = 30, match: str | None = None) -> list[str]:
    rows = list(csv.DictReader(open(path)))
    pat = re.compile(match) if match else None
    out = []
    if rows and "Counter_Name" in rows[0]:
        acc = collections.defaultdict(list)
        for d in rows:
            n = _short(d["Kernel_Name"])
            if pat and not pat.search(n):
                continue
            acc[(n, _grid(d), d["Counter_Name"])].append(float(d["Counter_Value"]))
        out.append("| kernel | grid | counter | dispatches | mean | min | max |")
        out.append("|---|---|---|---|---|---|---|")
        for (n, g, c), v in sorted(acc.items(), key=lambda kv: -len(kv[1]) * (sum(kv[1]) / len(kv[1])))[:top]:
            out.append(f"| {n} | {g} | {c} | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} |")
        return out
    acc = collections.defaultdict(lambda: [0, 0])
    t0, t1 = None, None
    for d in rows:
        n = _short(d["Kernel_Name"])
        s, e = int(d["Start_Timestamp"]), int(d["End_Timestamp"])
        t0 = s if t0 is None else min(t0, s)
        t1 = e if t1 is None else max(t1, e)
        if pat and not pat.search(n):
            continue
        a = acc[(n, _grid(d))]
        a[0] += 1
        a[1] += e - s
    out.append(f"trace span {(t1 - t0) / 1e6:.1f} ms, {len(rows)} dispatches")
    out.append("| kernel | grid | launches | mean us | total ms |")
    out.append("|---|---|---|---|---|")
    for (n, g), (c, ns) in sorted(acc.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"| {n} | {g} | {c} | {ns / c / 1e3:.2f} | {ns / 1e6:.2f} |")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("csv")
    ap.add_argument("--top", type=int, default=30)
    ap.add_argument("--match", default=None)
    a = ap.parse_args()
    print("\n".join(summarise(a.csv, a.top, a.match)))


if __name__ == "__main__":
    main()
