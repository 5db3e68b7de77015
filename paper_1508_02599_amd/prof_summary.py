"""Text summaries of rocprofv3 CSV output (kernel trace and PMC counters).

    python -m paper_1508_02599_amd.prof_summary trace <dir> [--top N] [--min-us T]
    python -m paper_1508_02599_amd.prof_summary pmc <counter_dir> [--kernel NAME] [--min-kib K]

``trace`` reads ``*_kernel_trace.csv`` and prints, per kernel, the launch count,
total device time, the mean over all launches and the mean over launches that
last at least ``--min-us`` microseconds.  The PCG kernels of one replayed graph
block that run after the stopping rule has been met return at once; the second
mean leaves those out and is the one to compare with the HIP-event timings of
the library's profiling mode.

``pmc`` reads ``*_counter_collection.csv`` of a single-counter run and prints,
per kernel, the mean counter value per dispatch (KiB), over all dispatches and
over dispatches reading at least ``--min-kib``.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import re
from collections import defaultdict


def _short(name: str) -> str:
    name = re.sub(r"\(.*\)$", "", name)
    return name.replace("void ", "").replace("feti::", "")


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise SystemExit(f"no file matches {pattern}")
    return hits[0]


def trace_table(d: str, top: int = 20, min_us: float = 0.0):
    f = _one(os.path.join(d, "**", "*kernel_trace.csv"))
    dur = defaultdict(list)
    with open(f) as fh:
        for row in csv.DictReader(fh):
            t = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-3
            dur[_short(row["Kernel_Name"])].append(t)
    total = sum(sum(v) for v in dur.values())
    rows = []
    for k, v in dur.items():
        act = [x for x in v if x >= min_us]
        rows.append((sum(v), k, len(v), sum(v) / len(v), len(act), (sum(act) / len(act)) if act else 0.0))
    rows.sort(reverse=True)
    out = [f"| kernel | launches | total ms | % | mean us (all) | launches >= {min_us:g} us | mean us (those) |",
           "|---|---|---|---|---|---|---|"]
    for tot, k, n, mean, na, mact in rows[:top]:
        out.append(f"| `{k}` | {n} | {tot * 1e-3:.3f} | {100 * tot / total:.1f} | {mean:.1f} | {na} | {mact:.1f} |")
    out.append(f"\nTotal device time in kernels: {total * 1e-3:.3f} ms over {sum(len(v) for v in dur.values())} launches.")
    return "\n".join(out)


def pmc_table(d: str, kernel: str | None = None, min_kib: float = 0.0):
    f = _one(os.path.join(d, "**", "*counter_collection.csv"))
    vals = defaultdict(list)
    cname = None
    with open(f) as fh:
        for row in csv.DictReader(fh):
            k = _short(row["Kernel_Name"])
            if kernel and kernel not in k:
                continue
            cname = row["Counter_Name"]
            vals[k].append(float(row["Counter_Value"]))
    out = [f"| kernel | dispatches | mean {cname} KiB (all) | dispatches >= {min_kib:g} KiB | mean KiB (those) |",
           "|---|---|---|---|---|"]
    for k, v in sorted(vals.items(), key=lambda kv: -sum(kv[1])):
        act = [x for x in v if x >= min_kib]
        out.append(f"| `{k}` | {len(v)} | {sum(v) / len(v):.1f} | {len(act)} | "
                   f"{(sum(act) / len(act)) if act else 0.0:.1f} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "pmc"])
    ap.add_argument("dir")
    ap.add_argument("--top", type=int, default=20)
    ap.add_argument("--min-us", type=float, default=0.0)
    ap.add_argument("--kernel", default=None)
    ap.add_argument("--min-kib", type=float, default=0.0)
    a = ap.parse_args()
    if a.mode == "trace":
        print(trace_table(a.dir, a.top, a.min_us))
    else:
        print(pmc_table(a.dir, a.kernel, a.min_kib))


if __name__ == "__main__":
    main()
