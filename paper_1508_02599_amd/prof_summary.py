"""Text summaries of rocprofv3 CSV output (kernel trace and PMC counters).

    python -m paper_1508_02599_amd.prof_summary trace <dir> [--top N] [--min-us T]
    python -m paper_1508_02599_amd.prof_summary pmc <counter_dir> [--kernel NAME] [--min-kib K]
    python -m paper_1508_02599_amd.prof_summary gaps <dir> [--top N]
    python -m paper_1508_02599_amd.prof_summary factor-gaps <dir>
    python -m paper_1508_02599_amd.prof_summary traffic --fp64 FETCH_DIR WRITE_DIR
                                                        [--mixed FETCH_DIR WRITE_DIR]

``trace`` reads ``*_kernel_trace.csv`` and prints, per kernel, the launch count,
total device time, the mean over all launches and the mean over launches that
last at least ``--min-us`` microseconds.  The PCG kernels of one replayed graph
block that run after the stopping rule has been met return at once; the second
mean leaves those out and is the one to compare with the HIP-event timings of
the library's profiling mode.

``gaps`` prints the device's idle time between consecutive kernels,
attributed to the kernel that follows each gap; ``factor-gaps`` the idle time
between the launches of each factorisation phase.

``pmc`` reads ``*_counter_collection.csv`` of a single-counter run and prints,
per kernel, the mean counter value per dispatch (KiB), over all dispatches and
over dispatches reading at least ``--min-kib``.

``traffic`` turns FETCH_SIZE and WRITE_SIZE runs of ``bench.py`` into the HBM
bytes per launch of the factor update (last factorisation of the run) and of
the GEMV, scaled by the copy calibration, and writes profiles/traffic.json
with the hash of each kernel's source (bench.py drops a figure whose source
has changed since).
"""
from __future__ import annotations

import argparse
import json
import csv
import glob
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


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


def overlap_table(d: str):
    """Concurrency of kernels on different streams in a kernel trace: the
    time during which at least one kernel ran (busy), the sum of kernel
    durations (work), and the time with kernels of two or more streams
    running at once (overlap), in ms."""
    f = _one(os.path.join(d, "**", "*kernel_trace.csv"))
    ev = []
    with open(f) as fh:
        for row in csv.DictReader(fh):
            a, b = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
            q = (row.get("Queue_Id"), row.get("Stream_Id"))
            ev.append((a, 1, q))
            ev.append((b, -1, q))
    ev.sort(key=lambda e: (e[0], e[1]))
    active = defaultdict(int)
    busy = over = work = 0
    last = None
    streams = set()
    for t, d_, q in ev:
        if last is not None and t > last:
            n_str = sum(1 for v in active.values() if v > 0)
            n_k = sum(active.values())
            if n_k:
                busy += t - last
                work += n_k * (t - last)
            if n_str >= 2:
                over += t - last
        active[q] += d_
        streams.add(q)
        last = t
    span = (ev[-1][0] - ev[0][0]) if ev else 0
    return (f"streams {len(streams)}; trace span {span * 1e-6:.1f} ms; busy {busy * 1e-6:.1f} ms; "
            f"kernel time {work * 1e-6:.1f} ms; two or more streams running at once {over * 1e-6:.1f} ms "
            f"({100 * over / max(1, busy):.0f}% of busy time); kernel time / busy time {work / max(1, busy):.2f}")


def _sorted_kernels(d: str):
    f = _one(os.path.join(d, "**", "*kernel_trace.csv"))
    with open(f) as fh:
        return sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short(r["Kernel_Name"]))
                      for r in csv.DictReader(fh))


def gaps_table(d: str, top: int = 20):
    """Idle time of the device between consecutive kernels (any stream),
    attributed to the kernel that starts after each gap."""
    rows = _sorted_kernels(d)
    if not rows:
        return "empty trace"
    end = rows[0][1]
    idle = 0
    by = defaultdict(lambda: [0, 0])
    sizes = [0, 0, 0, 0]
    for s, e, n in rows[1:]:
        g = s - end
        if g > 0:
            idle += g
            by[n][0] += g
            by[n][1] += 1
            sizes[0 if g < 2000 else 1 if g < 10000 else 2 if g < 50000 else 3] += g
        end = max(end, e)
    span = rows[-1][1] - rows[0][0]
    out = [f"span {span * 1e-6:.1f} ms, idle {idle * 1e-6:.1f} ms ({100 * idle / span:.1f}%), kernels {len(rows)}",
           "idle by gap size (<2us, <10us, <50us, >=50us) ms: " + str([round(x * 1e-6, 1) for x in sizes])]
    for n, (g, c) in sorted(by.items(), key=lambda kv: -kv[1][0])[:top]:
        out.append(f"  before {n}: {g * 1e-6:.1f} ms over {c} gaps ({g / c * 1e-3:.1f} us mean)")
    return "\n".join(out)


_FACTOR = ("k_update", "k_diag", "k_trsm", "k_trtri", "k_lauum", "k_copy_iface", "k_regularise", "k_rho", "k_wb")
_BESIDE = ("k_init_arena", "k_coarse", "k_modes", "copyBuffer")


def factor_gaps_table(d: str, last: int = 6):
    """Idle time inside the factorisation: each maximal run of factor kernels
    (kernels of the coarse stream that run beside it do not end a run) with
    its launch count, span and the gaps between its kernels; the last runs."""
    runs, cur = [], []
    for s, e, n in _sorted_kernels(d):
        if any(k in n for k in _FACTOR):
            cur.append((s, e))
        elif cur and not any(k in n for k in _BESIDE):
            if len(cur) > 20:
                runs.append(cur)
            cur = []
    if len(cur) > 20:
        runs.append(cur)
    out = []
    for r in runs[-last:]:
        span = r[-1][1] - r[0][0]
        end, gaps = r[0][0], 0
        for s, e in r:
            if s > end:
                gaps += s - end
            end = max(end, e)
        out.append(f"factor phase: {len(r)} launches, span {span * 1e-6:.2f} ms, idle gaps {gaps * 1e-6:.2f} ms "
                   f"({100 * gaps / span:.1f}%)")
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


def _dispatches(d: str):
    """(dispatch id, kernel, workgroups, counter value) of a single-counter run, in order."""
    f = _one(os.path.join(d, "**", "*counter_collection.csv"))
    out = []
    with open(f) as fh:
        for row in csv.DictReader(fh):
            wg = int(row["Grid_Size"]) // max(1, int(row["Workgroup_Size"]))
            out.append((int(row["Dispatch_Id"]), _short(row["Kernel_Name"]), wg, float(row["Counter_Value"])))
    out.sort()
    return out


def update_bytes_per_launch(fetch_dir: str, write_dir: str, fetch_scale: float, write_scale: float):
    """HBM bytes per factor-update launch, from the last factorisation of the
    run: the dispatches after the last full-size k_init_arena.  Every update
    launch of the batched factorisation is one k_update / k_update_db /
    k_update_wide dispatch of at least 64 workgroups (the diagonal tiles of
    its column alone are 64 for cube32_s4); the coarse factorisation's update
    launches are far smaller and left out.  Counter values are KiB per
    dispatch, scaled by the copy calibration."""
    tot, n = 0.0, 0
    for d, scale in ((fetch_dir, fetch_scale), (write_dir, write_scale)):
        rows = _dispatches(d)
        starts = [i for i, r in enumerate(rows) if r[1].startswith("k_init_arena") and r[2] > 10000]
        upd = [r for r in rows[starts[-1]:] if r[1].startswith("k_update") and r[2] >= 64]
        tot += scale * 1024.0 * sum(r[3] for r in upd)
        n = len(upd)
    return tot / n, n


def gemv_bytes_per_launch(fetch_dir: str, write_dir: str, fetch_scale: float, write_scale: float,
                          min_kib: float = 1000.0):
    """HBM bytes per GEMV launch: mean over the k_symv_one dispatches that did
    the work (a replayed graph block's launches after the stopping rule return
    at once and read nothing)."""
    f = [r[3] for r in _dispatches(fetch_dir) if r[1].startswith("k_symv_one") and r[3] >= min_kib]
    w = [r[3] for r in _dispatches(write_dir) if r[1].startswith("k_symv_one")]
    w = sorted(w)[len(w) - len(f):] if len(w) >= len(f) else w
    return 1024.0 * (fetch_scale * sum(f) / len(f) + write_scale * sum(w) / max(1, len(w)))


def write_traffic(out: str, runs: dict, fetch_scale: float, write_scale: float, summary: str):
    """runs: precision -> (fetch_dir, write_dir).  Writes the per-launch HBM
    bytes of the update and GEMV kernels with the hash of their sources."""
    import hashlib
    root = os.path.dirname(HERE)

    def sha(rel):
        with open(os.path.join(root, rel), "rb") as fh:
            return hashlib.sha256(fh.read()).hexdigest()[:16]

    rec = {}
    for prec, (fd, wd) in runs.items():
        suffix = "" if prec == "fp64" else "_f32"
        ub, n = update_bytes_per_launch(fd, wd, fetch_scale, write_scale)
        gb = gemv_bytes_per_launch(fd, wd, fetch_scale, write_scale)
        rec["k_update" + suffix] = {"source": "paper_1508_02599_amd/csrc/k_dense.hip",
                                    "source_sha": sha("paper_1508_02599_amd/csrc/k_dense.hip"),
                                    "hbm_bytes_per_launch": round(ub), "launches": n, "summary": summary}
        rec["k_symv_one" + suffix] = {"source": "paper_1508_02599_amd/csrc/k_symv.hip",
                                        "source_sha": sha("paper_1508_02599_amd/csrc/k_symv.hip"),
                                        "hbm_bytes_per_launch": round(gb), "summary": summary}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "pmc", "traffic", "overlap", "gaps", "factor-gaps"])
    ap.add_argument("dir", nargs="?")
    ap.add_argument("--top", type=int, default=20)
    ap.add_argument("--min-us", type=float, default=0.0)
    ap.add_argument("--kernel", default=None)
    ap.add_argument("--min-kib", type=float, default=0.0)
    ap.add_argument("--fp64", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--mixed", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--fetch-scale", type=float, default=2.0)
    ap.add_argument("--write-scale", type=float, default=1.0)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(HERE), "profiles", "traffic.json"))
    ap.add_argument("--summary", default="profiles/feti_cube32_s4_traffic.md")
    a = ap.parse_args()
    if a.mode == "trace":
        print(trace_table(a.dir, a.top, a.min_us))
    elif a.mode == "overlap":
        print(overlap_table(a.dir))
    elif a.mode == "gaps":
        print(gaps_table(a.dir, a.top))
    elif a.mode == "factor-gaps":
        print(factor_gaps_table(a.dir))
    elif a.mode == "pmc":
        print(pmc_table(a.dir, a.kernel, a.min_kib))
    else:
        runs = {}
        if a.fp64:
            runs["fp64"] = tuple(a.fp64)
        if a.mixed:
            runs["mixed"] = tuple(a.mixed)
        print(json.dumps(write_traffic(a.out, runs, a.fetch_scale, a.write_scale, a.summary), indent=1))


if __name__ == "__main__":
    main()
