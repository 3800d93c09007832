"""Summaries of rocprofv3 kernel traces (the SQLite database rocprofv3 writes
with --kernel-trace) and of its counter runs (--pmc), as the markdown tables
kept beside the benchmark's figures.

    python -m paper_2308_05007_amd.profsum trace DB|TRACE.csv [--window REGEX N]
    python -m paper_2308_05007_amd.profsum pmc DB COUNTER REGEX N

trace: per-kernel count, total, average, minimum and maximum duration over
every dispatch; with --window, the average duration of the last N
dispatches of the kernels matching REGEX (a benchmark's timed launches),
the span of that window on the GPU clock, the other kernels inside it and
the idle time between dispatches.
pmc: the average per dispatch of a counter over the last N dispatches of the
kernels matching REGEX.
"""
import argparse
import re
import sqlite3
import sys

import numpy as np


def _rows(db):
    """(name, start ns, end ns, grid size) of every dispatch, from a rocprofv3
    database or its kernel-trace CSV (--output-format csv)."""
    if db.endswith(".csv"):
        import csv
        with open(db) as fh:
            rows = [(r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"]),
                     int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
                    for r in csv.DictReader(fh)]
        return sorted(rows, key=lambda r: r[1])
    c = sqlite3.connect(db)
    return list(c.execute("select name, start, end, grid_x * grid_y * grid_z from kernels order by start"))


def _short(name):
    return name.split("(")[0].replace("void ", "")


def _table(rows):
    stats = {}
    for n, s, e, _ in rows:
        stats.setdefault(_short(n), []).append((e - s) / 1e3)
    out = ["| kernel | dispatches | total ms | average us | min us | max us |", "|---|---|---|---|---|---|"]
    for k, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        v = np.array(v)
        out.append("| `%s` | %d | %.3f | %.2f | %.2f | %.2f |" % (k, v.size, v.sum() / 1e3, v.mean(), v.min(), v.max()))
    return out


def _window(rows, regex, n):
    pat = re.compile(regex)
    sel = [r for r in rows if pat.search(r[0])]
    if not sel:
        raise SystemExit("no dispatch matches %r" % regex)
    last = sel[-n:]
    t0, t1 = last[0][1], last[-1][2]
    win = [r for r in rows if r[1] >= t0 and r[2] <= t1]
    return last, win, t0, t1


def trace(db, window=None):
    rows = _rows(db)
    out = ["All dispatches:", ""] + _table(rows)
    if window:
        regex, n = window
        last, win, t0, t1 = _window(rows, regex, n)
        d = np.array([(e - s) / 1e3 for _, s, e, _ in last])
        busy = sum(e - s for _, s, e, _ in win)
        st = np.array([s for _, s, _, _ in win], float)
        en = np.array([e for _, _, e, _ in win], float)
        gaps = (st[1:] - en[:-1]).clip(0) if len(win) > 1 else np.zeros(1)
        out += ["", "Window: the last %d dispatches of kernels matching `%s`:" % (len(last), regex),
                "", "- average duration %.2f us (min %.2f, max %.2f)" % (d.mean(), d.min(), d.max()),
                "- span on the GPU clock %.3f ms for %d dispatches of all kernels; busy %.3f ms, idle %.2f%%"
                % ((t1 - t0) / 1e6, len(win), busy / 1e6, 100.0 * (1 - busy / (t1 - t0))),
                "- gaps between consecutive dispatches: median %.2f us, mean %.2f us, total %.3f ms"
                % (np.median(gaps) / 1e3, gaps.mean() / 1e3, gaps.sum() / 1e6), "", "Kernels inside the window:", ""]
        out += _table(win)
    return "\n".join(out)


def pmc(db, counter, regex, n):
    c = sqlite3.connect(db)
    cols = [d[1] for d in c.execute("pragma table_info(counters_collection)")]
    name_col = "counter_name" if "counter_name" in cols else "name"
    val_col = "value" if "value" in cols else "counter_value"
    kname = "kernel_name" if "kernel_name" in cols else "name"
    q = ("select %s, %s, grid_size, dispatch_id from counters_collection where %s = ? order by dispatch_id"
         % (kname, val_col, name_col))
    rows = [r for r in c.execute(q, (counter,)) if re.search(regex, r[0])]
    if not rows:
        raise SystemExit("no %s values for %r" % (counter, regex))
    full = rows[-n:]
    v = np.array([r[1] for r in full], float)
    return {"counter": counter, "kernel": _short(full[0][0]), "dispatches": int(v.size), "average": float(v.mean()),
            "min": float(v.min()), "max": float(v.max())}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--window", nargs=2, metavar=("REGEX", "N"))
    p = sub.add_parser("pmc")
    p.add_argument("db")
    p.add_argument("counter")
    p.add_argument("regex")
    p.add_argument("n", type=int)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        w = (a.window[0], int(a.window[1])) if a.window else None
        print(trace(a.db, w))
    else:
        print(pmc(a.db, a.counter, a.regex, a.n))


if __name__ == "__main__":
    sys.exit(main())
