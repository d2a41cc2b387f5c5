"""Summaries of rocprofv3 output for the profiles folder.

kernel trace (rocpd SQLite):  python -m paper_2509_07690_amd.prof_summary trace DB TITLE COMMAND
counters (CSV):               python -m paper_2509_07690_amd.prof_summary counters CSV TITLE COMMAND

The trace summary lists launches, total and average duration per kernel and
adds one line per kernel family over its template instances.  The counter
summary lists, per kernel, the mean value per dispatch of every counter.
"""
import csv
import re
import sqlite3
import sys
from collections import defaultdict


def _short(name):
    short = name.replace("hylu::(anonymous namespace)::", "").replace("void ", "")
    head = short.split("(")[0]
    if ">(" in short:
        return short[:short.index(">(") + 1]
    return head


def summary(db_path, title, command):
    cur = sqlite3.connect(db_path).cursor()
    rows = cur.execute("select name, count(*), sum(end-start), avg(end-start) from kernels "
                       "group by name order by 3 desc").fetchall()
    tot = sum(r[2] for r in rows)
    out = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "", "```", command, "```", "",
           "| kernel | launches | total ms | avg us | share |", "|---|---:|---:|---:|---:|"]
    fam = defaultdict(lambda: [0, 0.0])
    for name, n, t, a in rows:
        short = _short(name)
        out.append(f"| `{short}` | {n} | {t / 1e6:.3f} | {a / 1e3:.2f} | {100 * t / tot:.1f}% |")
        base = short.split("<")[0]
        fam[base][0] += n
        fam[base][1] += t
    out += ["", "Kernel families (all template instances together):", "",
            "| family | launches | total ms | avg us |", "|---|---:|---:|---:|"]
    for base, (n, t) in sorted(fam.items(), key=lambda kv: -kv[1][1]):
        if n:
            out.append(f"| `{base}` | {n} | {t / 1e6:.3f} | {t / n / 1e3:.2f} |")
    out.append("")
    out.append(f"Total kernel time {tot / 1e6:.2f} ms over all launches in the traced run.")
    return "\n".join(out) + "\n"


def counters(csv_path, title, command):
    vals = defaultdict(lambda: defaultdict(list))
    with open(csv_path, newline="") as f:
        for rec in csv.DictReader(f):
            name = _short(rec["Kernel_Name"]).split("<")[0]
            vals[name][rec["Counter_Name"]].append(float(rec["Counter_Value"]))
    out = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "", "```", command, "```", "",
           "| kernel family | counter | dispatches | mean per dispatch | total |", "|---|---|---:|---:|---:|"]
    for name in sorted(vals):
        for cn in sorted(vals[name]):
            v = vals[name][cn]
            out.append(f"| `{name}` | {cn} | {len(v)} | {sum(v) / len(v):.1f} | {sum(v):.1f} |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    mode, path, title, cmd = sys.argv[1:5]
    sys.stdout.write(summary(path, title, cmd) if mode == "trace" else counters(path, title, cmd))
