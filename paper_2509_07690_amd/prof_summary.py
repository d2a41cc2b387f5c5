"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) as a markdown
table: launches, total and average duration per kernel."""
import sqlite3
import sys


def summary(db_path, title, command, per_step_div=1):
    cur = sqlite3.connect(db_path).cursor()
    rows = cur.execute("select name, count(*), sum(end-start), avg(end-start) from kernels "
                       "group by name order by 3 desc").fetchall()
    tot = sum(r[2] for r in rows)
    out = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "", "```", command, "```", "",
           "| kernel | launches | total ms | avg us | share |", "|---|---:|---:|---:|---:|"]
    for name, n, t, a in rows:
        short = name.replace("hylu::(anonymous namespace)::", "").replace("void ", "")
        short = short.split("(")[0] if "<" not in short.split("(")[0] or ">" in short.split("(")[0] else short
        short = short[:short.index(">(") + 1] if ">(" in short else short.split("(")[0]
        out.append(f"| `{short}` | {n} | {t / 1e6:.3f} | {a / 1e3:.2f} | {100 * t / tot:.1f}% |")
    out.append("")
    out.append(f"Total kernel time {tot / 1e6:.2f} ms over all launches in the traced run.")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    db, title, cmd = sys.argv[1], sys.argv[2], sys.argv[3]
    sys.stdout.write(summary(db, title, cmd))
