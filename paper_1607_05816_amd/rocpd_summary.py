"""Per-launch-shape kernel summary of a rocprofv3 trace database.

    python -m paper_1607_05816_amd.rocpd_summary <run_results.db> [--top N]

rocprofv3's own --stats table averages every launch of a kernel symbol; the
same symbol runs here at several launch shapes (one field vs a batch of
fields), so this groups the dispatches by (kernel, grid size) and prints a
markdown table of calls and durations in ns.
"""
import argparse
import sqlite3


def summarize(path, top=12):
    db = sqlite3.connect(path)
    rows = db.execute(
        "select name, grid_x, grid_y, grid_z, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name, grid_x, grid_y, grid_z order by sum(duration) desc limit ?", (top,)).fetchall()
    out = ["| kernel | grid (work-items) | calls | total (ns) | average (ns) | min (ns) | max (ns) |",
           "|:--|:--|--:|--:|--:|--:|--:|"]
    for name, gx, gy, gz, n, tot, avg, mn, mx in rows:
        short = name.split("(")[0].replace("void ", "")
        out.append("| `%s` | %d x %d x %d | %d | %d | %.0f | %d | %d |" % (short, gx, gy, gz, n, tot, avg, mn, mx))
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=12)
    a = ap.parse_args()
    print(summarize(a.db, a.top))


if __name__ == "__main__":
    main()
