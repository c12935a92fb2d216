"""Per-launch-shape kernel summaries of rocprofv3 output.

    python -m paper_1607_05816_amd.rocpd_summary <run_results.db> [--top N]
    python -m paper_1607_05816_amd.rocpd_summary --pmc <fetch.csv> <write.csv> [--copy-bytes B]
    python -m paper_1607_05816_amd.rocpd_summary --counters <a.csv> [<b.csv> ...] [--match S] [--last N]

rocprofv3's own --stats table averages every launch of a kernel symbol; the
same symbol runs here at several launch shapes (one field vs a batch of
fields), so this groups the dispatches by (kernel, grid size) and prints a
markdown table of calls and durations in ns.

--counters: counter_collection.csv files of `rocprofv3 --pmc` runs (any
counters); per kernel (and launch size) the mean of each counter over the
dispatches, one column per counter (--last N: over the last N dispatches of
each, in dispatch order); --match keeps kernels whose name holds S.

--pmc: the counter_collection.csv files of two `rocprofv3 --pmc FETCH_SIZE`
and `--pmc WRITE_SIZE` runs of the same program (--last N: means over the
last N dispatches of each kernel and launch size).  Both counters read KiB per
dispatch; each is calibrated by the largest single `__amd_rocclr_copyBuffer`
dispatch of the run, a plain device copy of --copy-bytes bytes (it fetches
and writes exactly that many), and the table gives calibrated bytes per
launch (--match keeps kernels whose name holds S).
"""
import argparse
import collections
import csv
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


def _counter_means(path, last=0):
    """Mean counter value per (kernel, grid size), over the last `last`
    dispatches of each in dispatch order (all when 0)."""
    agg = collections.defaultdict(list)
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r.get("Dispatch_Id") or 0))
    for r in rows:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        agg[(name, int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    if last > 0:
        agg = {k: v[-last:] for k, v in agg.items()}
    return {k: sum(v) / len(v) for k, v in agg.items()}, {k: len(v) for k, v in agg.items()}


def _largest_copy(path):
    """Counter value of the largest single __amd_rocclr_copyBuffer dispatch
    (the calibration copy; other copies of the run share its kernel and
    sometimes its launch size, so dispatches are not averaged here)."""
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if r["Kernel_Name"].split("(")[0].replace("void ", "") == "__amd_rocclr_copyBuffer"]
    return max(vals)


def summarize_pmc(fetch_csv, write_csv, copy_bytes, top=12, match=None, last=0):
    f, nf = _counter_means(fetch_csv, last)
    w, _ = _counter_means(write_csv, last)
    cf, cw = _largest_copy(fetch_csv), _largest_copy(write_csv)
    kf = copy_bytes / (cf * 1024.0)
    kw = copy_bytes / (cw * 1024.0)
    out = ["Calibration: copy of %d bytes reads FETCH_SIZE %.1f KiB, WRITE_SIZE %.1f KiB -> factors %.4f (fetch), "
           "%.4f (write)." % (copy_bytes, cf, cw, kf, kw), "",
           "| kernel | grid (work-items) | launches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | read (bytes) | written (bytes) |",
           "|:--|:--|--:|--:|--:|--:|--:|"]
    keys = [k for k in f if not match or match in k[0]]
    for k in sorted(keys, key=lambda k: -f[k] * nf[k])[:top]:
        wk = w.get(k, float("nan"))
        out.append("| `%s` | %d | %d | %.1f | %.1f | %.0f | %.0f |" % (k[0], k[1], nf[k], f[k], wk, f[k] * 1024 * kf,
                                                                   wk * 1024 * kw))
    return "\n".join(out)


def summarize_counters(paths, match=None, last=0):
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    names = []
    for path in paths:
        rows = list(csv.DictReader(open(path)))
        rows.sort(key=lambda r: int(r.get("Dispatch_Id") or 0))
        for r in rows:
            name = r["Kernel_Name"].split("(")[0].replace("void ", "")
            if match and match not in name:
                continue
            c = r["Counter_Name"]
            if c not in names:
                names.append(c)
            agg[(name, int(r["Grid_Size"]))][c].append(float(r["Counter_Value"]))
    out = ["| kernel | grid (work-items) | " + " | ".join(names) + " |",
           "|:--|--:|" + "--:|" * len(names)]
    for k in sorted(agg):
        sel = {c: agg[k][c][-last:] if last > 0 else agg[k][c] for c in names}
        vals = [("%.4g" % (sum(sel[c]) / len(sel[c]))) if sel[c] else "" for c in names]
        out.append("| `%s` | %d | %s |" % (k[0], k[1], " | ".join(vals)))
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="?")
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--copy-bytes", type=int, default=256 << 20)
    ap.add_argument("--counters", nargs="+")
    ap.add_argument("--match")
    ap.add_argument("--last", type=int, default=0)
    a = ap.parse_args()
    if a.counters:
        print(summarize_counters(a.counters, a.match, a.last))
    elif a.pmc:
        print(summarize_pmc(a.pmc[0], a.pmc[1], a.copy_bytes, a.top, a.match, a.last))
    else:
        print(summarize(a.db, a.top))


if __name__ == "__main__":
    main()
