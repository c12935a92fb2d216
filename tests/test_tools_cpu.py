"""Host-side tools: the rocprofv3 summaries the profiles are written with
(kernel-trace grouping by launch shape, calibrated HBM bytes, counter means),
on small synthetic inputs."""
import csv
import sqlite3

from paper_1607_05816_amd import rocpd_summary as R


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"], r)))


def test_trace_groups_by_kernel_and_launch_shape(tmp_path):
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, grid_x int, grid_y int, grid_z int, duration int)")
    rows = [("void uot::k_a(int)", 256, 1, 1, 100), ("void uot::k_a(int)", 256, 1, 1, 300),
            ("void uot::k_a(int)", 1024, 1, 1, 1000), ("void uot::k_b()", 64, 2, 1, 50)]
    con.executemany("insert into kernels values (?, ?, ?, ?, ?)", rows)
    con.commit()
    out = R.summarize(str(db), top=10).splitlines()
    assert out[2].startswith("| `uot::k_a` | 1024 x 1 x 1 | 1 | 1000 |")        # largest total first
    assert "| `uot::k_a` | 256 x 1 x 1 | 2 | 400 | 200 | 100 | 300 |" in out
    assert "| `uot::k_b` | 64 x 2 x 1 | 1 | 50 | 50 | 50 | 50 |" in out


def test_pmc_bytes_are_calibrated_by_the_copy(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    # the copy of 1 MiB reads 2048 KiB and writes 512 KiB as counted: factors 0.5 and 2
    _csv(f, [("__amd_rocclr_copyBuffer", 512, "FETCH_SIZE", 2048), ("uot::k(int)", 256, "FETCH_SIZE", 100),
             ("uot::k(int)", 256, "FETCH_SIZE", 300)])
    _csv(w, [("__amd_rocclr_copyBuffer", 512, "WRITE_SIZE", 512), ("uot::k(int)", 256, "WRITE_SIZE", 10),
             ("uot::k(int)", 256, "WRITE_SIZE", 30)])
    out = R.summarize_pmc(str(f), str(w), 1 << 20)
    assert "factors 0.5000 (fetch), 2.0000 (write)" in out
    # kernel: mean FETCH 200 KiB -> 102400 bytes, mean WRITE 20 KiB -> 40960 bytes
    assert "| `uot::k` | 256 | 2 | 200.0 | 20.0 | 102400 | 40960 |" in out


def test_counter_means_per_kernel(tmp_path):
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    _csv(a, [("void uot::k_x<3>(float)", 1024, "SQ_WAVES", 16), ("void uot::k_x<3>(float)", 1024, "SQ_WAVES", 32),
             ("void uot::other()", 64, "SQ_WAVES", 1)])
    _csv(b, [("void uot::k_x<3>(float)", 1024, "SQ_INSTS_MFMA", 5)])
    out = R.summarize_counters([str(a), str(b)], match="k_x").splitlines()
    assert out[0] == "| kernel | grid (work-items) | SQ_WAVES | SQ_INSTS_MFMA |"
    assert out[2] == "| `uot::k_x<3>` | 1024 | 24 | 5 |"
    assert len(out) == 3


def test_counter_means_over_last_dispatches(tmp_path):
    a = tmp_path / "a.csv"
    fields = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    rows = [(3, "uot::k_y()", 512, "SQ_WAVES", 30), (1, "uot::k_y()", 512, "SQ_WAVES", 1000),
            (4, "uot::k_y()", 512, "SQ_WAVES", 50), (2, "uot::k_y()", 512, "SQ_WAVES", 10)]
    with open(a, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(fields, r)))
    # the last two in dispatch order are 30 and 50; all four average 272.5
    assert R.summarize_counters([str(a)], last=2).splitlines()[2] == "| `uot::k_y` | 512 | 40 |"
    assert R.summarize_counters([str(a)]).splitlines()[2] == "| `uot::k_y` | 512 | 272.5 |"
