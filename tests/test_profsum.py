"""The rocprofv3 summary tool on synthetic SQLite files shaped like the
profiler's output views: kernel statistics, per-dispatch counters, and the
copy-calibrated traffic arithmetic."""
import sqlite3

import pytest

from paper_2508_12627_amd import profsum


def _db(path, counters=(), kernels=()):
    con = sqlite3.connect(path)
    con.execute("create table top_kernels (name text, total_calls int, total_duration real, "
                "average real, percentage real)")
    con.execute("create table counters_collection (kernel_name text, dispatch_id int, "
                "counter_name text, value real)")
    con.execute("create table kernels (name text, grid_x int, workgroup_x int, lds_size int, "
                "vgpr_count int, accum_vgpr_count int, scratch_size int, start int)")
    for row in kernels:
        con.execute("insert into top_kernels values (?,?,?,?,?)", row)
    for row in counters:
        con.execute("insert into counters_collection values (?,?,?,?)", row)
    con.commit()
    con.close()


def test_kernel_stats_and_markdown(tmp_path):
    db = str(tmp_path / "kt.db")
    _db(db, kernels=[("void k_gemm<2>(GemmDesc const*, int)", 5, 1600.0, 320.0, 60.0),
                     ("k_rbf(double const*)", 5, 250.0, 50.0, 9.0)])
    st = profsum.kernel_stats(db)
    assert st[0][:4] == ("void k_gemm<2>(GemmDesc const*, int)", 5, 1600.0, 320.0)
    md = str(tmp_path / "k.md")
    assert profsum.main(["kernels", db, "--md", md, "--title", "T", "--command", "rocprofv3 x"]) == 0
    text = open(md).read()
    assert "rocprofv3 x" in text and "| `void k_gemm<2>` | 5 | 1600.0 | 320.00 |" in text


def test_traffic_is_scaled_by_the_copy_calibration(tmp_path):
    GiB = 1 << 30
    cal_f, cal_w = str(tmp_path / "cf.db"), str(tmp_path / "cw.db")
    # the counters read half of the copy's reads and all of its writes (KiB)
    _db(cal_f, counters=[("copyBuffer", 1, "FETCH_SIZE", GiB / 2 / 1024)])
    _db(cal_w, counters=[("copyBuffer", 1, "WRITE_SIZE", GiB / 1024)])
    f, w = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    # two launches; FETCH_SIZE is split over two counter instances per dispatch
    _db(f, counters=[("k_gemm<2>", 1, "FETCH_SIZE", 100.0), ("k_gemm<2>", 1, "FETCH_SIZE", 50.0),
                     ("k_gemm<2>", 2, "FETCH_SIZE", 150.0), ("k_rbf", 3, "FETCH_SIZE", 7.0)])
    _db(w, counters=[("k_gemm<2>", 1, "WRITE_SIZE", 64.0), ("k_gemm<2>", 2, "WRITE_SIZE", 64.0)])
    rec = profsum.traffic(f, w, cal_f, cal_w, GiB, "k_gemm")
    assert rec["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert rec["calibration"]["write_scale"] == pytest.approx(1.0)
    k = rec["kernels"]["k_gemm<2>"]
    assert k["launches"] == 2
    assert k["fetch_bytes"] == pytest.approx(150.0 * 1024 * 2.0)
    assert k["write_bytes"] == pytest.approx(64.0 * 1024)
    assert k["bytes_per_launch"] == pytest.approx(150.0 * 1024 * 2.0 + 64.0 * 1024)
    assert "k_rbf" not in rec["kernels"]
    assert rec["source_hash"] == profsum.kernel_source_hash()
