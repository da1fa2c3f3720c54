"""The profiler-summary helper on small synthetic databases with the columns rocprofv3 writes."""
import json
import sqlite3

from paper_2010_15069_amd import profile_summary as ps


def _trace_db(path):
    c = sqlite3.connect(path)
    c.execute("create table kernels (name text, grid_x int, grid_y int, workgroup_x int, vgpr_count int, "
              "lds_size int, scratch_size int, start int, end int)")
    rows = [("void sgpe::col_kernel<1024, 1, 1, 16>(sgpe::ColArgsT<float>)", 131072, 1, 512, 124, 78336, 0, 0, 14000),
            ("void sgpe::col_kernel<1024, 1, 1, 16>(sgpe::ColArgsT<float>)", 131072, 1, 512, 124, 78336, 0, 0, 16000),
            ("void sgpe::row_kernel<1024, 2, true, false, 1, 16>(sgpe::RowArgsT<float>)", 131072, 1, 128, 96, 17408,
             0, 0, 12000)]
    c.executemany("insert into kernels values (?,?,?,?,?,?,?,?,?)", rows)
    c.commit()
    c.close()


def _counter_db(path, counter, per_dispatch):
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (dispatch_id int, kernel_name text, counter_name text, value real)")
    rows = []
    for d, (kernel, values) in enumerate(per_dispatch):
        for v in values:      # one row per counter instance; the helper sums them per dispatch
            rows.append((d, kernel, counter, v))
    c.executemany("insert into counters_collection values (?,?,?,?)", rows)
    c.commit()
    c.close()


def test_trace_table_groups_and_orders_by_total_time(tmp_path):
    db = str(tmp_path / "t.db")
    _trace_db(db)
    lines = ps.trace_table(db).splitlines()
    assert lines[2].startswith("| `col_kernel<1024, 1, 1, 16>` | 256 | 512 | 124 | 78336 | 0 | 2 | 15.00 | 15.00 | 14.00 | 16.00 |")
    assert lines[3].startswith("| `row_kernel<1024, 2, true, false, 1, 16>` | 1024 | 128 |")


def test_traffic_record_scales_by_the_copy(tmp_path):
    col = "void sgpe::col_kernel<1024, 1, 1, 16>(sgpe::ColArgsT<float>)"
    copy = "__amd_rocclr_copyBuffer"
    _counter_db(str(tmp_path / "kf.db"), "FETCH_SIZE", [(col, [4000.0, 4400.0])] * 3)
    _counter_db(str(tmp_path / "kw.db"), "WRITE_SIZE", [(col, [8192.0, 8192.0])] * 3)
    _counter_db(str(tmp_path / "cf.db"), "FETCH_SIZE", [(copy, [65536.0, 65536.0])] * 5)      # half of 256 MiB
    _counter_db(str(tmp_path / "cw.db"), "WRITE_SIZE", [(copy, [131072.0, 131072.0])] * 5)
    rec = ps.traffic_record(*(str(tmp_path / f"{n}.db") for n in ("kf", "kw", "cf", "cw")))
    assert rec["calibration"]["fetch_scale"] == 2.0 and rec["calibration"]["write_scale"] == 1.0
    k = rec["kernels"]["col_pass"]
    assert k["dispatches"] == 3
    assert k["read_bytes"] == 8400 * 1024 * 2 and k["written_bytes"] == 16384 * 1024
    assert abs(k["ratio_to_alg"] - (8400 * 2048 + 16384 * 1024) / (32 << 20)) < 1e-12
    json.dumps(rec)
