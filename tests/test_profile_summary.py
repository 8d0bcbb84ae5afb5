"""The counter summaries turn FETCH_SIZE / WRITE_SIZE into bytes by scaling
with what the same counter reads for a 1 GiB copy: checked on a synthetic
database with the tables and columns the rocprofv3 output provides."""

import sqlite3

from paper_1904_08616_amd import profile_summary as ps


def make_db(path, counter, copy_kib, kernel_kib):
    c = sqlite3.connect(path)
    c.execute("create table kernels (dispatch_id integer, name text, duration integer, grid_x integer, "
              "workgroup_x integer, lds_size integer, vgpr_count integer, scratch_size integer)")
    c.execute("create table pmc_events (dispatch_id integer, name text, counter_name text, counter_value real)")
    rows = [(1, "__amd_rocclr_copyBuffer", 400000, 131072, 512, 0, 8, 0, copy_kib)]
    for d in range(2, 6):
        rows.append((d, "void dirac::k_dslash_stream<0, 0, 18, false, 0, 256>(dirac::DslashArgs)", 33000 + d,
                     65536, 256, 122880, 128, 0, kernel_kib + d))
    for r in rows:
        c.execute("insert into kernels values (?, ?, ?, ?, ?, ?, ?, ?)", r[:8])
        c.execute("insert into pmc_events values (?, ?, ?, ?)", (r[0], r[1], counter, r[8]))
    c.commit()
    c.close()


def test_counter_report_scales_by_the_copy(tmp_path):
    f, w = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    # FETCH_SIZE counts a 1 GiB copy as half its bytes (128-byte requests weighed as 64), WRITE_SIZE exactly
    make_db(f, "FETCH_SIZE", 524288.0, 1000.0)
    make_db(w, "WRITE_SIZE", 1048576.0, 500.0)
    text, res = ps.counter_report(f, w, "k_dslash_stream", "fetch cmd", "write cmd")
    assert abs(res["FETCH_SIZE"]["scale"] - 2.0) < 1e-12
    assert abs(res["WRITE_SIZE"]["scale"] - 1.0) < 1e-12
    fetch_kib = sum(1000.0 + d for d in range(2, 6)) / 4
    write_kib = sum(500.0 + d for d in range(2, 6)) / 4
    assert abs(res["traffic_bytes"] - (2.0 * fetch_kib + write_kib) * 1024) < 1e-6
    assert "fetch cmd" in text and "write cmd" in text


def test_trace_report_lists_each_kernel(tmp_path):
    f = str(tmp_path / "t.db")
    make_db(f, "FETCH_SIZE", 524288.0, 1000.0)
    text = ps.trace_report(f, "the command")
    assert text.startswith("command: the command")
    line = [l for l in text.splitlines() if "k_dslash_stream" in l][0]
    assert line.split()[0] == "4"  # calls
    assert abs(float(line.split()[2]) - (33002 + 33003 + 33004 + 33005) / 4) <= 0.5  # average, printed rounded
