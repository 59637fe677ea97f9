"""Host-side check of the rocprofv3 summary tool on small synthetic result files:
timed-region window, counter calibration and measured/algorithmic ratios."""
import json
import sqlite3
import subprocess
import sys

from paper_2211_09958_amd import rocprof_summary as rs

COPY = "__amd_rocclr_copyBuffer"
MARK = "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<unsigned char>>()"
R2C = "void pmx::(anonymous namespace)::k_fft_x_r2c<16>(HIP_vector_type<float, 2u>*, int)"


def make_db(path, counter=None, values=None):
    con = sqlite3.connect(path)
    con.execute("create table kernels (dispatch_id int, name text, grid_y int, duration real)")
    con.execute("create table pmc_events (dispatch_id int, counter_name text, counter_value real)")
    rows = [(1, R2C, 1, 100.0), (2, COPY, 1, 50.0), (3, MARK, 1, 1.0), (4, R2C, 1, 200.0),
            (5, R2C, 3, 600.0), (6, MARK, 1, 1.0), (7, R2C, 1, 999.0)]
    con.executemany("insert into kernels values (?, ?, ?, ?)", rows)
    if counter:
        con.executemany("insert into pmc_events values (?, ?, ?)",
                        [(d, counter, values[d]) for d in values])
    con.commit()
    con.close()


def test_short_names_and_families():
    assert rs.short(R2C) == "k_fft_x_r2c<16>"
    assert rs.family("k_fft_x_r2c<16>", 16) == ("fft_x", "rc_per_buf")
    assert rs.family("k_gather_tile<16, 2>", 16) == ("unkick_vjp", "72P+3r")
    assert rs.family("k_fft_x_r2c<8>", 16) == (None, None)   # another mesh size


def test_window_calibration_and_ratio(tmp_path):
    n = 16
    r, c = 4.0 * n ** 3, 8.0 * n * n * (n // 2 + 1)
    calib = 2.0 ** 20
    # counters in KiB: the copy of calib bytes reads 0.5x on FETCH, 1x on WRITE; the
    # timed r2c dispatches move exactly their algorithmic bytes (r in, c out per buffer)
    fetch = {2: 0.5 * calib / 1024, 4: 0.5 * r / 1024, 5: 0.5 * 3 * r / 1024, 1: 1.0, 7: 1.0,
             3: 0.0, 6: 0.0}
    write = {2: calib / 1024, 4: c / 1024, 5: 3 * c / 1024, 1: 1.0, 7: 1.0, 3: 0.0, 6: 0.0}
    kt, fe, wr = tmp_path / "kt.db", tmp_path / "f.db", tmp_path / "w.db"
    make_db(kt)
    make_db(fe, "FETCH_SIZE", fetch)
    make_db(wr, "WRITE_SIZE", write)
    rows, marked = rs.timed_window(rs.dispatches(str(kt)))
    assert marked and [d[0] for d in rows] == [4, 5]
    assert abs(rs.calibration(rs.dispatches(str(fe), "FETCH_SIZE"), calib)[0] - 2.0) < 1e-12
    out = tmp_path / "out"
    subprocess.run([sys.executable, "-m", "paper_2211_09958_amd.rocprof_summary", "--kt", str(kt),
                    "--fetch", str(fe), "--write", str(wr), "--ptcl", "8", "--mesh", str(n),
                    "--workload", "t", "--out", str(out), "--calib-bytes", str(calib)],
                   check=True, capture_output=True, timeout=120)
    t = json.loads((out / "traffic.json").read_text())
    assert abs(t["families"]["fft_x"]["measured_over_algorithmic"] - 1.0) < 1e-9
    assert t["families"]["fft_x"]["dispatches"] == 2
    md = (out / "kernel-trace_all-kernels_t.md").read_text()
    assert "| fft_x | 2 | 0.00 |" in md    # 800 ns over the two timed dispatches


def test_source_hash_ignores_comments_only():
    """Counter figures stay valid across comment edits, not across code edits."""
    base = "__global__ void k(float* p) {  // doubles\n    p[0] *= 2.f;  /* in place */\n}\n"
    reworded = "// a kernel\n__global__ void k(float* p) {  // twice the value\n\n    p[0] *= 2.f;\n}\n"
    changed = "__global__ void k(float* p) {\n    p[0] *= 3.f;\n}\n"
    quoted = 'const char* s = "a // b"; char c = \'/\';'
    assert rs.code_only(base) == rs.code_only(reworded)
    assert rs.code_only(base) != rs.code_only(changed)
    assert rs.code_only(quoted) == quoted
