"""Host logic of bench.py that needs no GPU: the summaries of rocprofv3 databases (on small synthetic databases with
the columns of rocprofv3's kernel view) and the one-GPU guard."""
import contextlib
import importlib.util
import io
import os
import sqlite3
import subprocess
import sys

from conftest import ROOT


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _db(path, launches):
    """A kernel view of dispatches (name, grid, workgroup, duration ns, gap ns to the next one)."""
    c = sqlite3.connect(path)
    c.execute("create table kernels(name text, grid_x int, workgroup_x int, start int, end int, duration int)")
    t = 0
    for nm, gx, wx, d, gap in launches:
        c.execute("insert into kernels values(?,?,?,?,?,?)", (nm, gx, wx, t, t + d, d))
        t += d + gap
    c.commit()
    c.close()


def test_solve_trace_summary_keeps_the_solves_after_the_autotuner(tmp_path):
    ns = "void excmg::(anonymous namespace)::"
    launches = [
        (ns + "cg1_iter_kernel<2, 4>(excmg::Sweep)", 32768, 256, 99_000, 1_000),  # an autotuner trial: dropped
        (ns + "tune_selfred_kernel(excmg::CgState*)", 256, 256, 2_000, 1_000),
        ("delay_kernel(long long)", 64, 64, 120_000, 0),
        (ns + "cg1_iter_kernel<2, 4>(excmg::Sweep)", 32768, 256, 8_000, 2_000),
        (ns + "cg1_iter_kernel<2, 4>(excmg::Sweep)", 32768, 256, 8_000, 2_000),
        (ns + "cg1_iter_kernel<2, 4>(excmg::Sweep)", 32768, 256, 1_000, 2_000),  # after convergence: not working
        (ns + "cg_selfred_a_kernel<double, 3, true, 4>(excmg::Sweep)", 131072, 256, 13_000, 500),
        (ns + "exp_finite_kernel<false>(excmg::Grid)", 1024, 256, 70_000, 0),  # not a CG launch: not listed
        (ns + "cg_pass_b_kernel<double, 3, true, 16>(excmg::Sweep)", 262144, 1024, 950_000, 0),
        ("last", 1, 1, 1_000, 0),
    ]
    db = str(tmp_path / "trace.db")
    _db(db, launches)
    out = io.StringIO()
    with contextlib.redirect_stdout(out):
        _bench().solve_trace_summary(db)
    lines = out.getvalue().splitlines()
    assert lines[0] == "solve launches after the autotuner: 7 dispatches"
    # per line: kernel name (may hold spaces), grid, workgroup, calls, working, working average (us), gap (us)
    by_grid = {int(ln.split()[-6]): ln.split()[-5:] for ln in lines[2:]}
    assert sorted(by_grid) == [32768, 131072, 262144]
    assert lines[2].startswith("cg1_iter_kernel<2, 4>")
    wg, calls, working, avg, gap = by_grid[32768]
    assert (wg, calls, working) == ("256", "3", "2")
    assert float(avg) == 8.0 and float(gap) == 2.0
    assert by_grid[131072][1:] == ["1", "1", "13.00", "0.50"]
    assert 1024 not in by_grid


def test_trace_summary_groups_by_kernel_and_grid(tmp_path):
    ns = "void excmg::(anonymous namespace)::"
    db = str(tmp_path / "trace.db")
    _db(db, [(ns + "cg_pass_b_kernel<double, 3, true, 16>(excmg::Sweep)", 262144, 1024, 950_000, 0)] * 3 +
        [(ns + "cg_pass_b_kernel<double, 3, true, 16>(excmg::Sweep)", 262144, 1024, 500_000, 0)])
    c = sqlite3.connect(db)
    c.execute("create table counters_collection(kernel_name text, grid_size int, counter_name text, value real)")
    c.commit()
    c.close()
    out = io.StringIO()
    with contextlib.redirect_stdout(out):
        _bench().trace_summary(db)
    text = out.getvalue()
    assert "kernel trace: 4 dispatches" in text
    row = [ln for ln in text.splitlines() if ln.startswith("cg_pass_b_kernel")][0].split()
    # 4 calls, 3.35 ms in all (average 837.5 us), 3 working (the short launch is below 0.9 of the longest) at 950 us
    assert row[-5:] == ["4", "3.350", "837.50", "3", "950.00"]


def test_bench_runs_on_one_gpu_only():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
