"""Host-side checks of the benchmark script and the profile summary tool
(CPU only): the one-GPU guard, the multi-process oracle baseline over
independent instances, the one-core oracle solver baseline, and per-dispatch
counter averages."""

import os
import sqlite3
import subprocess
import sys

import numpy as np

from paper_2011_11880_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_parallel_oracle_baseline_counts_every_instance():
    sys.path.insert(0, ROOT)
    import bench
    net = synth.tiny_grid(3)
    I = 6
    ls = np.exp(0.1 * np.random.default_rng(1).normal(size=(I, net.n_load)))
    ps = np.ones((I, net.n_pv))
    out = np.full(I, -1, np.int32)
    out[3:] = synth.contingencies(net, 3, seed=2)
    Y = synth.random_states(net, I, seed=3)
    items = [(ls[k] if k < 3 else None, ps[k] if k < 3 else None, int(out[k]), Y[k])
             for k in range(I)]
    r = bench.cpu_baseline_parallel(net, items, 30.0, "instances")
    assert r["kind"] == "oracle" and r["unit"] == "evals/s" and r["value"] > 0
    assert 1 <= r["cores"] <= min(16, I)
    assert r["sample"].startswith(f"{I} of the {I} instances")
    # one grid and state per item, no base network
    r = bench.cpu_baseline_parallel(None, [(net, Y[0]), (net, Y[1])], 30.0, "grids")
    assert r["sample"].startswith("2 of the 2 grids")


def test_counter_summary_averages_per_dispatch(tmp_path):
    from paper_2011_11880_amd import rocprof_summary as R
    db = tmp_path / "run_results.db"
    c = sqlite3.connect(db)
    c.execute("create table counters_collection (kernel_name text, dispatch_id int, "
              "counter_name text, value real)")
    rows = [("k_a(int)", 1, "FETCH_SIZE", 10.0), ("k_a(int)", 1, "FETCH_SIZE", 6.0),
            ("k_a(int)", 2, "FETCH_SIZE", 20.0), ("k_b(int)", 3, "FETCH_SIZE", 99.0),
            ("k_a(int)", 1, "SQ_WAVES", 4.0), ("k_a(int)", 2, "SQ_WAVES", 8.0)]
    c.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    c.commit()
    c.close()
    out = R.counters(str(db), "k_a")
    # per dispatch, values of one counter are summed (over the device's units)
    assert out["FETCH_SIZE"] == ((16.0 + 20.0) / 2, 2)
    assert out["SQ_WAVES"] == (6.0, 2)


def test_solver_baseline_reports_the_oracle_loop():
    sys.path.insert(0, ROOT)
    import bench
    net = synth.tiny_grid(3)
    y0 = synth.random_states(net, seed=4)
    calls = []

    def run(O):
        calls.append(O)
        _, norms, _ = O.newton(net, y0, tol=1e-10, max_iter=3)
        return len(norms) - 1, norms[-1]
    r = bench.cpu_baseline_solve(run, "oracle Newton on the tiny grid")
    assert len(calls) == 1 and calls[0].__name__ == "oracle.oracle"
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["total_ms"] > 0
    assert 0 <= r["iterations"] <= 3 and np.isfinite(r["final_mismatch"])
    assert r["sample"] == "oracle Newton on the tiny grid"


def test_traffic_counter_takes_the_last_dispatches(tmp_path):
    from paper_2011_11880_amd import rocprof_summary as R
    db = tmp_path / "run_results.db"
    c = sqlite3.connect(db)
    c.execute("create table counters_collection (kernel_name text, dispatch_id int, "
              "counter_name text, value real)")
    # an autotuning phase (dispatches 1-3) before two timed launches (7, 9)
    rows = [("k_a(int)", d, "WRITE_SIZE", v) for d, v in
            ((1, 50.0), (2, 70.0), (3, 90.0), (7, 10.0), (9, 4.0), (9, 8.0))]
    rows.append(("k_b(int)", 8, "WRITE_SIZE", 1000.0))
    c.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    c.commit()
    c.close()
    assert R.counter_per_dispatch(str(db), "WRITE_SIZE", "k_a", last=2) == (11.0, 2)
    assert R.counter_per_dispatch(str(db), "WRITE_SIZE", "k_a") == ((50 + 70 + 90 + 10 + 12) / 5, 5)


def test_host_cpu_record():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.host_cpu()
    assert 1 <= h["usable_cores"] <= h["cpus"]
    assert h["model"] is None or isinstance(h["model"], str)


def test_fp64_summary_and_bench_rate(tmp_path, monkeypatch):
    """The FP64 counter summary scales the per-dispatch instruction count by
    64 lanes; the bench turns it into a rate only for the kernel source it
    was taken on and the same launch size."""
    from paper_2011_11880_amd import rocprof_summary as R
    db = tmp_path / "run_results.db"
    c = sqlite3.connect(db)
    c.execute("create table counters_collection (kernel_name text, dispatch_id int, "
              "counter_name text, value real)")
    rows = [("k_eval_batch<a>", 1, "SQ_INSTS_VALU_FLOPS_FP64", 100.0),
            ("k_eval_batch<a>", 1, "SQ_INSTS_VALU_FLOPS_FP64", 50.0),
            ("k_eval_batch<a>", 2, "SQ_INSTS_VALU_FLOPS_FP64", 250.0),
            ("k_other", 3, "SQ_INSTS_VALU_FLOPS_FP64", 7.0)]
    c.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    c.commit()
    c.close()
    out = tmp_path / "fp64.json"
    R.main(["fp64", str(db), "--kernel", "k_eval_batch", "--units", "10", "--out", str(out)])
    import json
    d = json.load(open(out))
    assert d["sq_insts_valu_flops_fp64_per_dispatch"] == 200.0
    assert d["fp64_flops_per_launch"] == 64 * 200.0 and d["dispatches"] == 2
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    os.replace(out, tmp_path / "profiles" / "fp64.json")
    r = bench.fp64_rate("fp64.json", 10, 2.0)
    assert abs(r["fp64_tflops"] - 64 * 200.0 / 2e-3 / 1e12) < 1e-18
    assert bench.fp64_rate("fp64.json", 11, 2.0) == {"fp64_tflops": None}
    assert bench.fp64_rate("missing.json", 10, 2.0) == {"fp64_tflops": None}
