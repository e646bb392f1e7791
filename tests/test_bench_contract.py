"""Host-side checks of the benchmark's contract (no GPU): more than one GPU
is refused with a JSON message, and the algorithmic byte counts reproduce
the figures the workload definitions give for the 128^3 factor and the
power-law matrix (4(n+1) + nnz(4+s) + 2nks for a forward solve)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_solve_bytes_match_the_workload_figures():
    # 128^3 7-point lower factor: n = 2,097,152, nnz = 8,339,456 (FP64, k = 1)
    n = 128 ** 3
    nnz = n + 3 * n - 3 * 128 * 128
    assert nnz == 8_339_456
    assert bench.bytes_solve(n, nnz, 1, 8) == 142_016_516        # 142.0 MB
    assert round(bench.bytes_solve(n, nnz, 1, 4) / 1e6, 1) == 91.9
    assert round(bench.bytes_solve(n, nnz, 64, 8) / 1e9, 3) == 2.256
    # power-law 1M with about 8.97M stored entries, 64 right-hand sides
    assert round(bench.bytes_solve(1_000_000, 8_970_000, 64, 8) / 1e9, 3) == 1.136


def test_transposed_and_adjoint_bytes_are_consistent():
    n, nnz, k, s = 1000, 4000, 3, 8
    # the transposed solve's algorithmic bytes are the system's own (pattern,
    # values, G read, Y written): the successor-list indirection is the
    # implementation's extra, not counted
    assert bench.bytes_solve_t(n, nnz, k, s) == bench.bytes_solve(n, nnz, k, s)
    assert bench.bytes_grad_vals(n, nnz, k, s) == 4 * (n + 1) + nnz * (4 + s) + 2 * n * k * s
    assert bench.bytes_apply_mt(n, k, s, 0) == 2 * n * k * s + 4 * (n + 1)


def test_sections_and_headline_flags():
    """Unknown sections are refused; the batch is the default headline."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--sections", "nope"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "unknown sections" in r.stderr
    assert bench.SECTIONS[0] == "batch"


def test_batched_bytes_add_solves_and_candidates():
    n, nnz = 1000, 4000
    assert bench.bytes_levels(n, nnz) == 4 * (n + 1) + 4 * (nnz - n) + 4 * n
    r = bench.roof(8e9, 2.0, "k", levels=100, hop_ns=600.0)
    assert abs(r["achieved"] - 4000.0) < 1e-9 and abs(r["frac"] - 0.5) < 1e-12
    assert abs(r["latency_floor_ms"] - 0.06) < 1e-12 and abs(r["bandwidth_floor_ms"] - 1.0) < 1e-12


def test_traffic_is_reported_only_for_the_profiled_configuration(tmp_path, monkeypatch):
    """HBM traffic from the committed counter runs is attached to the bench
    line only when the solve sources, block size and staging of outside
    values are those the counters were taken with."""
    tj = tmp_path / "profiles" / "traffic.json"
    tj.parent.mkdir()
    key = "lap3d_128:f64:k_solve_sf<double, true, 1>"
    tj.write_text(json.dumps({key: {"src_hash": "abc", "stage_outside": "off", "block_rows": 4096,
                                    "hbm_bytes_per_launch": 5.0e8}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic(key, "abc", "off", 4096) == 5.0e8
    assert bench.load_traffic(key, "abd", "off", 4096) is None      # sources changed
    assert bench.load_traffic(key, "abc", "on", 4096) is None       # other staging
    assert bench.load_traffic(key, "abc", "off", 2048) is None      # other block size
    assert bench.load_traffic("other", "abc", "off", 4096) is None
    tj.write_text("not json")
    assert bench.load_traffic(key, "abc", "off", 4096) is None



def test_roofline_kernel_names_follow_the_schedule():
    # the names the profiler reports for the kernel a plan launches: the
    # walk has no column-count parameter; sync-free blocks take four
    # columns per chain when the chain has more than one, the level-by-level
    # solve when the solve has more than one column
    assert bench.solve_kernel("walk", "double", False, 64, 1) == "k_solve_walk<double, false>"
    assert bench.solve_kernel("walk", "float", True, 1, 1) == "k_solve_walk<float, true>"
    assert bench.solve_kernel("syncfree", "double", False, 64, 1) == "k_solve_sf<double, false, 1>"
    assert bench.solve_kernel("syncfree", "double", True, 64, 4) == "k_solve_sf<double, true, 4>"
    assert bench.solve_kernel("level", "double", False, 1, 1) == "k_solve_level<double, false, 1>"
    assert bench.solve_kernel("level", "float", True, 32, 1) == "k_solve_level<float, true, 4>"
    # the names appear in the library's own launch code
    src = open(os.path.join(ROOT, "paper_2609_40159_amd", "csrc", "solve.hip")).read()
    for frag in ("k_solve_walk<double, false>", "k_solve_walk<float, true>",
                 "k_solve_sf<T, TRANS, 4>", "k_solve_sf<T, TRANS, 1>",
                 "k_solve_level<T, TRANS, 4>", "k_solve_level<T, TRANS, 1>"):
        assert frag in src, frag
