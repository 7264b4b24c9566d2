"""bench.py's command line on a machine without a GPU: only the argument handling runs."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_workloads_are_declared():
    sys.path.insert(0, ROOT)
    import bench
    assert {"search_1000x1000_1e7", "batch_256maps_1e6", "precision_2000x2000_1e8", "refine_1000x1000_1e6",
            "paper_table3_151x500_2e7", "plain_100x128_1e4"} <= set(bench.WORKLOADS)
    w = bench.WORKLOADS["search_1000x1000_1e7"]
    assert (w["T"], w["F"], w["n"]) == (1000, 1000, 10_000_000)
