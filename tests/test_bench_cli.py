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


def test_every_workload_has_a_runner():
    """Each declared workload names a kind that main() dispatches, and the map-formation and
    background legs segment and slide the strain the same way (the pipeline forms the maps whose
    formation is timed on its own)."""
    sys.path.insert(0, ROOT)
    import bench
    src = open(os.path.join(ROOT, "bench.py")).read()
    for name, w in bench.WORKLOADS.items():
        assert f'"{w["kind"]}": run_' in src, name
    assert {"maxdelay_1000x1000_1e6x16", "tmid_1000x1000_1e7", "mapform_1000x1000_256slides",
            "background_256slides_1e6"} <= set(bench.WORKLOADS)
    mf, bg = bench.WORKLOADS["mapform_1000x1000_256slides"], bench.WORKLOADS["background_256slides_1e6"]
    for k in ("fs", "M", "T", "k_lo", "F", "nb", "n_slides", "slide_cols", "seed"):
        assert mf[k] == bg[k], k
    # 1 s columns at a 0.5 s stride covering T columns, bins of 1 Hz from 100 Hz
    assert mf["M"] / mf["fs"] == 1.0 and mf["k_lo"] * mf["fs"] / mf["M"] == 100.0
