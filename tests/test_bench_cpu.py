"""Host logic of bench.py that runs without a GPU: the one-GPU guard and the
oracle baseline (one thread, then independent threads over event ranges)."""
import os
import subprocess
import sys

from paper_2103_14737_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_oracle_baseline_threads_cover_the_workload():
    sys.path.insert(0, ROOT)
    import bench
    w = W.subset_events(W.single_particle_sweep(), 100, 240)
    rec = bench.oracle_baseline(w, W.make_geometry(), W.make_param(), max_threads=4,
                                budget_one=0.0, budget_all=0.0)
    # the threads' event ranges sum to the one-thread pass (checked inside)
    assert rec["kind"] == "oracle" and rec["unit"] == "hits/s"
    assert rec["cores"] == min(4, len(os.sched_getaffinity(0)))
    assert rec["value"] > 0 and rec["one_core"]["value"] > 0 and rec["one_core"]["cores"] == 1
    assert "event ranges" in rec["sample"]
