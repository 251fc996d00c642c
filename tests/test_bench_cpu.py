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
    import oracle
    w = W.subset_events(W.single_particle_sweep(), 100, 240)
    geo, par = W.make_geometry(), W.make_param()
    rec = bench.oracle_baseline(w, geo, par, max_threads=4, one_core_events=30,
                                budget_one=0.0, budget_all=0.0)
    # the threads' event ranges cover the workload: their hits sum to one
    # pass over the whole of it
    whole = oracle.simulate(oracle.Geometry(geo), oracle.Param(par), w.particles,
                            w.event_offsets, w.seed, event_index_base=100)
    assert rec["hits_per_pass"] == whole["n_hits_total"]
    assert rec["kind"] == "oracle" and rec["unit"] == "hits/s"
    assert rec["cores"] == min(4, len(os.sched_getaffinity(0)))
    assert rec["nproc"] == len(os.sched_getaffinity(0))
    assert rec["value"] > 0 and rec["one_core"]["value"] > 0 and rec["one_core"]["cores"] == 1
    assert "events 0-29" in rec["one_core"]["sample"] and "event ranges" in rec["sample"]
