"""Jobs sharing one GPU: several library contexts, each driven by its own
host thread and torch stream, simulate their own events at the same time.
Every context's results equal the oracle's for its events (counts and cell
ids exact, energies within tolerance), in both launch forms, whatever the
other contexts run meanwhile."""
import threading

import numpy as np
import pytest

from paper_2103_14737_amd import workloads as W

pytestmark = pytest.mark.gpu
REL, ABS = 1e-5, 1e-3


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test on a host without a GPU"
    return torch


@pytest.fixture(scope="module")
def jobs(oracle_lib, geom_full, param_full):
    sweep = W.single_particle_sweep()
    ws = [W.subset_events(sweep, 200 * k, 40) for k in range(3)]
    ws.append(W.subset_events(W.hard_scatter(), 7, 2))
    refs = [oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                                event_index_base=w.notes["event_index_base"],
                                hit_energy_scale=w.hit_energy_scale) for w in ws]
    return ws, refs


@pytest.mark.parametrize("mode", ["batched", "per_event"])
def test_contexts_used_at_once_from_threads(torch_cuda, jobs, mode):
    torch = torch_cuda
    from paper_2103_14737_amd.fcs import Simulator, particles_to_device
    ws, refs = jobs
    geo, par = W.make_geometry(), W.make_param()
    sims, inputs, streams = [], [], []
    for w in ws:
        s = Simulator(0)
        s.load_geometry(geo)
        s.load_parametrization(par)
        sims.append(s)
        inputs.append((particles_to_device(w.particles),
                       torch.from_numpy(w.event_offsets).cuda()))
        streams.append(torch.cuda.Stream())
    torch.cuda.synchronize()
    results = [[] for _ in ws]
    errors = []
    start = threading.Barrier(len(ws))
    keys = ("counts", "event_cell_offsets", "cell_ids", "cell_e")

    def job(k):
        w = ws[k]
        dp, doff = inputs[k]
        try:
            with torch.cuda.stream(streams[k]):
                start.wait()
                for _ in range(3):
                    r = sims[k].simulate_events(dp, doff, w.seed,
                                                event_index_base=w.notes["event_index_base"],
                                                mode=mode, outputs=("compact", "counts"),
                                                hit_energy_scale=w.hit_energy_scale)
                    results[k].append({"stats": r["stats"]} |
                                      {key: r[key].cpu().numpy() for key in keys})
        except BaseException as e:  # reported below
            errors.append(e)

    threads = [threading.Thread(target=job, args=(k,)) for k in range(len(ws))]
    print(f"[sharing] {mode}: {len(ws)} contexts at once", flush=True)
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=100)
    assert not any(t.is_alive() for t in threads), "a job did not finish"
    torch.cuda.synchronize()
    for s in sims:
        s.close()
    assert not errors, errors
    for k, (w, ref) in enumerate(zip(ws, refs)):
        assert len(results[k]) == 3
        for r in results[k]:
            label = f"{w.name} ({mode})"
            assert r["stats"]["n_hits"] == ref["n_hits_total"], label
            assert np.array_equal(r["counts"], ref["n"]), label
            assert np.array_equal(r["event_cell_offsets"], ref["ev_cell_off"]), label
            assert np.array_equal(r["cell_ids"], geo["cell_id"][ref["cell_idx"]]), label
            e = r["cell_e"].astype(np.float64)
            tol = np.maximum(REL * np.abs(ref["cell_e"]), ABS)
            assert np.all(np.abs(e - ref["cell_e"]) <= tol), label
