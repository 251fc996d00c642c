"""fcs_simulate_events_noalloc (through the C ABI) against fcs_simulate_events
on the same inputs: two calls in a row, the second on a smaller batch, in
both cell-output forms; an asynchronous call; and the size limit of its
scratch array."""
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
def sim(torch_cuda):
    from paper_2103_14737_amd.fcs import Simulator
    s = Simulator(0)
    s.load_geometry(W.make_geometry())
    s.load_parametrization(W.make_param())
    yield s
    s.close()


def _np(x):
    return x.cpu().numpy()


def _dev(w, torch):
    from paper_2103_14737_amd.fcs import particles_to_device
    return particles_to_device(w.particles), torch.from_numpy(w.event_offsets).cuda()


def _buffers(torch, n_events, n_tasks, cells, hits, n_cells, dense):
    d = "cuda"
    out = {"cell_ids": torch.full((cells,), -7, dtype=torch.int64, device=d),
           "cell_e": torch.full((cells,), -7.0, dtype=torch.float32, device=d),
           "event_cell_offsets": torch.full((n_events + 1,), -7, dtype=torch.int64, device=d),
           "counts": torch.full((n_tasks,), -7, dtype=torch.int32, device=d),
           "elayer": torch.full((n_tasks,), -7.0, dtype=torch.float32, device=d)}
    if hits:
        for k, dt in (("hit_eta", torch.float32), ("hit_phi", torch.float32),
                      ("hit_e", torch.float32), ("hit_cell", torch.int32)):
            out[k] = torch.full((hits,), -7, dtype=dt, device=d)
        out["task_hit_offsets"] = torch.full((n_tasks + 1,), -7, dtype=torch.int64, device=d)
    if dense:
        out["cells"] = torch.full((n_events, n_cells), -7.0, dtype=torch.float32, device=d)
    return out


def _compare(ref, got, with_hits, dense, label):
    st_r, st_g = ref["stats"], got["stats"]
    for k in ("n_hits", "n_hits_out_of_acceptance", "n_cells_nonzero", "n_tasks"):
        assert st_r[k] == st_g[k], (label, k)
    nnz = st_r["n_cells_nonzero"]
    for k in ("counts", "event_cell_offsets"):
        assert np.array_equal(_np(ref[k]), _np(got[k])), (label, k)
    assert np.array_equal(_np(ref["elayer"]).view(np.uint32), _np(got["elayer"]).view(np.uint32)), label
    assert np.array_equal(_np(ref["cell_ids"][:nnz]), _np(got["cell_ids"][:nnz])), label
    a = _np(ref["cell_e"][:nnz]).astype(np.float64)
    b = _np(got["cell_e"][:nnz]).astype(np.float64)
    assert np.all(np.abs(a - b) <= np.maximum(REL * np.abs(a), ABS)), label
    if with_hits:
        n = st_r["n_hits"]
        assert np.array_equal(_np(ref["task_hit_offsets"]), _np(got["task_hit_offsets"])), label
        for k in ("hit_eta", "hit_phi", "hit_e", "hit_cell"):
            assert np.array_equal(_np(ref[k][:n]).view(np.uint32), _np(got[k][:n]).view(np.uint32)), (label, k)
    if dense:
        a = _np(ref["cells"]).astype(np.float64)
        b = _np(got["cells"]).astype(np.float64)
        assert np.all(np.abs(a - b) <= np.maximum(REL * np.abs(a), ABS)), label
        assert np.array_equal(a != 0, b != 0), label


def _run_pair(sim, torch, w, base, with_hits, dense, label):
    dp, doff = _dev(w, torch)
    outputs = ("compact", "counts", "elayer") + (("hits",) if with_hits else ()) + \
        (("dense",) if dense else ())
    q = sim.query_sizes(dp, doff, w.seed, event_index_base=base,
                        hit_energy_scale=w.hit_energy_scale)
    L = sim.n_layers
    n_tasks = w.n_particles * L
    kw = dict(event_index_base=base, outputs=outputs, hit_energy_scale=w.hit_energy_scale,
              cell_capacity=q["max_cells"], hit_capacity=q["n_hits"])
    ref = sim.simulate_events(dp, doff, w.seed,
                              out=_buffers(torch, w.n_events, n_tasks, q["max_cells"],
                                           q["n_hits"] if with_hits else 0, sim.n_cells, dense),
                              **kw)
    got = sim.simulate_events(dp, doff, w.seed, noalloc=True,
                              out=_buffers(torch, w.n_events, n_tasks, q["max_cells"],
                                           q["n_hits"] if with_hits else 0, sim.n_cells, dense),
                              **kw)
    torch.cuda.synchronize()
    print(f"[noalloc] {label}: {got['stats']['n_hits']} hits, "
          f"{got['stats']['n_cells_nonzero']} cells", flush=True)
    _compare(ref, got, with_hits, dense, label)


def test_noalloc_matches_the_allocating_call(sim, torch_cuda):
    """Two no-allocation calls in a row, the second on a smaller batch (the
    scratch array keeps the first call's contents), each against
    fcs_simulate_events on the same inputs; then the same with the dense
    output (the accumulator is then the caller's buffer)."""
    big = W.subset_events(W.hard_scatter(), 20, 6)
    small = W.subset_events(W.single_particle_sweep(), 300, 40)
    _run_pair(sim, torch_cuda, big, 20, True, False, "hard scatter[20:26], hits")
    _run_pair(sim, torch_cuda, small, 300, False, False, "sweep[300:340]")
    _run_pair(sim, torch_cuda, big, 20, False, True, "hard scatter[20:26], dense")
    _run_pair(sim, torch_cuda, small, 300, True, True, "sweep[300:340], dense and hits")


def test_noalloc_asynchronous(sim, torch_cuda):
    torch = torch_cuda
    w = W.subset_events(W.single_particle_sweep(), 1000, 30)
    dp, doff = _dev(w, torch)
    q = sim.query_sizes(dp, doff, w.seed, event_index_base=1000)
    L = sim.n_layers
    ref = sim.simulate_events(dp, doff, w.seed, event_index_base=1000,
                              outputs=("compact", "counts", "elayer"),
                              out=_buffers(torch, w.n_events, w.n_particles * L, q["max_cells"],
                                           0, sim.n_cells, False),
                              cell_capacity=q["max_cells"])
    out = _buffers(torch, w.n_events, w.n_particles * L, q["max_cells"], 0, sim.n_cells, False)
    for _ in range(2):
        sim.simulate_events(dp, doff, w.seed, event_index_base=1000, noalloc=True,
                            async_launch=True, outputs=("compact", "counts", "elayer"), out=out,
                            cell_capacity=q["max_cells"])
    st = sim.synchronize()
    torch.cuda.synchronize()
    assert st["n_calls"] == 2 and st["n_hits"] == 2 * ref["stats"]["n_hits"]
    got = dict(out)
    got["stats"] = dict(ref["stats"])
    _compare(ref, got, False, False, "asynchronous")


def test_noalloc_refuses_what_it_cannot_do(sim, torch_cuda):
    """Batches beyond the scratch array, host buffers and the per-event form
    are refused with FCS_E_INVALID_ARG before any device work."""
    from paper_2103_14737_amd.fcs import FCS_E_INVALID_ARG, FcsError
    torch = torch_cuda
    big = W.pileup()          # 270,000 particles: 6.5 M tasks, far beyond 64 MiB
    dp, doff = _dev(big, torch)
    out = _buffers(torch, big.n_events, 1, 16, 0, sim.n_cells, False)
    with pytest.raises(FcsError) as e:
        sim.simulate_events(dp, doff, big.seed, noalloc=True, outputs=("compact",), out=out,
                            cell_capacity=16, hit_energy_scale=big.hit_energy_scale)
    assert e.value.code == FCS_E_INVALID_ARG and "scratch" in str(e.value)
    w = W.subset_events(W.single_particle_sweep(), 0, 5)
    with pytest.raises(FcsError) as e:
        sim.simulate_events(w.particles, w.event_offsets, w.seed, noalloc=True,
                            outputs=("compact",), cell_capacity=1000)
    assert e.value.code == FCS_E_INVALID_ARG and "device inputs" in str(e.value)
    dp, doff = _dev(w, torch)
    with pytest.raises(FcsError) as e:
        sim.simulate_events(dp, doff, w.seed, noalloc=True, mode="per_event", outputs=("compact",),
                            out=_buffers(torch, 5, 5 * 24, 1000, 0, sim.n_cells, False),
                            cell_capacity=1000)
    assert e.value.code == FCS_E_INVALID_ARG
    # the context still works afterwards
    _run_pair(sim, torch, w, 0, False, False, "after refusals")
