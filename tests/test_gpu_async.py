"""Asynchronous batched calls (fcs_simulate_events with async_launch and
fcs_synchronize) on the GPU: the same results as synchronous calls, errors
and capacity overflows reported at the synchronization, and a context that
stays clean after a rejected batch."""
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


def _dev(w, torch):
    from paper_2103_14737_amd.fcs import particles_to_device
    return particles_to_device(w.particles), torch.from_numpy(w.event_offsets).cuda()


def _np(x):
    return x.cpu().numpy()


def test_async_matches_sync(sim, torch_cuda, oracle_lib, geom_full, param_full):
    torch = torch_cuda
    full = W.single_particle_sweep()
    batches = [W.subset_events(full, a, n) for a, n in ((0, 300), (300, 500), (800, 37))]
    sync, outs = [], []
    for b in batches:
        dp, doff = _dev(b, torch)
        r = sim.simulate_events(dp, doff, b.seed, event_index_base=b.notes["event_index_base"],
                                outputs=("compact", "counts"))
        torch.cuda.synchronize()
        sync.append({k: _np(v) for k, v in r.items() if k != "stats"} | {"stats": r["stats"]})
    print("[async] synchronous references done", flush=True)
    sim.synchronize()
    for b, s in zip(batches, sync):
        dp, doff = _dev(b, torch)
        cap = int(s["stats"]["n_cells_nonzero"]) + 5
        r = sim.simulate_events(dp, doff, b.seed, event_index_base=b.notes["event_index_base"],
                                outputs=("compact", "counts"), cell_capacity=cap, profile=True,
                                async_launch=True)
        assert r["stats"] is None
        outs.append((r, dp, doff))
    st = sim.synchronize()
    torch.cuda.synchronize()
    print(f"[async] {st}", flush=True)
    assert st["n_calls"] == 3
    assert st["n_hits"] == sum(s["stats"]["n_hits"] for s in sync)
    assert st["n_cells_nonzero"] == sum(s["stats"]["n_cells_nonzero"] for s in sync)
    assert st["n_hits_out_of_acceptance"] == sum(s["stats"]["n_hits_out_of_acceptance"] for s in sync)
    assert st["kernel_ms"] > 0
    for (r, _, _), s in zip(outs, sync):
        off = _np(r["event_cell_offsets"])
        assert np.array_equal(off, s["event_cell_offsets"])
        n = off[-1]
        assert np.array_equal(_np(r["cell_ids"])[:n], s["cell_ids"])
        assert np.array_equal(_np(r["counts"]), s["counts"])
        e, es = _np(r["cell_e"])[:n].astype(np.float64), s["cell_e"].astype(np.float64)
        assert np.all(np.abs(e - es) <= np.maximum(REL * np.abs(es), ABS))
    # the last batch against the oracle directly
    b = batches[2]
    ref = oracle_lib.simulate(geom_full, param_full, b.particles, b.event_offsets, b.seed,
                              event_index_base=b.notes["event_index_base"])
    r = outs[2][0]
    n = int(_np(r["event_cell_offsets"])[-1])
    assert n == ref["n_cells_nonzero"]
    assert np.array_equal(_np(r["counts"]), ref["n"])
    e = _np(r["cell_e"])[:n].astype(np.float64)
    assert np.all(np.abs(e - ref["cell_e"]) <= np.maximum(REL * np.abs(ref["cell_e"]), ABS))


def test_async_errors_reported_at_synchronize(sim, torch_cuda):
    torch = torch_cuda
    from paper_2103_14737_amd.fcs import FCS_E_CAPACITY, FCS_E_INVALID_ARG, FcsError, particles_to_device
    w = W.subset_events(W.single_particle_sweep(), 0, 20)
    bad = w.particles.copy()
    bad["pdg"][7] = 13
    dp, doff = particles_to_device(bad), torch.from_numpy(w.event_offsets).cuda()
    r = sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=10 ** 6,
                            async_launch=True)
    with pytest.raises(FcsError) as e:
        sim.synchronize()
    assert e.value.code == FCS_E_INVALID_ARG and "pdg" in str(e.value)
    print("[async] invalid particle reported", flush=True)
    # a cell capacity that is too small
    dp, doff = _dev(w, torch)
    r = sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=3,
                            async_launch=True)
    with pytest.raises(FcsError) as e:
        sim.synchronize()
    assert e.value.code == FCS_E_CAPACITY
    print("[async] capacity reported", flush=True)
    # the context is clean afterwards: a synchronous call gives the usual result
    r1 = sim.simulate_events(dp, doff, w.seed, outputs=("compact",))
    r2 = sim.simulate_events(dp, doff, w.seed, outputs=("compact",))
    torch.cuda.synchronize()
    assert np.array_equal(_np(r1["cell_ids"]), _np(r2["cell_ids"]))
    assert sim.synchronize()["n_calls"] == 0


def test_particle_count_mismatch_is_rejected(sim, torch_cuda):
    """A particle buffer with more records than the offsets cover is an
    error found on the device; no task of that batch deposits anything."""
    torch = torch_cuda
    from paper_2103_14737_amd.fcs import FCS_E_INVALID_ARG, FcsError, particles_to_device
    w = W.subset_events(W.single_particle_sweep(), 40, 10)
    extra = np.concatenate([w.particles, w.particles[:3]])
    dp, doff = particles_to_device(extra), torch.from_numpy(w.event_offsets).cuda()
    with pytest.raises(FcsError) as e:
        sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=10 ** 6)
    assert e.value.code == FCS_E_INVALID_ARG and "event_offsets" in str(e.value)
    dp, doff = _dev(w, torch)
    a = sim.simulate_events(dp, doff, w.seed, event_index_base=40, outputs=("compact",))
    b = sim.simulate_events(dp, doff, w.seed, event_index_base=40, outputs=("compact",))
    torch.cuda.synchronize()
    assert np.array_equal(_np(a["cell_ids"]), _np(b["cell_ids"]))
    assert np.allclose(_np(a["cell_e"]), _np(b["cell_e"]), rtol=REL, atol=ABS)


def test_async_training_steps_match_synchronous(sim, torch_cuda):
    """simulate_dense and its backward enqueued asynchronously, three steps
    back to back: every step's cells and gradients equal those of a
    synchronous step, and synchronize() then reports no error and does not
    count the adjoint calls."""
    torch = torch_cuda
    from paper_2103_14737_amd.autograd import simulate_dense
    w = W.subset_events(W.single_pion_diff(), 0, 8)
    dp, doff = _dev(w, torch)
    base = sim.simulate_events(dp, doff, w.seed, outputs=("dense", "elayer"))
    el0 = base["elayer"].detach()
    target = base["cells"] * 0.9
    wt0 = torch.from_numpy(W.make_param()["weights"]).cuda()

    def step(async_launch):
        el = el0.clone().requires_grad_()
        wt = wt0.clone().requires_grad_()
        cells = simulate_dense(sim, dp, doff, w.seed, el, wt, async_launch=async_launch)
        loss = torch.nn.functional.mse_loss(cells, target, reduction="sum")
        loss.backward()
        return cells.detach(), el.grad, wt.grad

    ref = step(False)
    torch.cuda.synchronize()
    sim.synchronize()
    outs = [step(True) for _ in range(3)]
    st = sim.synchronize()
    torch.cuda.synchronize()
    assert st["n_calls"] == 3 and st["n_hits"] == 3 * base["stats"]["n_hits"]
    # dense-only calls fold their nonzero-cell counts in the count-reset pass
    assert st["n_cells_nonzero"] == 3 * base["stats"]["n_cells_nonzero"] > 0
    for o in outs:
        for a, b in zip(o, ref):
            a, b = _np(a).astype(np.float64), _np(b).astype(np.float64)
            assert np.count_nonzero(b) > 0
            # same kernels: FP32 and FP64 atomic order only
            assert np.all(np.abs(a - b) <= 1e-5 * np.abs(b) + 1e-7 * np.abs(b).max())


def test_override_errors_reach_synchronize(sim, torch_cuda):
    """A negative layer-energy override is an error of the call: raised by a
    synchronous forward or adjoint call, and by synchronize() after an
    asynchronous dense-only forward call or an asynchronous adjoint call;
    the context is clean afterwards."""
    torch = torch_cuda
    from paper_2103_14737_amd.fcs import FCS_E_INVALID_ARG, FcsError
    w = W.subset_events(W.single_pion_diff(), 0, 8)
    dp, doff = _dev(w, torch)
    base = sim.simulate_events(dp, doff, w.seed, outputs=("dense", "elayer"))
    torch.cuda.synchronize()
    sim.synchronize()
    bad = base["elayer"].detach().clone()
    bad[5] = -1.0
    g = torch.ones(8 * sim.info()["n_cells"], device="cuda")
    with pytest.raises(FcsError) as e:
        sim.simulate_events(dp, doff, w.seed, outputs=("dense",), elayer_override=bad)
    assert e.value.code == FCS_E_INVALID_ARG and "elayer_override" in str(e.value)
    with pytest.raises(FcsError) as e:
        sim.backward(dp, doff, w.seed, g, elayer_override=bad)
    assert e.value.code == FCS_E_INVALID_ARG and "elayer_override" in str(e.value)
    print("[async] synchronous override errors raised", flush=True)
    sim.simulate_events(dp, doff, w.seed, outputs=("dense",), elayer_override=bad, async_launch=True)
    with pytest.raises(FcsError) as e:
        sim.synchronize()
    assert e.value.code == FCS_E_INVALID_ARG and "elayer_override" in str(e.value)
    print("[async] dense-only forward override error reported", flush=True)
    sim.backward(dp, doff, w.seed, g, elayer_override=bad, async_launch=True)
    with pytest.raises(FcsError) as e:
        sim.synchronize()
    assert e.value.code == FCS_E_INVALID_ARG and "elayer_override" in str(e.value)
    print("[async] adjoint override error reported", flush=True)
    el = base["elayer"].detach()
    r = sim.simulate_events(dp, doff, w.seed, outputs=("dense",), elayer_override=el, async_launch=True)
    ge, _ = sim.backward(dp, doff, w.seed, g, elayer_override=el, async_launch=True)
    st = sim.synchronize()
    torch.cuda.synchronize()
    assert st["n_calls"] == 1 and st["n_hits"] == base["stats"]["n_hits"]
    assert torch.count_nonzero(r["cells"]).item() == base["stats"]["n_cells_nonzero"]
    assert torch.isfinite(ge).all().item()


@pytest.mark.parametrize("wgs", [0, 1, 64, -1])
def test_async_calls_into_pinned_host_buffers(sim, torch_cuda, oracle_lib, geom_full, param_full,
                                              wgs):
    """Asynchronous calls that leave their {cell_id, E} lists in pinned host
    buffers (fcs_host_alloc): several batches back to back (the two device
    staging sets used in turn, each copied while the next batch runs), each
    into its own host buffers, all equal to the oracle after the
    synchronization; the last call's buffers overflow and that is reported.
    The copy kernel at the default, one and 64 workgroups, and the
    runtime's copies (-1)."""
    from paper_2103_14737_amd.fcs import FCS_E_CAPACITY, FCS_E_INVALID_ARG, FcsError
    torch = torch_cuda
    geo = W.make_geometry()
    ws = [W.subset_events(W.hard_scatter(), 5 * k, 4) for k in range(3)] + \
         [W.subset_events(W.single_particle_sweep(), 100, 200)]
    bufs, refs = [], []
    for w in ws:
        dp, doff = _dev(w, torch)
        q = sim.query_sizes(dp, doff, w.seed, event_index_base=w.notes["event_index_base"])
        cap = q["max_cells"]
        out = {"cell_ids": sim.host_empty((cap,), np.int64),
               "cell_e": sim.host_empty((cap,), np.float32),
               "event_cell_offsets": sim.host_empty((w.n_events + 1,), np.int64)}
        bufs.append((w, dp, doff, out, cap))
        refs.append(oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                                        event_index_base=w.notes["event_index_base"]))
    for _ in range(2):  # every batch twice: the staging sets alternate
        for w, dp, doff, out, cap in bufs:
            for a in out.values():
                a.fill(-1)
            sim.simulate_events(dp, doff, w.seed, event_index_base=w.notes["event_index_base"],
                                outputs=("compact",), out=out, cell_capacity=cap, async_launch=True,
                                host_outputs=True, host_copy_workgroups=wgs)
        st = sim.synchronize()
        assert st["n_calls"] == len(bufs)
        for (w, _, _, out, _), ref in zip(bufs, refs):
            nnz = ref["n_cells_nonzero"]
            print(f"[async host] {w.name}: {nnz} cells", flush=True)
            assert np.array_equal(out["event_cell_offsets"], ref["ev_cell_off"])
            assert np.array_equal(out["cell_ids"][:nnz], geo["cell_id"][ref["cell_idx"]])
            e = out["cell_e"][:nnz].astype(np.float64)
            assert np.all(np.abs(e - ref["cell_e"]) <= np.maximum(REL * ref["cell_e"], ABS))
    # too small a capacity: the copy stops at the capacity, synchronize reports it
    w, dp, doff, out, cap = bufs[0]
    sim.simulate_events(dp, doff, w.seed, event_index_base=w.notes["event_index_base"],
                        outputs=("compact",), out=out, cell_capacity=10, async_launch=True,
                        host_outputs=True, host_copy_workgroups=wgs)
    with pytest.raises(FcsError) as e:
        sim.synchronize()
    assert e.value.code == FCS_E_CAPACITY
    # pageable host arrays are refused
    plain = {k: np.empty_like(v) for k, v in out.items()}
    with pytest.raises(FcsError) as e:
        sim.simulate_events(dp, doff, w.seed, outputs=("compact",), out=plain, cell_capacity=cap,
                            async_launch=True, host_outputs=True)
    assert e.value.code == FCS_E_INVALID_ARG and "pinned" in str(e.value)


def test_host_copy_flushed_by_other_calls(sim, torch_cuda, oracle_lib, geom_full, param_full):
    """The copy of an asynchronous call's lists to the host is enqueued by the
    next call into the context: a synchronous call, a query and an adjoint
    call in between each take it along, and lists whose host views start
    8 bytes into a pinned allocation (no 16-byte moves) and a capacity equal
    to the compacted total arrive whole."""
    torch = torch_cuda
    geo = W.make_geometry()
    w = W.subset_events(W.hard_scatter(), 7, 3)
    base = w.notes["event_index_base"]
    dp, doff = _dev(w, torch)
    ref = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                              event_index_base=base)
    nnz = ref["n_cells_nonzero"]
    raw = {"cell_ids": sim.host_empty((nnz + 1,), np.int64),
           "cell_e": sim.host_empty((nnz + 2,), np.float32),
           "event_cell_offsets": sim.host_empty((w.n_events + 2,), np.int64)}
    out = {"cell_ids": raw["cell_ids"][1:], "cell_e": raw["cell_e"][2:],
           "event_cell_offsets": raw["event_cell_offsets"][1:]}

    def check(label):
        print(f"[host copy] {label}", flush=True)
        assert np.array_equal(out["event_cell_offsets"], ref["ev_cell_off"]), label
        assert np.array_equal(out["cell_ids"], geo["cell_id"][ref["cell_idx"]]), label
        e = out["cell_e"].astype(np.float64)
        assert np.all(np.abs(e - ref["cell_e"]) <= np.maximum(REL * ref["cell_e"], ABS)), label

    def launch(wgs):
        for a in raw.values():
            a.fill(-1)
        sim.simulate_events(dp, doff, w.seed, event_index_base=base, outputs=("compact",),
                            out=out, cell_capacity=nnz, async_launch=True, host_outputs=True,
                            host_copy_workgroups=wgs)

    for wgs in (0, 3, -1):
        launch(wgs)
        r = sim.simulate_events(dp, doff, w.seed, event_index_base=base, outputs=("compact",))
        torch.cuda.synchronize()
        assert r["stats"]["n_cells_nonzero"] == nnz
        sim.synchronize()
        check(f"{wgs} workgroups, then a synchronous call")
        launch(wgs)
        sim.query_sizes(dp, doff, w.seed, event_index_base=base)
        sim.synchronize()
        check(f"{wgs} workgroups, then a query")
        launch(wgs)
        sim.backward(dp, doff, w.seed, torch.zeros(w.n_events, geo["n_cells"], device="cuda"),
                     event_index_base=base)
        sim.synchronize()
        check(f"{wgs} workgroups, then an adjoint call")


def test_staging_set_reused_while_its_copy_runs(sim, torch_cuda, oracle_lib, geom_full, param_full):
    """A call that reuses a device staging set waits for the copy out of it
    only before its own compaction: a pile-up pair of events (4 MB of lists,
    copied by one workgroup) and then two single-particle events, the second
    of which compacts into the pile-up call's set while that copy may still
    run; after the synchronization every call's host lists equal the
    oracle's, twice in a row."""
    torch = torch_cuda
    geo = W.make_geometry()
    ws = [W.subset_events(W.pileup(), 0, 2)] + \
         [W.subset_events(W.single_particle_sweep(), k, 1) for k in (11, 12)]
    calls = []
    for w in ws:
        base = w.notes["event_index_base"]
        dp, doff = _dev(w, torch)
        ref = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                                  event_index_base=base, hit_energy_scale=w.hit_energy_scale)
        nnz = ref["n_cells_nonzero"]
        out = {"cell_ids": sim.host_empty((nnz,), np.int64),
               "cell_e": sim.host_empty((nnz,), np.float32),
               "event_cell_offsets": sim.host_empty((w.n_events + 1,), np.int64)}
        calls.append((w, base, dp, doff, ref, out))
    for rep in range(2):
        for w, base, dp, doff, ref, out in calls:
            for a in out.values():
                a.fill(-1)
            sim.simulate_events(dp, doff, w.seed, event_index_base=base, outputs=("compact",),
                                out=out, cell_capacity=ref["n_cells_nonzero"], async_launch=True,
                                host_outputs=True, host_copy_workgroups=1,
                                hit_energy_scale=w.hit_energy_scale)
        sim.synchronize()
        for w, base, dp, doff, ref, out in calls:
            print(f"[staging reuse] pass {rep}: {w.name}, {ref['n_cells_nonzero']} cells", flush=True)
            assert np.array_equal(out["event_cell_offsets"], ref["ev_cell_off"])
            assert np.array_equal(out["cell_ids"], geo["cell_id"][ref["cell_idx"]])
            e = out["cell_e"].astype(np.float64)
            assert np.all(np.abs(e - ref["cell_e"]) <= np.maximum(REL * ref["cell_e"], ABS))
