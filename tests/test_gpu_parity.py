"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: hit counts, hit positions (bit patterns), hit cells and the set and
order of compacted cells are identical; cell energies (FP32 accumulation)
agree with the FP64 oracle within relative 1e-5 or absolute 1e-3 MeV."""
import os

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
def geo():
    return W.make_geometry()


@pytest.fixture(scope="module")
def par():
    return W.make_param()


@pytest.fixture(scope="module")
def sim(torch_cuda, geo, par):
    from paper_2103_14737_amd.fcs import Simulator
    s = Simulator(0)
    s.load_geometry(geo)
    s.load_parametrization(par)
    yield s
    s.close()


def _np(x):
    return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)


def _dev(w, torch):
    from paper_2103_14737_amd.fcs import particles_to_device
    return particles_to_device(w.particles), torch.from_numpy(w.event_offsets).cuda()


def check_parity(r, ref, geo, hits=True, counts=True, label=""):
    print(f"[parity] {label}: {ref['n_hits_total']} hits, {ref['n_cells_nonzero']} cells",
          flush=True)
    st = r["stats"]
    assert st["n_hits"] == ref["n_hits_total"], label
    assert st["n_hits_out_of_acceptance"] == ref["n_out_of_acc"], label
    if counts:
        assert np.array_equal(_np(r["counts"]), ref["n"]), label
    if hits:
        h = ref["hits"]
        assert np.array_equal(_np(r["hit_cell"]), h["cell"]), label
        assert np.array_equal(_np(r["hit_eta"]).view(np.uint32), h["eta"].view(np.uint32)), label
        assert np.array_equal(_np(r["hit_phi"]).view(np.uint32), h["phi"].view(np.uint32)), label
        assert np.array_equal(_np(r["hit_e"]).view(np.uint32), h["e"].view(np.uint32)), label
        off = _np(r["task_hit_offsets"])
        assert off[0] == 0 and np.array_equal(np.diff(off), ref["n"]), label
    assert np.array_equal(_np(r["event_cell_offsets"]), ref["ev_cell_off"]), label
    assert np.array_equal(_np(r["cell_ids"]), geo["cell_id"][ref["cell_idx"]]), label
    e = _np(r["cell_e"]).astype(np.float64)
    err = np.abs(e - ref["cell_e"])
    tol = np.maximum(REL * np.abs(ref["cell_e"]), ABS)
    bad = err > tol
    assert not bad.any(), (label, int(bad.sum()), float((err / np.maximum(np.abs(ref["cell_e"]), 1e-30)).max()))


def run_both(sim, oracle_lib, geom_o, param_o, geo, w, torch, mode="batched", hits=True,
             device_inputs=True, base=0, **kw):
    outputs = ("compact", "counts", "hits") if hits else ("compact", "counts")
    if device_inputs:
        dp, doff = _dev(w, torch)
        r = sim.simulate_events(dp, doff, w.seed, event_index_base=base, mode=mode,
                                outputs=outputs, hit_energy_scale=w.hit_energy_scale, **kw)
        torch.cuda.synchronize()
    else:
        r = sim.simulate_events(w.particles, w.event_offsets, w.seed, event_index_base=base,
                                mode=mode, outputs=outputs, hit_energy_scale=w.hit_energy_scale,
                                **kw)
    ref = oracle_lib.simulate(geom_o, param_o, w.particles, w.event_offsets, w.seed,
                              event_index_base=base, hit_energy_scale=w.hit_energy_scale,
                              hit_list=hits)
    return r, ref


# ------------------------------------------------------------- workloads ---
@pytest.mark.parametrize("mode", ["batched", "per_event", "per_task"])
@pytest.mark.parametrize("device_inputs", [True, False])
def test_single_electron(sim, oracle_lib, geom_full, param_full, geo, torch_cuda, mode,
                         device_inputs):
    w = W.single_electron()
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, mode=mode,
                      device_inputs=device_inputs)
    check_parity(r, ref, geo, label=f"single electron {mode}")


@pytest.mark.parametrize("mode", ["batched", "per_event", "per_task"])
def test_single_particle_sweep_slice(sim, oracle_lib, geom_full, param_full, geo, torch_cuda,
                                     mode):
    w = W.subset_events(W.single_particle_sweep(), 1000, 300)
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, mode=mode,
                      base=1000)
    check_parity(r, ref, geo, label=f"sweep[1000:1300] {mode}")


@pytest.mark.parametrize("mode", ["batched", "per_event", "per_task"])
def test_hard_scatter_slice(sim, oracle_lib, geom_full, param_full, geo, torch_cuda, mode):
    w = W.subset_events(W.hard_scatter(), 10, 3)
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, mode=mode,
                      base=10)
    check_parity(r, ref, geo, label=f"hard scatter[10:13] {mode}")


def test_pileup_one_event(sim, oracle_lib, geom_full, param_full, geo, torch_cuda):
    w = W.subset_events(W.pileup(), 5, 1)
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, base=5)
    check_parity(r, ref, geo, label="pileup[5]")


def test_single_pion_diff_config(sim, oracle_lib, geom_full, param_full, geo, torch_cuda):
    w = W.single_pion_diff()
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda)
    check_parity(r, ref, geo, label="single pions")


@pytest.mark.parametrize("tuning", [
    dict(chunk_hits=64, big_task_hits=1, tile_hits=64, wg_per_cu=1),
    dict(chunk_hits=8192, big_task_hits=512, tile_hits=512, wg_per_cu=8),
    dict(chunk_hits=1000, big_task_hits=37, tile_hits=192, wg_per_cu=2, use_graph=False),
])
def test_tuning_does_not_change_results(sim, oracle_lib, geom_full, param_full, geo, torch_cuda,
                                        tuning):
    w = W.subset_events(W.hard_scatter(), 0, 2)
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, **tuning)
    check_parity(r, ref, geo, label=f"tuning {tuning}")


def test_dense_output_matches_compact(sim, oracle_lib, geom_full, param_full, geo, torch_cuda):
    w = W.subset_events(W.single_particle_sweep(), 0, 20)
    dp, doff = _dev(w, torch_cuda)
    r = sim.simulate_events(dp, doff, w.seed, outputs=("dense", "compact"))
    ref = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed)
    check_parity(r, ref, geo, hits=False, counts=False, label="dense+compact")
    dense = _np(r["cells"])
    C = geo["n_cells"]
    want = np.zeros((w.n_events, C))
    for e in range(w.n_events):
        s, t = ref["ev_cell_off"][e], ref["ev_cell_off"][e + 1]
        want[e, ref["cell_idx"][s:t]] = ref["cell_e"][s:t]
    assert np.all(np.abs(dense - want) <= np.maximum(REL * np.abs(want), ABS))
    assert np.count_nonzero(dense) == ref["n_cells_nonzero"]


# ------------------------------------------------------------ edge cases ---
def _particles(rows):
    p = np.zeros(len(rows), W.PARTICLE_DTYPE)
    for i, r in enumerate(rows):
        p[i] = r
    return p


def test_edge_cases(sim, oracle_lib, geom_full, param_full, geo, torch_cuda):
    pi_f = np.float32(np.pi)
    rows = [(11, 65000.0, 3.6, 0.0),             # all hits out of acceptance
            (11, 65000.0, 3.2, 1.0),             # acceptance edge
            (22, 50000.0, -3.1999998, -pi_f),    # phi = -pi_f
            (211, 40000.0, 1.4, np.nextafter(pi_f, np.float32(0))),  # region edge, phi ~ pi
            (11, 4.0e6, 0.0, 0.5),               # 4 TeV: hit cap
            (-211, 1000.0, -1.4, 2.0),           # soft pion at a region edge
            (22, 2.0e5, 2.49, -3.0)]
    parts = _particles(rows)
    # events: [0,2), empty, [2,5), [5,7)
    # 20 MeV per expected hit so that the 4 TeV electron reaches the hit cap
    w = W.Workload("edges", 77, parts, np.array([0, 2, 2, 5, 7], np.int64),
                   hit_energy_scale=20.0)
    for mode in ("batched", "per_event", "per_task"):
        r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, mode=mode)
        check_parity(r, ref, geo, label=f"edges {mode}")
        assert ref["n"].max() == 20000
        assert ref["ev_cell_off"][1] == ref["ev_cell_off"][2]


def test_tiny_geometry(torch_cuda, oracle_lib):
    from paper_2103_14737_amd.fcs import Simulator
    g, p = W.make_tiny_geometry(), W.make_param(n_layers=3)
    s = Simulator(0)
    s.load_geometry(g)
    s.load_parametrization(p)
    rng = np.random.default_rng(3)
    n = 200
    parts = _particles([(int(rng.choice([11, 22, 211])), float(np.exp(rng.uniform(8, 13))),
                         float(rng.uniform(-3.4, 3.4)), float(rng.uniform(-np.pi, np.pi)))
                        for _ in range(n)])
    off = np.array([0, 50, 120, 200], np.int64)
    w = W.Workload("tiny", 5, parts, off)
    go, po = oracle_lib.Geometry(g), oracle_lib.Param(p)
    r, ref = run_both(s, oracle_lib, go, po, g, w, torch_cuda)
    check_parity(r, ref, g, label="tiny geometry")
    s.close()


def test_capacity_and_errors(sim, geo, torch_cuda):
    from paper_2103_14737_amd.fcs import FCS_E_CAPACITY, FCS_E_INVALID_ARG, FcsError
    w = W.subset_events(W.single_particle_sweep(), 0, 10)
    dp, doff = _dev(w, torch_cuda)
    with pytest.raises(FcsError) as e:
        sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=5)
    assert e.value.code == FCS_E_CAPACITY and "cell_capacity" in str(e.value)
    with pytest.raises(FcsError) as e:
        sim.simulate_events(dp, doff, w.seed, outputs=("hits",), hit_capacity=10)
    assert e.value.code == FCS_E_CAPACITY
    bad = w.particles.copy()
    bad["pdg"][4] = 2212
    from paper_2103_14737_amd.fcs import particles_to_device
    with pytest.raises(FcsError) as e:
        sim.simulate_events(particles_to_device(bad), doff, w.seed, cell_capacity=10 ** 6)
    assert e.value.code == FCS_E_INVALID_ARG and "pdg" in str(e.value)
    # the context stays usable after errors, and the accumulator stays clean
    r1 = sim.simulate_events(dp, doff, w.seed)
    r2 = sim.simulate_events(dp, doff, w.seed)
    assert np.array_equal(_np(r1["cell_ids"]), _np(r2["cell_ids"]))
    assert np.array_equal(_np(r1["cell_e"]), _np(r2["cell_e"])) or np.allclose(
        _np(r1["cell_e"]), _np(r2["cell_e"]), rtol=REL, atol=ABS)


@pytest.mark.parametrize("mode", ["batched", "per_event", "per_task"])
def test_bad_device_offsets_rejected(sim, geo, torch_cuda, mode):
    """Decreasing event offsets on the device: the call reports
    FCS_E_INVALID_ARG (checked by the setup kernels in batched mode, on the
    host copy in per-event mode) and the context stays clean."""
    from paper_2103_14737_amd.fcs import FCS_E_INVALID_ARG, FcsError
    torch = torch_cuda
    w = W.subset_events(W.hard_scatter(), 0, 3)
    dp, doff = _dev(w, torch)
    off = w.event_offsets.copy()
    off[1], off[2] = off[2], off[1]
    with pytest.raises(FcsError) as e:
        sim.simulate_events(dp, torch.from_numpy(off).cuda(), w.seed, mode=mode, cell_capacity=10 ** 7)
    assert e.value.code == FCS_E_INVALID_ARG and ("offsets" in str(e.value))
    r1 = sim.simulate_events(dp, doff, w.seed)
    r2 = sim.simulate_events(dp, doff, w.seed, mode=mode)
    torch.cuda.synchronize()
    assert np.array_equal(_np(r1["cell_ids"]), _np(r2["cell_ids"]))
    assert np.allclose(_np(r1["cell_e"]), _np(r2["cell_e"]), rtol=REL, atol=ABS)


def test_modes_and_graph_replay_agree(sim, geo, torch_cuda):
    w = W.subset_events(W.hard_scatter(), 20, 4)
    dp, doff = _dev(w, torch_cuda)
    outs = []
    for kw in (dict(mode="batched"), dict(mode="batched"), dict(mode="batched", use_graph=False),
               dict(mode="per_event"), dict(mode="per_task")):
        r = sim.simulate_events(dp, doff, w.seed, event_index_base=20,
                                outputs=("compact", "counts", "hits"), **kw)
        torch_cuda.cuda.synchronize()
        outs.append({k: _np(v) for k, v in r.items() if k != "stats"})
    for o in outs[1:]:
        for k in ("cell_ids", "event_cell_offsets", "counts", "hit_cell", "task_hit_offsets"):
            assert np.array_equal(o[k], outs[0][k]), k
        assert np.allclose(o["cell_e"], outs[0]["cell_e"], rtol=REL, atol=ABS)


# ------------------------------------------- full-size launch configurations ---
def test_full_single_particle_sweep(sim, oracle_lib, geom_full, param_full, geo, torch_cuda):
    w = W.single_particle_sweep()
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, hits=False)
    check_parity(r, ref, geo, hits=False, label="sweep 10k events (full)")


def test_full_sweep_in_the_benchmark_configuration(sim, oracle_lib, geom_full, param_full, geo,
                                                   torch_cuda, tmp_path):
    """The 10,000-event sweep as bench.py times it: autotuned launch, three
    asynchronous calls back to back into the same preallocated device
    buffers, profiled hit kernel; the last call's output against the oracle."""
    torch = torch_cuda
    from paper_2103_14737_amd import autotune
    w = W.single_particle_sweep()
    dp, doff = _dev(w, torch)
    q = sim.query_sizes(dp, doff, w.seed, hit_energy_scale=w.hit_energy_scale)
    cap = q["max_cells"]
    out = {"cell_ids": torch.empty(cap, dtype=torch.int64, device="cuda"),
           "cell_e": torch.empty(cap, dtype=torch.float32, device="cuda"),
           "event_cell_offsets": torch.empty(w.n_events + 1, dtype=torch.int64, device="cuda")}
    tuning = autotune.tune(sim, dp, doff, w.seed, out=out, cell_capacity=cap,
                           hit_energy_scale=w.hit_energy_scale,
                           cache_path=str(tmp_path / "tune.json"))
    print(f"[parity] sweep, tuning {tuning}", flush=True)
    for _ in range(3):
        sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap, out=out,
                            profile=True, hit_energy_scale=w.hit_energy_scale, async_launch=True,
                            **tuning)
    st = sim.synchronize()
    torch.cuda.synchronize()
    ref = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed)
    assert st["n_calls"] == 3 and st["n_hits"] == 3 * ref["n_hits_total"]
    nnz = ref["n_cells_nonzero"]
    assert st["n_cells_nonzero"] == 3 * nnz
    off = _np(out["event_cell_offsets"])
    assert np.array_equal(off, ref["ev_cell_off"])
    assert np.array_equal(_np(out["cell_ids"][:nnz]), geo["cell_id"][ref["cell_idx"]])
    e = _np(out["cell_e"][:nnz]).astype(np.float64)
    assert np.all(np.abs(e - ref["cell_e"]) <= np.maximum(REL * ref["cell_e"], ABS))


def test_full_hard_scatter(sim, oracle_lib, geom_full, param_full, geo, torch_cuda):
    w = W.hard_scatter()
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, hits=False)
    check_parity(r, ref, geo, hits=False, label="hard scatter 100 events (full)")


@pytest.mark.parametrize("n_events", [20, 28])
def test_setup_groupings(sim, oracle_lib, geom_full, param_full, geo, torch_cuda, n_events):
    """Hard-scatter slices whose particle counts give the setup two and three
    scan blocks per workgroup (the full batch gives four, small ones one)."""
    w = W.subset_events(W.hard_scatter(), 0, n_events)
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, hits=False)
    check_parity(r, ref, geo, hits=False, label=f"hard scatter {n_events} events ({len(w.particles)} particles)")


def test_full_pileup_every_event(sim, oracle_lib, geom_full, param_full, geo, torch_cuda):
    """The whole 20-event pile-up batch (214 M hits) in one batched call, as
    the benchmark runs it; every event against the oracle (run per event in
    host threads: events are independent and keyed by their global index)."""
    from concurrent.futures import ThreadPoolExecutor
    full = W.pileup()
    dp, doff = _dev(full, torch_cuda)
    r = sim.simulate_events(dp, doff, full.seed, outputs=("compact", "counts"),
                            hit_energy_scale=full.hit_energy_scale)
    torch_cuda.cuda.synchronize()
    print(f"[parity] pileup full: {r['stats']['n_hits']} hits", flush=True)
    ids, es, off = _np(r["cell_ids"]), _np(r["cell_e"]), _np(r["event_cell_offsets"])
    counts = _np(r["counts"])
    L = 24

    def ref_event(e):
        sub = W.subset_events(full, e, 1)
        return oracle_lib.simulate(geom_full, param_full, sub.particles, sub.event_offsets,
                                   full.seed, event_index_base=e,
                                   hit_energy_scale=full.hit_energy_scale)

    n_thr = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(max_workers=n_thr) as ex:
        refs = list(ex.map(ref_event, range(full.n_events)))
    assert sum(x["n_hits_total"] for x in refs) == r["stats"]["n_hits"]
    assert sum(x["n_out_of_acc"] for x in refs) == r["stats"]["n_hits_out_of_acceptance"]
    nnz = 0
    for e, ref in enumerate(refs):
        a, b = full.event_offsets[e], full.event_offsets[e + 1]
        assert np.array_equal(counts[a * L:b * L], ref["n"]), e
        s, t = off[e], off[e + 1]
        assert s == nnz and t - s == ref["n_cells_nonzero"], e
        nnz = t
        assert np.array_equal(ids[s:t], geo["cell_id"][ref["cell_idx"]]), e
        err = np.abs(es[s:t].astype(np.float64) - ref["cell_e"])
        assert np.all(err <= np.maximum(REL * ref["cell_e"], ABS)), e
    assert off[full.n_events] == nnz == r["stats"]["n_cells_nonzero"]


# --------------------------------------------------------------- adjoint ---
@pytest.mark.parametrize("fluct", [False, True])
def test_backward_matches_oracle_gradient(sim, oracle_lib, geom_full, param_full, geo, torch_cuda,
                                          fluct):
    """fcs_backward against the oracle's FP64 gradient, for the constant hit
    energy and for the per-hit energy fluctuation variant."""
    torch = torch_cuda
    w = W.single_pion_diff()
    C = geo["n_cells"]
    ep = oracle_lib.perturbed_elayer(param_full, w.particles, w.event_offsets, w.seed)
    T = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                            elayer_override=ep, hit_energy_fluct=fluct)
    E = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                            hit_energy_fluct=fluct)

    def dense(res):
        d = np.zeros(w.n_events * C)
        o = res["ev_cell_off"]
        for e in range(w.n_events):
            d[e * C + res["cell_idx"][o[e]:o[e + 1]]] = res["cell_e"][o[e]:o[e + 1]]
        return d

    g = (2.0 * (dense(E) - dense(T))).astype(np.float32)
    dE_ref, dW_ref = oracle_lib.gradient(geom_full, param_full, w.particles, w.event_offsets,
                                         w.seed, g, hit_energy_fluct=fluct)
    dp, doff = _dev(w, torch)
    dE, dW = sim.backward(dp, doff, w.seed, torch.from_numpy(g).cuda(), hit_energy_fluct=fluct)
    torch.cuda.synchronize()
    dE, dW = _np(dE).astype(np.float64), _np(dW).astype(np.float64)
    sE = np.abs(dE_ref).max()
    assert np.all(np.abs(dE - dE_ref) <= 1e-5 * np.abs(dE_ref) + 1e-6 * sE)
    sW = np.abs(dW_ref).max()
    assert np.all(np.abs(dW - dW_ref) <= 1e-5 * np.abs(dW_ref) + 1e-6 * sW)
    assert np.count_nonzero(dW_ref) > 0


def test_autograd_function(sim, oracle_lib, geom_full, param_full, geo, par, torch_cuda):
    """simulate_dense: forward equals the oracle run with the same layer
    energies; backward equals fcs_backward on the incoming gradient."""
    torch = torch_cuda
    from paper_2103_14737_amd.autograd import simulate_dense
    w = W.subset_events(W.single_pion_diff(), 0, 16)
    C = geo["n_cells"]
    base = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed)
    el_ref = base["elayer"].astype(np.float32)
    ref = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                              elayer_override=el_ref)
    ep = oracle_lib.perturbed_elayer(param_full, w.particles, w.event_offsets, w.seed)
    T = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                            elayer_override=ep)
    Td = np.zeros((w.n_events, C))
    for e in range(w.n_events):
        s, t = T["ev_cell_off"][e], T["ev_cell_off"][e + 1]
        Td[e, T["cell_idx"][s:t]] = T["cell_e"][s:t]

    dp, doff = _dev(w, torch)
    el = torch.from_numpy(el_ref).cuda().requires_grad_()
    wt = torch.from_numpy(par["weights"]).cuda().requires_grad_()
    cells = simulate_dense(sim, dp, doff, w.seed, el, wt)
    torch.cuda.synchronize()
    print(f"[parity] autograd forward: {ref['n_hits_total']} hits", flush=True)
    got = _np(cells.detach()).astype(np.float64)
    for e in range(w.n_events):
        s, t = ref["ev_cell_off"][e], ref["ev_cell_off"][e + 1]
        idx = ref["cell_idx"][s:t]
        assert np.count_nonzero(got[e]) == t - s
        err = np.abs(got[e, idx] - ref["cell_e"][s:t])
        assert np.all(err <= np.maximum(REL * np.abs(ref["cell_e"][s:t]), ABS))

    loss = ((cells - torch.from_numpy(Td).float().cuda()) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    g = (2.0 * (cells.detach() - torch.from_numpy(Td).float().cuda())).reshape(-1)
    dE, dW = sim.backward(dp, doff, w.seed, g, elayer_override=el.detach())
    torch.cuda.synchronize()
    for a, b in ((el.grad, dE), (wt.grad, dW)):
        a, b = _np(a).astype(np.float64), _np(b).astype(np.float64)
        assert np.count_nonzero(b) > 0
        # same kernel, same incoming gradient: FP64 atomic order only
        assert np.all(np.abs(a - b) <= 1e-6 * np.abs(b) + 1e-9 * np.abs(b).max())


def test_dense_only_then_compact(sim, oracle_lib, geom_full, param_full, geo, torch_cuda):
    """A dense-only call skips the compaction: its nonzero-cell count still
    matches the oracle, and a compacted call after it starts clean."""
    torch = torch_cuda
    w = W.subset_events(W.single_particle_sweep(), 0, 20)
    dp, doff = _dev(w, torch)
    ref = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed)
    r = sim.simulate_events(dp, doff, w.seed, outputs=("dense",))
    torch.cuda.synchronize()
    assert r["stats"]["n_cells_nonzero"] == ref["n_cells_nonzero"]
    dense = _np(r["cells"])
    assert np.count_nonzero(dense) == ref["n_cells_nonzero"]
    w2 = W.subset_events(W.hard_scatter(), 0, 2)
    r2, ref2 = run_both(sim, oracle_lib, geom_full, param_full, geo, w2, torch)
    check_parity(r2, ref2, geo, label="compact after dense-only")
    r3 = sim.simulate_events(dp, doff, w.seed, outputs=("dense", "compact"))
    check_parity(r3, ref, geo, hits=False, counts=False, label="dense+compact after dense-only")


def test_backward_repeats_and_partial_gradients(sim, geo, torch_cuda):
    """The adjoint's accumulators are cleared by the passes that read them:
    repeated calls, and calls asking for one gradient only, agree."""
    torch = torch_cuda
    w = W.subset_events(W.single_pion_diff(), 0, 8)
    dp, doff = _dev(w, torch)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    g = torch.randn(w.n_events * geo["n_cells"], generator=gen, device="cuda")
    e1, w1 = sim.backward(dp, doff, w.seed, g)
    e2, _ = sim.backward(dp, doff, w.seed, g, need_weights=False)
    _, w3 = sim.backward(dp, doff, w.seed, g, need_elayer=False)
    e4, w4 = sim.backward(dp, doff, w.seed, g)
    torch.cuda.synchronize()
    for a, b in ((e1, e2), (e1, e4), (w1, w3), (w1, w4)):
        a, b = _np(a).astype(np.float64), _np(b).astype(np.float64)
        assert np.count_nonzero(a) > 0
        # FP64 atomic order only
        assert np.all(np.abs(a - b) <= 1e-6 * np.abs(a) + 1e-9 * np.abs(a).max())


def test_backward_reuses_the_forward_queue_only_when_it_matches(sim, geo, torch_cuda):
    """reuse_forward_queue: right after the forward call the adjoint runs on
    its work queue; after another call rebuilt the queue (other inputs), or
    with other options, the flag falls back to a full adjoint.  Every variant
    gives the gradients of the plain call."""
    torch = torch_cuda
    w = W.subset_events(W.single_pion_diff(), 0, 12)
    dp, doff = _dev(w, torch)
    other = W.subset_events(W.single_pion_diff(), 12, 5)
    dpo, doffo = _dev(other, torch)
    el = sim.simulate_events(dp, doff, w.seed, outputs=("elayer",))["elayer"]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    g = torch.randn(w.n_events * geo["n_cells"], generator=gen, device="cuda")
    ref_e, ref_w = sim.backward(dp, doff, w.seed, g, elayer_override=el)

    def fwd():
        sim.simulate_events(dp, doff, w.seed, outputs=("dense",), elayer_override=el)

    variants = []
    fwd()
    variants.append(sim.backward(dp, doff, w.seed, g, elayer_override=el, reuse_forward_queue=True))
    variants.append(sim.backward(dp, doff, w.seed, g, elayer_override=el, reuse_forward_queue=True))
    fwd()
    sim.simulate_events(dpo, doffo, other.seed, outputs=("dense",))
    variants.append(sim.backward(dp, doff, w.seed, g, elayer_override=el, reuse_forward_queue=True))
    fwd()
    variants.append(sim.backward(dp, doff, w.seed, g, elayer_override=el, reuse_forward_queue=True,
                                 hit_energy_scale=150.0))
    fwd()
    variants.append(sim.backward(dp, doff, w.seed, g, elayer_override=el, reuse_forward_queue=True,
                                 async_launch=True))
    sim.synchronize()
    torch.cuda.synchronize()
    a_e, a_w = _np(ref_e).astype(np.float64), _np(ref_w).astype(np.float64)
    assert np.count_nonzero(a_e) > 0 and np.count_nonzero(a_w) > 0
    for i, (e, wg) in enumerate(variants):
        if i == 3:
            # a different hit energy scale: different counts, different gradients
            assert not np.allclose(_np(e), a_e)
            continue
        for a, b in ((a_e, e), (a_w, wg)):
            b = _np(b).astype(np.float64)
            assert np.all(np.abs(a - b) <= 1e-6 * np.abs(a) + 1e-9 * np.abs(a).max()), i


# ------------------------------------------- tables at full-sample volume ---
@pytest.fixture(scope="module")
def fine_tables(oracle_lib):
    par = W.make_param(n_ebins=64, n_etabins=64)
    return par, oracle_lib.Param(par)


def test_fine_binned_tables(torch_cuda, oracle_lib, geom_full, geo, fine_tables):
    """A 64 x 64-bin parametrization (294,912 histograms, the table volume of
    a full physics sample) loaded once and resident: sweep and hard-scatter
    slices against the oracle on the same tables."""
    from paper_2103_14737_amd.fcs import Simulator
    par, par_o = fine_tables
    s = Simulator(0)
    try:
        s.load_geometry(geo)
        s.load_parametrization(par)
        assert s.info()["n_histograms"] == 3 * 64 * 64 * 24
        for w in (W.subset_events(W.single_particle_sweep(), 2000, 60),
                  W.subset_events(W.hard_scatter(), 30, 2)):
            base = w.notes["event_index_base"]
            r, ref = run_both(s, oracle_lib, geom_full, par_o, geo, w, torch_cuda, hits=False,
                              base=base)
            check_parity(r, ref, geo, hits=False, label=f"{w.name}, 64 x 64 tables")
    finally:
        s.close()


def _edge_weights(n_hist, seed=7):
    """Histograms whose cumulative tables sit on the sampler's guide
    thresholds (multiples of 1/1024) or leave runs of guide entries to a
    single bin: equal weights (cum = (b + 1) / 256), one nonzero bin, random
    integer weights summing to 1024 with zero runs, powers of two over 60
    octaves, and a zero first half."""
    rng = np.random.default_rng(seed)
    w = np.zeros((n_hist, 256), np.float32)
    for h in range(n_hist):
        k = h % 5
        if k == 0:
            w[h] = 4.0
        elif k == 1:
            w[h, rng.integers(0, 256)] = 1.0
        elif k == 2:
            live = rng.random(256) < 0.3
            live[rng.integers(0, 256)] = True
            idx = np.flatnonzero(live)
            cuts = np.sort(rng.integers(0, 1025, len(idx) - 1))
            w[h, idx] = np.diff(np.concatenate(([0], cuts, [1024]))).astype(np.float32)
        elif k == 3:
            w[h] = np.exp2((np.arange(256) % 61) - 30.0).astype(np.float32)
        else:
            w[h, 128:] = rng.random(128).astype(np.float32) + 0.5
    return w


def test_edge_histogram_tables(torch_cuda, oracle_lib, geom_full, geo):
    """Sampling tables built on the GPU from histograms with exact guide
    boundaries, empty bins and single-bin mass: every hit's sampled bin, hence
    its position and cell, against the oracle's plain inverse CDF."""
    from paper_2103_14737_amd.fcs import Simulator
    par = W.make_param()
    n_hist = par["weights"].size // 256
    par["weights"] = _edge_weights(n_hist).reshape(-1)
    par_o = oracle_lib.Param(par)
    s = Simulator(0)
    try:
        s.load_geometry(geo)
        s.load_parametrization(par)
        for w in (W.subset_events(W.single_particle_sweep(), 0, 40),
                  W.subset_events(W.hard_scatter(), 0, 1)):
            base = w.notes.get("event_index_base", 0)
            r, ref = run_both(s, oracle_lib, geom_full, par_o, geo, w, torch_cuda, base=base)
            check_parity(r, ref, geo, label=f"{w.name}, edge tables")
    finally:
        s.close()


# --------------------------------------------------- FP64 placement variant ---
@pytest.mark.parametrize("case,mode", [("sweep", "batched"), ("hard_scatter", "batched"),
                                       ("sweep", "per_event"), ("hard_scatter", "per_task")])
def test_fp64_placement(sim, oracle_lib, geom_full, param_full, geo, torch_cuda, case, mode):
    """The FP64 placement variant against the oracle's FP64 placement: hit
    counts, positions and cells bit for bit, energies within tolerance; the
    FP32 call that follows on the same context gives the FP32 results."""
    if case == "sweep":
        w, base = W.subset_events(W.single_particle_sweep(), 3000, 100), 3000
    else:
        w, base = W.subset_events(W.hard_scatter(), 40, 1), 40
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, mode=mode,
                      base=base, placement_fp64=True)
    ref = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                              event_index_base=base, hit_energy_scale=w.hit_energy_scale,
                              hit_list=True, placement_fp64=True)
    check_parity(r, ref, geo, label=f"{case} {mode}, FP64 placement")
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, mode=mode,
                      base=base)
    check_parity(r, ref, geo, label=f"{case} {mode}, FP32 after FP64")


# -------------------------------------------- energy fluctuation variant ---
@pytest.mark.parametrize("case,mode", [("sweep", "batched"), ("hard_scatter", "batched"),
                                       ("sweep", "per_event"), ("hard_scatter", "per_task")])
def test_energy_fluctuation(sim, oracle_lib, geom_full, param_full, geo, torch_cuda, case, mode):
    """The per-hit energy fluctuation variant against the oracle's: hit
    energies bit for bit (same FP64 log series and rounding), cells and
    counts exact, cell energies within tolerance; the constant-energy call
    that follows on the same context gives the usual results."""
    if case == "sweep":
        w, base = W.subset_events(W.single_particle_sweep(), 4000, 100), 4000
    else:
        w, base = W.subset_events(W.hard_scatter(), 50, 1), 50
    r, _ = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, mode=mode,
                    base=base, hit_energy_fluct=True)
    ref = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                              event_index_base=base, hit_energy_scale=w.hit_energy_scale,
                              hit_list=True, hit_energy_fluct=True)
    check_parity(r, ref, geo, label=f"{case} {mode}, energy fluctuation")
    r, ref = run_both(sim, oracle_lib, geom_full, param_full, geo, w, torch_cuda, mode=mode,
                      base=base)
    check_parity(r, ref, geo, label=f"{case} {mode}, constant energy after fluctuation")


def test_dense_output_in_every_launch_form(sim, torch_cuda):
    """Dense cell output (zero fill and count reset instead of compaction)
    in the three launch forms: the same cells, energies within tolerance,
    and the same nonzero-cell statistic."""
    torch = torch_cuda
    w = W.subset_events(W.hard_scatter(), 60, 2)
    dp, doff = _dev(w, torch)
    outs = []
    for mode in ("batched", "per_event", "per_task"):
        r = sim.simulate_events(dp, doff, w.seed, event_index_base=60, mode=mode, outputs=("dense",))
        torch.cuda.synchronize()
        outs.append((_np(r["cells"]), r["stats"]["n_cells_nonzero"]))
        print(f"[parity] dense output, {mode}: {r['stats']['n_cells_nonzero']} cells", flush=True)
    ref, nnz = outs[0]
    assert nnz == np.count_nonzero(ref) > 0
    for d, n in outs[1:]:
        assert n == nnz
        assert np.array_equal(d != 0, ref != 0)
        assert np.allclose(d, ref, rtol=REL, atol=ABS)


@pytest.mark.parametrize("mode", ["batched", "per_event", "per_task"])
def test_profiled_phase_times(sim, torch_cuda, mode):
    """A profiled synchronous call reports its setup, hit-step and compaction
    times; together they fit in the call's device time, and the results equal
    an unprofiled call's."""
    w = W.subset_events(W.hard_scatter(), 3, 2)
    dp, doff = _dev(w, torch_cuda)
    base = w.notes["event_index_base"]
    r = sim.simulate_events(dp, doff, w.seed, event_index_base=base, mode=mode,
                            outputs=("compact",), profile=True)
    torch_cuda.cuda.synchronize()
    st = r["stats"]
    print(f"[phases] {mode}: setup {st['setup_ms']:.3f} hits {st['kernel_ms']:.3f} "
          f"compact {st['compact_ms']:.3f} device {st['device_ms']:.3f} ms", flush=True)
    assert st["setup_ms"] > 0 and st["kernel_ms"] > 0 and st["compact_ms"] > 0
    assert st["setup_ms"] + st["kernel_ms"] + st["compact_ms"] <= st["device_ms"] * 1.05 + 0.05
    r0 = sim.simulate_events(dp, doff, w.seed, event_index_base=base, mode=mode,
                             outputs=("compact",))
    torch_cuda.cuda.synchronize()
    assert r0["stats"]["kernel_ms"] == 0 and r0["stats"]["setup_ms"] == 0
    assert np.array_equal(_np(r["cell_ids"]), _np(r0["cell_ids"]))
    assert np.array_equal(_np(r["event_cell_offsets"]), _np(r0["event_cell_offsets"]))
