"""Seeded random workloads against the oracle on the GPU: event partitions
with empty events, every particle type (both signs), energies below and
above the parametrization's range, eta beyond the acceptance, phi anywhere,
random hit-energy scales, launch forms, tunings and chain variants.  Hit
counts, hit positions, hit energies and cells bit for bit; cell energies
within tolerance."""
import numpy as np
import pytest

from paper_2103_14737_amd import workloads as W

pytestmark = pytest.mark.gpu
REL, ABS = 1e-5, 1e-3
TUNINGS = [dict(), dict(chunk_hits=64, big_task_hits=32, tile_hits=64, wg_per_cu=1),
           dict(chunk_hits=512, big_task_hits=64, tile_hits=256, wg_per_cu=4),
           dict(chunk_hits=8192, big_task_hits=256, tile_hits=512, wg_per_cu=8)]


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


def _workload(rng):
    n_events = int(rng.integers(1, 7))
    counts = rng.integers(0, 41, n_events)
    counts[rng.integers(0, n_events)] = max(1, counts.max())  # at least one particle
    n = int(counts.sum())
    pdg = rng.choice(np.array([11, -11, 22, 211, -211], np.int32), n)
    e = np.exp(rng.uniform(np.log(300.0), np.log(4.5e6), n))
    eta = rng.uniform(-3.5, 3.5, n)
    phi = rng.uniform(-np.pi, np.pi, n)
    parts = np.zeros(n, W.PARTICLE_DTYPE)
    parts["pdg"], parts["e"], parts["eta"], parts["phi"] = pdg, e, eta, phi
    off = np.zeros(n_events + 1, np.int64)
    off[1:] = np.cumsum(counts)
    scale = float(rng.choice([20.0, 100.0, 300.0]))
    return W.Workload("random", int(rng.integers(1, 2 ** 40)), parts, off, hit_energy_scale=scale)


@pytest.mark.parametrize("case", range(12))
def test_random_workload(sim, oracle_lib, geom_full, param_full, torch_cuda, case):
    torch = torch_cuda
    from paper_2103_14737_amd.fcs import particles_to_device
    rng = np.random.default_rng(1000 + case)
    w = _workload(rng)
    base = int(rng.integers(0, 10 ** 6))
    mode = ["batched", "per_event", "per_task"][case % 3]
    tuning = TUNINGS[int(rng.integers(0, len(TUNINGS)))]
    variant = [dict(), dict(), dict(placement_fp64=True), dict(hit_energy_fluct=True)][case % 4]
    print(f"[random] case {case}: {w.n_events} events, {len(w.particles)} particles, {mode}, "
          f"{tuning}, {variant}, scale {w.hit_energy_scale}", flush=True)
    dp = particles_to_device(w.particles)
    doff = torch.from_numpy(w.event_offsets).cuda()
    r = sim.simulate_events(dp, doff, w.seed, event_index_base=base, mode=mode,
                            outputs=("compact", "counts", "hits"),
                            hit_energy_scale=w.hit_energy_scale, **tuning, **variant)
    torch.cuda.synchronize()
    ref = oracle_lib.simulate(geom_full, param_full, w.particles, w.event_offsets, w.seed,
                              event_index_base=base, hit_energy_scale=w.hit_energy_scale,
                              hit_list=True, **variant)
    st = r["stats"]
    assert st["n_hits"] == ref["n_hits_total"]
    assert st["n_hits_out_of_acceptance"] == ref["n_out_of_acc"]
    assert np.array_equal(r["counts"].cpu().numpy(), ref["n"])
    h = ref["hits"]
    assert np.array_equal(r["hit_cell"].cpu().numpy(), h["cell"])
    for k in ("eta", "phi", "e"):
        assert np.array_equal(r[f"hit_{k}"].cpu().numpy().view(np.uint32), h[k].view(np.uint32)), k
    geo_ids = W.make_geometry()["cell_id"]
    assert np.array_equal(r["event_cell_offsets"].cpu().numpy(), ref["ev_cell_off"])
    assert np.array_equal(r["cell_ids"].cpu().numpy(), geo_ids[ref["cell_idx"]])
    e = r["cell_e"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(e - ref["cell_e"]) <= np.maximum(REL * np.abs(ref["cell_e"]), ABS))
