"""Reloading the geometry or the tables between calls, and overrides that
would give subnormal hit energies (through the C ABI, against the oracle)."""
import math

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


def _np(x):
    return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)


def _dev(w, torch):
    from paper_2103_14737_amd.fcs import particles_to_device
    return particles_to_device(w.particles), torch.from_numpy(w.event_offsets).cuda()


def _two_layouts():
    """Two geometries of 1,024 cells each: one layer of two eta regions, and
    two layers of one region."""
    a = W._build_geometry([500.0], [(0.1, 2 * math.pi / 16)], [(0.1, 2 * math.pi / 16)],
                          bounds=(-3.2, 0.0, 3.2))
    b = W._build_geometry([500.0, 700.0], [(0.2, 2 * math.pi / 16)] * 2,
                          [(0.2, 2 * math.pi / 16)] * 2, bounds=(-3.2, 3.2))
    assert a["n_cells"] == b["n_cells"] == 1024
    assert (a["n_layers"], a["n_regions"]) != (b["n_layers"], b["n_regions"])
    return a, b


def test_geometry_reload_with_the_same_cell_count(torch_cuda, oracle_lib):
    """Captured launch sequences are keyed by batch shape; a geometry with the
    same cell count but other layer and region counts must not replay the
    previous geometry's grids and LDS sizes."""
    from paper_2103_14737_amd.fcs import Simulator
    torch = torch_cuda
    ga, gb = _two_layouts()
    w = W.subset_events(W.single_particle_sweep(), 0, 40)
    dp, doff = _dev(w, torch)
    s = Simulator(0)
    try:
        for g in (ga, gb, ga):
            p = W.make_param(n_layers=g["n_layers"])
            s.load_geometry(g)
            s.load_parametrization(p)
            r = s.simulate_events(dp, doff, w.seed, outputs=("compact", "counts"))
            torch.cuda.synchronize()
            ref = oracle_lib.simulate(oracle_lib.Geometry(g), oracle_lib.Param(p), w.particles,
                                      w.event_offsets, w.seed)
            print(f"[reload] {g['n_layers']} layers x {g['n_regions']} regions: "
                  f"{ref['n_hits_total']} hits", flush=True)
            assert r["stats"]["n_hits"] == ref["n_hits_total"]
            assert np.array_equal(_np(r["counts"]), ref["n"])
            assert np.array_equal(_np(r["event_cell_offsets"]), ref["ev_cell_off"])
            assert np.array_equal(_np(r["cell_ids"]), g["cell_id"][ref["cell_idx"]])
            e = _np(r["cell_e"]).astype(np.float64)
            assert np.all(np.abs(e - ref["cell_e"]) <= np.maximum(REL * ref["cell_e"], ABS))
    finally:
        s.close()


def test_backward_after_a_table_reload_recomputes_the_queue(torch_cuda):
    """A forward call leaves a work queue an adjoint may reuse; reloading the
    tables in between (same sizes, other weights) must make the adjoint
    rebuild it: reuse_forward_queue then gives the gradients of a plain
    call on the new tables."""
    from paper_2103_14737_amd.fcs import Simulator
    torch = torch_cuda
    geo = W.make_geometry()
    par = W.make_param()
    par2 = dict(par)
    rng = np.random.default_rng(5)
    par2["weights"] = (par["weights"] * rng.uniform(0.2, 5.0, par["weights"].shape)).astype(np.float32)
    w = W.subset_events(W.single_pion_diff(), 0, 10)
    dp, doff = _dev(w, torch)
    s = Simulator(0)
    try:
        s.load_geometry(geo)
        s.load_parametrization(par)
        el = s.simulate_events(dp, doff, w.seed, outputs=("elayer",))["elayer"]
        gen = torch.Generator(device="cuda")
        gen.manual_seed(3)
        g = torch.randn(w.n_events * geo["n_cells"], generator=gen, device="cuda")
        s.simulate_events(dp, doff, w.seed, outputs=("dense",), elayer_override=el)
        s.load_parametrization(par2)
        re_e, re_w = s.backward(dp, doff, w.seed, g, elayer_override=el, reuse_forward_queue=True)
        ref_e, ref_w = s.backward(dp, doff, w.seed, g, elayer_override=el)
        torch.cuda.synchronize()
        for a, b in ((ref_e, re_e), (ref_w, re_w)):
            a, b = _np(a).astype(np.float64), _np(b).astype(np.float64)
            assert np.count_nonzero(a) > 0
            assert np.all(np.abs(a - b) <= 1e-6 * np.abs(a) + 1e-9 * np.abs(a).max())
    finally:
        s.close()


@pytest.mark.parametrize("device_inputs", [False, True])
def test_override_giving_subnormal_hit_energies_is_rejected(torch_cuda, device_inputs):
    """An override below FLT_MIN x n for a (particle, layer) with n hits
    would deposit subnormal energies; the call fails with FCS_E_INVALID_ARG
    (host and device inputs), while the same tiny value on a layer without
    hits, or zero, is accepted."""
    from paper_2103_14737_amd.fcs import FCS_E_INVALID_ARG, FcsError, Simulator
    torch = torch_cuda
    s = Simulator(0)
    try:
        s.load_geometry(W.make_geometry())
        s.load_parametrization(W.make_param())
        w = W.single_electron()
        r = s.simulate_events(w.particles, w.event_offsets, w.seed, outputs=("counts", "elayer"))
        n, el = r["counts"], r["elayer"]
        with_hits = int(np.argmax(n > 0))
        ov = el.copy()
        ov[n == 0] = 1e-40          # ignored: no hits there
        if (n == 0).any():
            ov[int(np.argmax(n == 0))] = 0.0

        def run(v):
            if device_inputs:
                dp, doff = _dev(w, torch)
                res = s.simulate_events(dp, doff, w.seed, outputs=("compact",),
                                        elayer_override=torch.from_numpy(v).cuda())
                torch.cuda.synchronize()
                return res
            return s.simulate_events(w.particles, w.event_offsets, w.seed, outputs=("compact",),
                                     elayer_override=v)

        assert run(ov)["stats"]["n_hits"] == int(n.sum())
        bad = ov.copy()
        bad[with_hits] = np.float32(1e-39) * np.float32(n[with_hits])  # E/n = 1e-39, subnormal
        with pytest.raises(FcsError) as e:
            run(bad)
        assert e.value.code == FCS_E_INVALID_ARG and "FLT_MIN" in str(e.value)
        bad[with_hits] = np.float32(np.finfo(np.float32).tiny) * np.float32(n[with_hits]) * 2
        assert run(bad)["stats"]["n_hits"] == int(n.sum())   # normal again: accepted
    finally:
        s.close()


def test_tables_loaded_while_batches_run(torch_cuda, oracle_lib):
    """fcs_load_parametrization_async between asynchronous batches: the
    batches enqueued before it use the old tables, the ones after it the new
    ones (other weights of the same shape, then the 64 x 64-bin family),
    each equal to the oracle on its own tables; a synchronous call after a
    second asynchronous load takes it into use as well."""
    from paper_2103_14737_amd.fcs import Simulator, particles_to_device
    torch = torch_cuda
    geo = W.make_geometry()
    par1 = W.make_param()
    par2 = dict(par1)
    rng = np.random.default_rng(8)
    par2["weights"] = (par1["weights"] * rng.uniform(0.1, 3.0, par1["weights"].shape)).astype(np.float32)
    par3 = W.make_param(n_ebins=64, n_etabins=64)
    w = W.subset_events(W.single_particle_sweep(), 4000, 300)
    base = w.notes["event_index_base"]
    dp = particles_to_device(w.particles)
    doff = torch.from_numpy(w.event_offsets).cuda()
    go = oracle_lib.Geometry(geo)
    s = Simulator(0)
    try:
        s.load_geometry(geo)
        s.load_parametrization(par1)
        q = s.query_sizes(dp, doff, w.seed, event_index_base=base)
        cap = q["max_cells"] * 2

        def buffers():
            return {"cell_ids": torch.empty(cap, dtype=torch.int64, device="cuda"),
                    "cell_e": torch.empty(cap, dtype=torch.float32, device="cuda"),
                    "event_cell_offsets": torch.empty(w.n_events + 1, dtype=torch.int64,
                                                      device="cuda")}

        outs = [buffers() for _ in range(5)]

        def call(i):
            s.simulate_events(dp, doff, w.seed, event_index_base=base, outputs=("compact",),
                              out=outs[i], cell_capacity=cap, async_launch=True)

        call(0)
        call(1)
        s.load_parametrization(par2, async_load=True)   # while 0 and 1 run
        call(2)
        s.load_parametrization(par3, async_load=True)
        call(3)
        s.load_parametrization(par1, async_load=True)
        r4 = s.simulate_events(dp, doff, w.seed, event_index_base=base, outputs=("compact",),
                               cell_capacity=cap)        # synchronous: takes par1 in again
        s.synchronize()
        torch.cuda.synchronize()
        assert s.info()["n_histograms"] == 11520
        for i, par in ((0, par1), (1, par1), (2, par2), (3, par3), (4, par1)):
            ref = oracle_lib.simulate(go, oracle_lib.Param(par), w.particles, w.event_offsets,
                                      w.seed, event_index_base=base)
            o = r4 if i == 4 else outs[i]
            nnz = ref["n_cells_nonzero"]
            print(f"[async tables] call {i}: {ref['n_hits_total']} hits, {nnz} cells", flush=True)
            off = _np(o["event_cell_offsets"])
            assert np.array_equal(off, ref["ev_cell_off"]), i
            assert np.array_equal(_np(o["cell_ids"][:nnz]), geo["cell_id"][ref["cell_idx"]]), i
            e = _np(o["cell_e"][:nnz]).astype(np.float64)
            assert np.all(np.abs(e - ref["cell_e"]) <= np.maximum(REL * ref["cell_e"], ABS)), i
    finally:
        s.close()
