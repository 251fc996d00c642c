"""Benchmark of the batched hit simulation on one MI355X.

One step = one fcs_simulate_events call over the whole batch in batched mode
(per-(particle, layer) setup, work-queue build, the hit step -- window pass
for the small tasks and the persistent hit kernel for the large ones --,
ordered compaction and accumulator reset) plus the copy of its compacted
{cell_id, E} lists to pinned host buffers (as the paper's event loop copies
each call's results back), inputs resident in device memory.  Steps are
enqueued back to back as asynchronous calls: the copy of one batch runs on
a second stream beside the next batch.  The headline workload is the
pile-up batch: 20 events of 1,500 hard-scatter particles plus 200 x 60
soft ones, 214 M hits per step.

Also reported on the same JSON line: the same batch with the lists left in
device memory, as synchronous calls, and in the per-event launch form; the
hard-scatter batch (100 events of 500-2000 particles) and the
single-particle sweep (10,000 events) in the batched, per-event and
per-(particle, layer) forms; a roofline object for each of the three, on
the hit step's HIP-event time in the timed steps; forward+backward of the
differentiable workload (64 single pions); jobs sharing the GPU; the sweep
on 64 x 64-bin tables, with the FP64 placement and with the per-hit energy
fluctuation; an asynchronous table load beside a running batch; the
measured ceilings of the chip (atomics, HBM copy, VALU clock, launches);
and the CPU oracle timed on the host on a bounded sample of the headline
workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "hits/s & events/s, batched vs per-event launch; fwd+bwd hits/s (1 GPU)"

# peak figures of the chip (MI355X): 256 CUs, 4 SIMD x 16 lanes per CU, 2.4 GHz
N_CU, CLOCK_HZ = 256, 2.4e9
VALU_SLOT_PEAK = N_CU * 64 * CLOCK_HZ   # VALU lane-instruction slots per second
HBM_PEAK = 8.0e12

# Algorithmic work per hit in gfx950 VALU instruction slots (the fewest
# instructions that compute a hit's arithmetic): Philox4x32-10 = 10 rounds x
# (2 v_mad_u64_u32 32x32->64 products + 2 three-input xor v_bitop3) = 40;
# three 24-bit uniforms (shift, convert, scale) = 9; bin choice from the
# guide table (index + ~2 compares) = 3; radial / angular bin split = 2;
# radius = 4; octant sine and cosine (offset, square, 4 + 5 multiply-add
# steps, final multiply, quadrant select) = 24; deta / dphi = 4; eta / phi =
# 2; phi wrap = 3; region-grid lookup (acceptance, region, two
# floor-and-clamp indices, linear index) = 22; deposit = 1.  A Philox draw
# measured alone issues at 40 slots (run_ceilings), so its 80 32-bit
# operations (each product and each three-input xor counting twice) are
# counted as the 40 slots they take.
PHILOX_SLOTS = 40
SLOTS_PER_HIT = PHILOX_SLOTS + 9 + 3 + 2 + 4 + 24 + 4 + 2 + 3 + 22 + 1
OPS_PER_HIT = SLOTS_PER_HIT + PHILOX_SLOTS  # the same work in 32-bit operations
KERNEL_SOURCES = ("paper_2103_14737_amd/csrc/fcs_math.hpp",
                  "paper_2103_14737_amd/csrc/fcs_kernels.hpp",
                  "paper_2103_14737_amd/csrc/fcs_runtime.hip",
                  "paper_2103_14737_amd/build.py")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hit_step_traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, tuning):
    """HBM bytes per launch of the hit step (window pass + hit kernel) from
    the committed counter summaries: the entry taken on the current kernel
    sources, this workload and this tuning, if there is one; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            entries = json.load(f).get("entries", [])
    except (OSError, ValueError, AttributeError):
        return None
    h = kernel_source_hash()
    for t in entries:
        if t.get("source_hash") == h and t.get("workload") == workload and t.get("tuning") == tuning:
            return t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
    return None


TUNING_KEYS = ("chunk_hits", "big_task_hits", "tile_hits", "wg_per_cu", "window_particles")


def parse_tuning(text):
    """'chunk,big,tile,wg[,window_particles]' -> tuning dict"""
    vals = [int(x) for x in text.split(",")]
    return dict(zip(TUNING_KEYS, vals))


def _sync(torch):
    torch.cuda.synchronize()


def _time_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    _sync(torch)
    t0 = time.perf_counter()
    res = [fn() for _ in range(steps)]
    _sync(torch)
    return (time.perf_counter() - t0) / steps, res


def run_fwd_bwd(torch, sim, geo, par, dev, steps, warmup, tuning=None):
    """Forward (dense cells through the autograd binding) + loss + backward
    (the adjoint) on the 64-pion workload; hits of one forward per second.
    Training steps are enqueued back to back (asynchronous library calls, no
    host round trip inside a step) between two device synchronizations; the
    forward and backward times of a synchronized step are reported beside."""
    from paper_2103_14737_amd import workloads as W
    from paper_2103_14737_amd.fcs import particles_to_device
    wd = W.single_pion_diff()
    dpd = particles_to_device(wd.particles, dev)
    doffd = torch.from_numpy(wd.event_offsets).to(dev)
    base = sim.simulate_events(dpd, doffd, wd.seed, outputs=("dense", "elayer"))
    el = base["elayer"]
    # targets: the same particles with perturbed, renormalized layer fractions
    gen = torch.Generator(device=dev)
    gen.manual_seed(wd.seed)
    e2 = el.reshape(-1, sim.n_layers).double()
    pert = (e2 * (1 + 0.2 * torch.randn(e2.shape, generator=gen, device=dev,
                                        dtype=torch.float64))).clamp_min(0)
    pert = (pert * (e2.sum(1, keepdim=True) / pert.sum(1, keepdim=True))).float().reshape(-1)
    target = sim.simulate_events(dpd, doffd, wd.seed, outputs=("dense",),
                                 elayer_override=pert)["cells"]
    from paper_2103_14737_amd.autograd import simulate_dense
    # The library's default tuning: the step is bound by its launches and by
    # the loss's passes over the dense cells (measured the same, within
    # noise, for chunks of 64 to 2048 hits, tiles of 256 or 512 and 4 or 8
    # workgroups per CU).
    tuning = tuning or {}
    el_leaf = el.detach().clone().requires_grad_()
    wt_leaf = torch.from_numpy(par["weights"]).to(dev).requires_grad_()
    nh = int(base["stats"]["n_hits"])
    F = torch.nn.functional

    def step_fb(async_launch):
        # L = sum over cells of (E - T)^2, then dL/d(layer energies, weights)
        el_leaf.grad = None
        wt_leaf.grad = None
        cells = simulate_dense(sim, dpd, doffd, wd.seed, el_leaf, wt_leaf,
                               async_launch=async_launch, **tuning)
        loss = F.mse_loss(cells, target, reduction="sum")
        loss.backward()
        return nh

    for _ in range(warmup):
        step_fb(True)
    sim.synchronize()
    t_fb, _ = _time_steps(torch, lambda: step_fb(True), steps, 0)
    sim.synchronize()  # raises the first error of the asynchronous calls
    # one synchronized step at a time: forward (with the loss) and backward
    times = {"fwd": 0.0, "bwd": 0.0}
    for _ in range(steps):
        el_leaf.grad = None
        wt_leaf.grad = None
        torch.cuda.synchronize()
        a = time.perf_counter()
        cells = simulate_dense(sim, dpd, doffd, wd.seed, el_leaf, wt_leaf, **tuning)
        loss = F.mse_loss(cells, target, reduction="sum")
        torch.cuda.synchronize()
        b = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        times["fwd"] += b - a
        times["bwd"] += time.perf_counter() - b
    res = {"workload": "single_pion_diff", "n_events": wd.n_events,
           "hits_per_step": nh, "hits_per_s": nh / t_fb, "ms_per_step": t_fb * 1e3,
           "synchronized_step": {"t_fwd_ms": times["fwd"] / steps * 1e3,
                                 "t_bwd_ms": times["bwd"] / steps * 1e3},
           "tuning": tuning or "library defaults"}
    print(f"bench: fwd+bwd {nh / t_fb:.4g} hits/s ({t_fb * 1e3:.3f} ms/step), tuning {tuning}",
          flush=True)
    return res


def oracle_baseline(w, geo, par, max_threads=16, one_core_events=2, budget_one=10.0,
                    budget_all=10.0):
    """The oracle timed on the host on a bounded sample of the workload: one
    thread over its first `one_core_events` events (passes until about
    `budget_one` s, at most 5), then the whole workload split into event
    ranges run by independent threads at once (the oracle is re-entrant and
    its C code runs outside the interpreter lock; at most `max_threads`, the
    host share of one GPU, whatever nproc reports) until about `budget_all`
    s, at most 5 passes.  Median passes; returns the cpu_baseline record in
    hits/s, with the host's nproc."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_2103_14737_amd import workloads as W
    oracle.build(force=False)
    go, po = oracle.Geometry(geo), oracle.Param(par)

    def run(sw):
        return oracle.simulate(go, po, sw.particles, sw.event_offsets, sw.seed,
                               event_index_base=sw.notes.get("event_index_base", 0),
                               hit_energy_scale=sw.hit_energy_scale)["n_hits_total"]

    sample = W.subset_events(w, 0, min(one_core_events, w.n_events))
    runs = []
    while not runs or (len(runs) < 5 and sum(runs) < budget_one):
        t0 = time.perf_counter()
        n1 = run(sample)
        runs.append(time.perf_counter() - t0)
    dt = sorted(runs)[len(runs) // 2]
    one = {"value": n1 / dt, "cores": 1,
           "sample": f"events 0-{sample.n_events - 1} of {w.name} ({n1} hits), one thread, "
                     f"median of {len(runs)} passes ({sum(runs):.1f} s in all)"}
    print(f"bench: oracle {one['value']:.4g} hits/s on 1 core", flush=True)
    nproc = len(os.sched_getaffinity(0))
    n_thr = max(1, min(max_threads, nproc, w.n_events))
    bounds = np.linspace(0, w.n_events, n_thr + 1).astype(int)
    parts = [W.subset_events(w, int(a), int(b - a)) for a, b in zip(bounds[:-1], bounds[1:])
             if b > a]
    runs_n = []
    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        while not runs_n or (len(runs_n) < 5 and sum(runs_n) < budget_all):
            t0 = time.perf_counter()
            total = sum(ex.map(run, parts))
            runs_n.append(time.perf_counter() - t0)
    dt_n = sorted(runs_n)[len(runs_n) // 2]
    print(f"bench: oracle {total / dt_n:.4g} hits/s on {len(parts)} threads (nproc {nproc})",
          flush=True)
    return {"value": total / dt_n, "unit": "hits/s", "cores": len(parts), "kind": "oracle",
            "nproc": nproc, "hits_per_pass": total,
            "sample": f"the whole {w.name} workload ({w.n_events} events, {total} hits) split "
                      f"into {len(parts)} event ranges run by {len(parts)} threads at once "
                      f"(capped at {max_threads}, the host share of one GPU; nproc {nproc}), "
                      f"median of {len(runs_n)} passes ({sum(runs_n):.1f} s in all)",
            "one_core": one}


def run_sharing(torch, geo, par, dev, jobs=(1, 2, 4, 8, 16), events_per_call=100, seconds=1.0):
    """Several jobs on one GPU at once, as in the paper's study of concurrent
    processes sharing a GPU: each job is a host thread with its own library
    context (its own stream, workspace and tables) and its own torch stream,
    simulating its own slice of `events_per_call` single-particle events call
    after call and waiting for each call's results.  Per-event and batched
    forms; every job makes the same number of calls (sized so that one job
    alone runs about `seconds`).  Returns, per form, the hits per second of
    all jobs together for each job count."""
    import threading

    from paper_2103_14737_amd import workloads as W
    from paper_2103_14737_amd.fcs import Simulator, particles_to_device
    sweep = W.single_particle_sweep()
    ctx = []
    for j in range(max(jobs)):
        sim = Simulator(0)
        sim.load_geometry(geo)
        sim.load_parametrization(par)
        w = W.subset_events(sweep, j * events_per_call, events_per_call)
        base = w.notes["event_index_base"]
        dp = particles_to_device(w.particles, dev)
        doff = torch.from_numpy(w.event_offsets).to(dev)
        q = sim.query_sizes(dp, doff, w.seed, event_index_base=base)
        cap = q["max_cells"]
        out = {"cell_ids": torch.empty(cap, dtype=torch.int64, device=dev),
               "cell_e": torch.empty(cap, dtype=torch.float32, device=dev),
               "event_cell_offsets": torch.empty(w.n_events + 1, dtype=torch.int64, device=dev)}
        ctx.append({"sim": sim, "w": w, "base": base, "dp": dp, "doff": doff, "cap": cap,
                    "out": out, "hits": q["n_hits"], "stream": torch.cuda.Stream(device=dev)})
    torch.cuda.synchronize()

    def call(c, mode):
        r = c["sim"].simulate_events(c["dp"], c["doff"], c["w"].seed, event_index_base=c["base"],
                                     mode=mode, outputs=("compact",), cell_capacity=c["cap"],
                                     out=c["out"])
        assert r["stats"]["n_hits"] == c["hits"]

    res = {}
    for mode in ("per_event", "batched"):
        for c in ctx:  # warm-up: workspaces and graphs of every context
            with torch.cuda.stream(c["stream"]):
                call(c, mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        call(ctx[0], mode)
        n_calls = max(3, int(math.ceil(seconds / (time.perf_counter() - t0))))
        by_n = {}
        for n in jobs:
            start = threading.Barrier(n + 1)
            errors = []

            def job(k):
                c = ctx[k]
                try:
                    with torch.cuda.stream(c["stream"]):
                        start.wait()
                        for _ in range(n_calls):
                            call(c, mode)
                except BaseException as e:  # re-raised below
                    errors.append(e)

            threads = [threading.Thread(target=job, args=(k,)) for k in range(n)]
            for t in threads:
                t.start()
            start.wait()
            t0 = time.perf_counter()
            for t in threads:
                t.join()
            dt = time.perf_counter() - t0
            if errors:
                raise errors[0]
            hits = n_calls * sum(ctx[k]["hits"] for k in range(n))
            by_n[str(n)] = {"hits_per_s": hits / dt, "calls_per_job": n_calls, "s": dt}
            print(f"bench: sharing {mode} {n} jobs: {hits / dt:.4g} hits/s", flush=True)
        res[mode] = by_n
    for c in ctx:
        c["sim"].close()
    return {"events_per_call": events_per_call, "forms": res}


def run_fine_tables(torch, geo, dev, w, tuning, steps, warmup, n_bins=64):
    """The parametrization at the table volume of a full physics sample:
    n_bins x n_bins (E, |eta|) sets, about 0.3 M histograms, generated on the
    host, then loaded into a fresh context (timed: upload, cumulative and
    guide tables built on the device) and kept resident; the headline batch
    is timed on it as on the default tables.  Returns the record."""
    from paper_2103_14737_amd import workloads as W
    from paper_2103_14737_amd.fcs import Simulator, particles_to_device
    par = W.make_param(n_ebins=n_bins, n_etabins=n_bins)
    sim = Simulator(0)
    try:
        sim.load_geometry(geo)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.load_parametrization(par)
        torch.cuda.synchronize()
        load_ms = (time.perf_counter() - t0) * 1e3
        dp = particles_to_device(w.particles, dev)
        doff = torch.from_numpy(w.event_offsets).to(dev)
        q = sim.query_sizes(dp, doff, w.seed, hit_energy_scale=w.hit_energy_scale)
        cap = q["max_cells"]
        out = {"cell_ids": torch.empty(cap, dtype=torch.int64, device=dev),
               "cell_e": torch.empty(cap, dtype=torch.float32, device=dev),
               "event_cell_offsets": torch.empty(w.n_events + 1, dtype=torch.int64, device=dev)}

        def step():
            sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap,
                                out=out, hit_energy_scale=w.hit_energy_scale, async_launch=True,
                                **tuning)

        for _ in range(warmup):
            step()
        sim.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        st = sim.synchronize()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        assert st["n_hits"] == steps * q["n_hits"], st
        n_hist = sim.info()["n_histograms"]
    finally:
        sim.close()
    rec = {"n_ebins": n_bins, "n_etabins": n_bins, "n_histograms": n_hist,
           "weights_mb": par["weights"].nbytes / 1e6, "load_ms": load_ms,
           "hits_per_step": q["n_hits"], "ms_per_step": dt * 1e3,
           "hits_per_s": q["n_hits"] / dt}
    print(f"bench: {n_bins}x{n_bins} tables ({n_hist} histograms) loaded in {load_ms:.0f} ms; "
          f"{w.name} {q['n_hits'] / dt:.4g} hits/s on them", flush=True)
    rec["async_load"] = run_async_tables(torch, geo, dev, w, tuning, par)
    return rec


def run_async_tables(torch, geo, dev, w, tuning, par_new, n_before=200, n_after=20):
    """A table change overlapped with running batches: n_before batches on
    the default tables are enqueued, then fcs_load_parametrization_async of
    `par_new` (its host-side checks and staging timed), then n_after batches
    (which use the new tables); the whole sequence is timed against the same
    batches with no load in between.  The difference is what the load cost
    the batches' timeline."""
    from paper_2103_14737_amd import workloads as W
    from paper_2103_14737_amd.fcs import Simulator, particles_to_device
    par = W.make_param()
    sim = Simulator(0)
    try:
        sim.load_geometry(geo)
        sim.load_parametrization(par)
        dp = particles_to_device(w.particles, dev)
        doff = torch.from_numpy(w.event_offsets).to(dev)
        q = sim.query_sizes(dp, doff, w.seed, hit_energy_scale=w.hit_energy_scale)
        cap = q["max_cells"]
        out = {"cell_ids": torch.empty(cap, dtype=torch.int64, device=dev),
               "cell_e": torch.empty(cap, dtype=torch.float32, device=dev),
               "event_cell_offsets": torch.empty(w.n_events + 1, dtype=torch.int64, device=dev)}

        def batches(n):
            for _ in range(n):
                sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap,
                                    out=out, hit_energy_scale=w.hit_energy_scale,
                                    async_launch=True, **tuning)

        # both table sets at the new tables' size, as in a loop that keeps
        # switching tables of one family (the first growth waits for the
        # batches that may read the set it frees)
        for pp in (par_new, par_new, par):
            sim.load_parametrization(pp, async_load=True)
            batches(1)

        def timed(load):
            sim.load_parametrization(par, async_load=True)
            batches(3)
            sim.synchronize()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            batches(n_before)
            a = time.perf_counter()
            if load:
                sim.load_parametrization(par_new, async_load=True)
            host = time.perf_counter() - a
            batches(n_after)
            sim.synchronize()
            torch.cuda.synchronize()
            return time.perf_counter() - t0, host

        t0, _ = timed(False)
        t1, host = timed(True)
        t2, _ = timed(False)
    finally:
        sim.close()
    base = min(t0, t2)
    rec = {"batches_before": n_before, "batches_after": n_after,
           "ms_without_load": base * 1e3, "ms_with_async_load": t1 * 1e3,
           "load_cost_on_timeline_ms": (t1 - base) * 1e3, "host_call_ms": host * 1e3}
    print(f"bench: asynchronous table load between batches: {n_before}+{n_after} batches "
          f"{t1 * 1e3:.1f} ms with the load, {base * 1e3:.1f} ms without; host call "
          f"{host * 1e3:.1f} ms", flush=True)
    return rec


def run_per_task(torch, sim, prepare, w, n_events, batched_hits_per_s):
    """The per-(particle, layer) launch form on the first `n_events` events of
    a workload (one launch per task with hits, as the paper's first port);
    its hits/s beside the batched form's on the whole workload."""
    from paper_2103_14737_amd import workloads as W
    ws = W.subset_events(w, 0, n_events)
    dp, doff, out, cap, q = prepare(ws)

    def step():
        r = sim.simulate_events(dp, doff, ws.seed, mode="per_task", outputs=("compact",),
                                cell_capacity=cap, out=out, hit_energy_scale=ws.hit_energy_scale)
        return r["stats"]["n_hits"]

    t, res = _time_steps(torch, step, 2, 1)
    assert all(h == q["n_hits"] for h in res)
    rate = q["n_hits"] / t
    print(f"bench: per-task {ws.name}: {t * 1e3:.1f} ms per call, {rate:.4g} hits/s -> batched "
          f"is {batched_hits_per_s / rate:.1f}x faster", flush=True)
    return {"events": n_events, "hits_per_step": q["n_hits"], "ms_per_step": t * 1e3,
            "hits_per_s": rate, "events_per_s": n_events / t,
            "batched_over_per_task": batched_hits_per_s / rate}


def run_fp64_placement(torch, sim, w, dp, doff, out, cap, tuning, steps, warmup, fp32_hits_per_s):
    """The FP64 placement variant on the headline batch: its throughput
    (compact output, steps back to back as the headline) and the number of
    hits whose cell differs from the FP32 placement (both hit lists
    compared on the device), the quantity behind the paper's count of hits
    that CPU and GPU put in different cells."""
    def step():
        sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap, out=out,
                            hit_energy_scale=w.hit_energy_scale, async_launch=True,
                            placement_fp64=True, **tuning)

    for _ in range(warmup):
        step()
    sim.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    st = sim.synchronize()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    hits = st["n_hits"] // steps
    cells = {}
    for f64 in (False, True):
        r = sim.simulate_events(dp, doff, w.seed, outputs=("hits",),
                                hit_energy_scale=w.hit_energy_scale, placement_fp64=f64, **tuning)
        cells[f64] = r["hit_cell"]
        del r
    torch.cuda.synchronize()
    changed = int((cells[False] != cells[True]).sum().item())
    out_only = int(((cells[False] < 0) != (cells[True] < 0)).sum().item())
    del cells
    print(f"bench: FP64 placement {hits / dt:.4g} hits/s; {changed} of {hits} hits change cell "
          f"({out_only} at the acceptance edge)", flush=True)
    return {"hits_per_step": hits, "ms_per_step": dt * 1e3, "hits_per_s": hits / dt,
            "fp32_over_fp64": fp32_hits_per_s / (hits / dt), "hits_changing_cell": changed,
            "of_which_acceptance": out_only, "rate": changed / hits}


def run_hit_fluct(torch, sim, w, dp, doff, out, cap, tuning, steps, warmup, fp32_hits_per_s):
    """The per-hit energy fluctuation variant on the headline batch: its
    throughput (compact output, steps back to back as the headline) and the
    batch's deposited energy against the constant-energy chain (equal on
    average: the factor has mean 1)."""
    def step(**kw):
        sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap, out=out,
                            hit_energy_scale=w.hit_energy_scale, async_launch=True,
                            hit_energy_fluct=True, **tuning, **kw)

    for _ in range(warmup):
        step()
    sim.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    st = sim.synchronize()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    hits = st["n_hits"] // steps
    energy = {}
    for fl in (False, True):
        r = sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap,
                                out=out, hit_energy_scale=w.hit_energy_scale, hit_energy_fluct=fl,
                                **tuning)
        nnz = int(r["stats"]["n_cells_nonzero"])
        energy[fl] = float(out["cell_e"][:nnz].double().sum().item())
    print(f"bench: energy fluctuation {hits / dt:.4g} hits/s; deposited energy "
          f"{energy[True] / energy[False]:.6f} x the constant-energy chain", flush=True)
    return {"hits_per_step": hits, "ms_per_step": dt * 1e3, "hits_per_s": hits / dt,
            "fp32_over_variant": fp32_hits_per_s / (hits / dt),
            "energy_over_constant": energy[True] / energy[False]}


def run_ceilings(n_cells=191338, n_events_big=100):
    """Measured ceilings (libfcs_ceilings.so): FP32 device atomic adds into one
    event's cells (765 KB) and into a 100-event array (76.5 MB), uniform and
    in wave-sized "showers", with and without the returned value; an HBM
    copy; Philox4x32-10 draws per second with the shader clock under that
    load; and the cost of a launch (stream launches, hipGraph replays, a
    launch the host waits for).  Returns the record."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2103_14737_amd", "libfcs_ceilings.so"))
    d = C.c_double
    res = {"atomic_fp32_adds_per_s": {}}
    n_ops = 1 << 25
    for cells, label in ((n_cells, "765KB"), (n_cells * n_events_big, "76MB")):
        for pattern, pname in ((0, "uniform"), (1, "showers"), (2, "rows")):
            for ret in (0, 1):
                v = d()
                rc = lib.fcs_ceil_atomic(0, C.c_longlong(cells), C.c_longlong(n_ops), pattern, ret, 5,
                                         C.byref(v))
                assert rc == 0, rc
                key = f"{label}_{pname}_{'returning' if ret else 'no_return'}"
                res["atomic_fp32_adds_per_s"][key] = v.value
    v = d()
    assert lib.fcs_ceil_copy(0, C.c_longlong(1 << 30), 10, C.byref(v)) == 0
    res["hbm_copy_bytes_per_s"] = v.value
    draws, clk = d(), d()
    assert lib.fcs_ceil_philox(0, N_CU * 8, 4096, C.byref(draws), C.byref(clk)) == 0
    res["philox"] = {"draws_per_s": draws.value, "clock_hz": clk.value,
                     "slots_per_draw": PHILOX_SLOTS,
                     "lane_slots_per_s": draws.value * PHILOX_SLOTS,
                     "frac_of_valu_peak": draws.value * PHILOX_SLOTS / VALU_SLOT_PEAK,
                     "valu_peak_at_measured_clock": N_CU * 64 * clk.value,
                     "frac_at_measured_clock": draws.value * PHILOX_SLOTS / (N_CU * 64 * clk.value)}
    res["d2h_pinned_bytes_per_s"] = {}
    for mb in (1, 12, 48):
        v2 = d()
        assert lib.fcs_ceil_d2h(0, C.c_longlong(mb << 20), 10, C.byref(v2)) == 0
        res["d2h_pinned_bytes_per_s"][f"{mb}MB"] = v2.value
    a, b, c_ = d(), d(), d()
    assert lib.fcs_ceil_launch(0, 10000, 100, 2000, C.byref(a), C.byref(b), C.byref(c_)) == 0
    res["launch_us"] = {"stream": a.value, "graph": b.value, "host_waited": c_.value}
    at = res["atomic_fp32_adds_per_s"]
    print(f"bench: ceilings: atomics 765KB uniform {at['765KB_uniform_no_return']:.3g}/s "
          f"(returning {at['765KB_uniform_returning']:.3g}), 76MB uniform "
          f"{at['76MB_uniform_no_return']:.3g}/s (returning {at['76MB_uniform_returning']:.3g}), "
          f"showers {at['76MB_showers_no_return']:.3g}/s, rows {at['76MB_rows_no_return']:.3g}/s; "
          f"HBM copy {v.value / 1e12:.2f} TB/s; D2H to pinned host "
          f"{res['d2h_pinned_bytes_per_s']['48MB'] / 1e9:.1f} GB/s; "
          f"Philox {draws.value:.3g} draws/s at {clk.value / 1e9:.2f} GHz; launch "
          f"{a.value:.2f} us stream, {b.value:.2f} us graph, {c_.value:.1f} us host-waited",
          flush=True)
    return res


def roofline(hits, kernel_ms, workload, tuning):
    """The roofline object of the hit step (window pass + hit kernel, the
    dominant kernels; the task scans run beside the window pass and are
    inside the timed span) from its HIP-event time per launch: algorithmic
    VALU instruction slots per launch over that time, against the chip's
    issue rate at the nominal clock."""
    achieved = SLOTS_PER_HIT * hits / (kernel_ms * 1e-3)
    return {"kernel": "hit step (k_windows + k_hits)", "bound": "alu",
            "achieved": achieved / 1e12, "peak": VALU_SLOT_PEAK / 1e12,
            "unit": "T VALU lane-instruction slots/s", "frac": achieved / VALU_SLOT_PEAK,
            "traffic": measured_traffic(workload, tuning),
            "kernel_source_hash": kernel_source_hash(), "slots_per_hit": SLOTS_PER_HIT,
            "ops_per_hit": OPS_PER_HIT, "hits_per_launch": hits, "kernel_ms": kernel_ms}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fwd-bwd-only", action="store_true",
                    help="time only the forward + backward section and print its figures "
                         "(for profiling; not the benchmark line)")
    ap.add_argument("--fp64-placement-only", action="store_true",
                    help="time only the FP64 placement variant on the headline batch")
    ap.add_argument("--fine-tables-only", action="store_true",
                    help="time only the headline batch on 64 x 64-bin tables")
    ap.add_argument("--ceilings-only", action="store_true",
                    help="measure only the chip's ceilings and print them")
    ap.add_argument("--sharing-only", action="store_true",
                    help="time only the concurrent-jobs study and print its figures")
    ap.add_argument("--only-headline", action="store_true",
                    help="time only the headline batched workload (for profiling)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default tuning instead of the autotuner's")
    ap.add_argument("--tuning", type=str, default="",
                    help="chunk_hits,big_task_hits,tile_hits,wg_per_cu[,window_particles] "
                         "(skips the autotuner)")
    ap.add_argument("--workload", default="pileup",
                    choices=["single_particle_sweep", "hard_scatter", "pileup"],
                    help="headline workload to time (the other choices are for profiling)")
    ap.add_argument("--host-copy-workgroups", type=int, default=0,
                    help="workgroups of the copy kernel to the host buffers (0: tuned per workload)")
    ap.add_argument("--device-outputs", action="store_true",
                    help="headline steps leave their lists in device memory (for profiling)")
    ap.add_argument("--write-tuning", type=str, default="",
                    help="write the tuning used as chunk,big,tile,wg,window_particles to this file")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); events shard "
              "across GPUs by event range with no communication between them.",
              file=sys.stderr)
        return 2

    import torch
    from paper_2103_14737_amd import workloads as W
    from paper_2103_14737_amd.fcs import Simulator, particles_to_device

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    geo, par = W.make_geometry(), W.make_param()
    sim = Simulator(0)
    t0 = time.perf_counter()
    sim.load_geometry(geo)
    sim.load_parametrization(par)
    load_ms = (time.perf_counter() - t0) * 1e3

    if args.fwd_bwd_only:
        tun = parse_tuning(args.tuning) if args.tuning else None
        print(json.dumps(run_fwd_bwd(torch, sim, geo, par, dev, args.steps, args.warmup, tun)),
              flush=True)
        return 0
    if args.ceilings_only:
        print(json.dumps(run_ceilings()), flush=True)
        return 0
    if args.sharing_only:
        print(json.dumps(run_sharing(torch, geo, par, dev)), flush=True)
        return 0
    if args.fine_tables_only:
        w = W.BY_NAME["single_particle_sweep"]()
        print(json.dumps(run_fine_tables(torch, geo, dev, w, {}, args.steps, args.warmup)),
              flush=True)
        return 0

    def prepare(w, outputs=("compact",)):
        dp = particles_to_device(w.particles, dev)
        doff = torch.from_numpy(w.event_offsets).to(dev)
        q = sim.query_sizes(dp, doff, w.seed, hit_energy_scale=w.hit_energy_scale)
        out = {}
        cap = q["max_cells"]
        if "compact" in outputs:
            out["cell_ids"] = torch.empty(cap, dtype=torch.int64, device=dev)
            out["cell_e"] = torch.empty(cap, dtype=torch.float32, device=dev)
            out["event_cell_offsets"] = torch.empty(w.n_events + 1, dtype=torch.int64, device=dev)
        if "dense" in outputs:
            out["cells"] = torch.empty((w.n_events, geo["n_cells"]), dtype=torch.float32,
                                       device=dev)
        return dp, doff, out, cap, q

    if args.fp64_placement_only:
        w = W.BY_NAME["single_particle_sweep"]()
        dp, doff, out, cap, q = prepare(w)
        print(json.dumps(run_fp64_placement(torch, sim, w, dp, doff, out, cap, {}, args.steps,
                                            args.warmup, float("nan"))), flush=True)
        print(json.dumps(run_hit_fluct(torch, sim, w, dp, doff, out, cap, {}, args.steps,
                                       args.warmup, float("nan"))), flush=True)
        return 0

    def tune_for(w, dp, doff, out, cap):
        if args.tuning:
            return parse_tuning(args.tuning)
        if args.no_autotune:
            return {}
        from paper_2103_14737_amd import autotune
        t0 = time.perf_counter()
        tun = autotune.tune(sim, dp, doff, w.seed, out=out, cell_capacity=cap,
                            hit_energy_scale=w.hit_energy_scale,
                            verbose=bool(os.environ.get("FCS_TUNE_VERBOSE")))
        print(f"bench: {w.name}: autotuned {tun} in {time.perf_counter() - t0:.1f} s", flush=True)
        return tun

    def batched(w, dp, doff, out, cap, tun, steps, warmup, host_out, profile):
        """K asynchronous calls back to back between two synchronizations;
        with host_out the lists go to two sets of pinned host buffers in
        turn, sized to the batch's compacted total (+2 %), by the copy
        kernel (its workgroups tuned per workload).  With profile each call
        brackets its hit step with an event pair.  Returns (s per step, hit-step ms per launch or
        None, totals, host capacity)."""
        cap_h = cap
        if host_out:
            r0 = sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap,
                                     out=out, hit_energy_scale=w.hit_energy_scale, **tun)
            cap_h = int(r0["stats"]["n_cells_nonzero"] * 1.02) + 64
            hbufs = [{"cell_ids": sim.host_empty((cap_h,), np.int64),
                      "cell_e": sim.host_empty((cap_h,), np.float32),
                      "event_cell_offsets": sim.host_empty((w.n_events + 1,), np.int64)}
                     for _ in range(2)]
            if host_wgs.get(w.name) is None:
                if args.host_copy_workgroups:
                    host_wgs[w.name] = args.host_copy_workgroups
                else:
                    from paper_2103_14737_amd import autotune
                    host_wgs[w.name] = autotune.tune_host_copy(
                        sim, dp, doff, w.seed, hbufs, cap_h, hit_energy_scale=w.hit_energy_scale,
                        tuning=tun)
                    print(f"bench: {w.name}: copy kernel to the host with {host_wgs[w.name]} "
                          f"workgroups", flush=True)

        def step(i):
            sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap_h,
                                out=hbufs[i % 2] if host_out else out, profile=profile,
                                hit_energy_scale=w.hit_energy_scale, async_launch=True,
                                host_outputs=host_out,
                                host_copy_workgroups=host_wgs.get(w.name) or 0, **tun)

        for i in range(warmup):
            step(i)
        sim.synchronize()
        _sync(torch)
        t0 = time.perf_counter()
        for i in range(steps):
            step(i)
        st = sim.synchronize()
        _sync(torch)
        dt = (time.perf_counter() - t0) / steps
        assert st["n_calls"] == steps and st["n_hits"] == steps * q_hits[w.name], st
        if host_out:  # the copies hold what the device compacted
            ref = sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap,
                                      out=out, hit_energy_scale=w.hit_energy_scale, **tun)
            nnz = ref["stats"]["n_cells_nonzero"]
            hb = hbufs[(steps - 1) % 2]
            assert np.array_equal(hb["event_cell_offsets"], out["event_cell_offsets"].cpu().numpy())
            assert np.array_equal(hb["cell_ids"][:nnz], out["cell_ids"][:nnz].cpu().numpy())
        return dt, (st["kernel_ms"] / steps if profile else None), st, cap_h

    def per_event(w, dp, doff, out, cap, tun, steps=2):
        def step():
            r = sim.simulate_events(dp, doff, w.seed, mode="per_event", outputs=("compact",),
                                    cell_capacity=cap, out=out,
                                    hit_energy_scale=w.hit_energy_scale, **tun)
            return r["stats"]["n_hits"]
        t, res = _time_steps(torch, step, steps, 1)
        assert all(h == q_hits[w.name] for h in res)
        return t

    def per_event_best(w, dp, doff, out, cap, tun, steps):
        """The per-event form at its own best tuning: the batched form's
        tuning and its variants in the task split (and window size), each
        timed over two steps, the fastest then over `steps`."""
        cands = [dict(tun)] if tun else [{}]
        if tun:
            for b in (64, 128, 256):
                for wp in ((1024, 2048) if tun.get("window_particles") else (None,)):
                    c = dict(tun, big_task_hits=b)
                    if wp:
                        c["window_particles"] = wp
                    if c not in cands:
                        cands.append(c)
        times = [per_event(w, dp, doff, out, cap, c, steps=2) for c in cands]
        best = cands[int(np.argmin(times))]
        return per_event(w, dp, doff, out, cap, best, steps=steps), best, len(cands)

    q_hits = {}
    host_wgs = {}  # workgroups of the copy kernel to host buffers, per workload

    # ------------------------------------------------ headline: pile-up batch
    w = W.BY_NAME[args.workload]()
    dp, doff, out, cap, q = prepare(w)
    q_hits[w.name] = hits_per_step = q["n_hits"]
    print(f"bench: {w.name}: {w.n_events} events, {hits_per_step} hits per step", flush=True)
    tuning = tune_for(w, dp, doff, out, cap)
    if args.write_tuning:
        with open(args.write_tuning, "w") as f:
            f.write(",".join(str((tuning or {}).get(k, 0)) for k in TUNING_KEYS))
    host_out = not args.device_outputs
    # the timed steps run as a user's would: unprofiled (graph launches);
    # the hit step's duration for the roofline comes from a profiled pass of
    # the same batch with the lists in device memory
    t_step, _, st, cap_h = batched(w, dp, doff, out, cap, tuning, args.steps, args.warmup,
                                   host_out, False)
    value = hits_per_step / t_step
    nnz = st["n_cells_nonzero"] // args.steps
    t_dev, kernel_ms, _, _ = batched(w, dp, doff, out, cap, tuning, args.steps, args.warmup,
                                     False, True)
    print(f"bench: batched {t_step * 1e3:.3f} ms/step, {value:.4g} hits/s "
          f"({'lists copied to pinned host buffers' if host_out else 'lists in device memory'}); "
          f"profiled pass, lists in device memory: {t_dev * 1e3:.3f} ms/step, hit step "
          f"{kernel_ms:.3f} ms", flush=True)

    line = {
        "metric": METRIC, "value": value, "unit": "hits/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_events": w.n_events,
                   "n_particles": w.n_particles, "seed": w.seed,
                   "hit_energy_scale_MeV": w.hit_energy_scale, "n_cells": geo["n_cells"],
                   "mode": "batched",
                   "outputs": ("compact (cell_id, E) per event, copied to pinned host buffers "
                               "inside each step") if host_out else
                              "compact (cell_id, E) per event, in device memory",
                   "hits_per_step": hits_per_step, "cells_per_step": nnz,
                   "tuning": tuning or "library defaults",
                   "host_copy_workgroups": host_wgs.get(w.name) if host_out else None},
        "events_per_s": w.n_events / t_step,
        "geometry_param_load_ms": load_ms,
    }
    line["roofline"] = roofline(hits_per_step, kernel_ms, args.workload, tuning)
    line["d2h_bytes_per_step"] = nnz * 12 + (w.n_events + 1) * 8 if host_out else 0

    line["device_resident"] = {"ms_per_step": t_dev * 1e3, "hits_per_s": hits_per_step / t_dev,
                               "hit_step_ms": kernel_ms, "profiled": True}
    if not args.only_headline:
        t_dev0, _, _, _ = batched(w, dp, doff, out, cap, tuning, args.steps, args.warmup, False,
                                  False)
        line["device_resident"].update(ms_per_step_unprofiled=t_dev0 * 1e3,
                                       hits_per_s_unprofiled=hits_per_step / t_dev0)
        print(f"bench: lists kept in device memory, unprofiled: {t_dev0 * 1e3:.3f} ms/step",
              flush=True)
        # the same batch as synchronous calls (each waits for its results)
        wall = []

        def step_sync():
            t0 = time.perf_counter()
            r = sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap,
                                    out=out, hit_energy_scale=w.hit_energy_scale, **tuning)
            wall.append(time.perf_counter() - t0)
            return r["stats"]["n_hits"]

        t_sync, _ = _time_steps(torch, step_sync, args.steps, 1)
        wall_ms = np.array(wall[-args.steps:]) * 1e3
        line["synchronous_calls"] = {"ms_per_step": t_sync * 1e3,
                                     "hits_per_s": hits_per_step / t_sync,
                                     "median_ms": float(np.median(wall_ms)),
                                     "std_ms": float(np.std(wall_ms))}
        t_pe, tun_pe, n_tried = per_event_best(w, dp, doff, out, cap, tuning, steps=5)
        line["per_event_launch"] = {"ms_per_step": t_pe * 1e3, "hits_per_s": hits_per_step / t_pe,
                                    "events_per_s": w.n_events / t_pe, "steps": 5,
                                    "outputs": "compact, device memory",
                                    "tuning": tun_pe or "library defaults",
                                    "tunings_tried": n_tried}
        # both forms unprofiled, lists in device memory
        line["batched_over_per_event"] = t_pe / t_dev0
        print(f"bench: per-event {t_pe * 1e3:.2f} ms/step (best of {n_tried} tunings: {tun_pe}) -> "
              f"batched (device lists) is {t_pe / t_dev0:.2f}x faster", flush=True)

        # -------------------------------------------- the other two batches
        others = {}
        for key_o, wo in (("hard_scatter", W.hard_scatter()),
                          ("single_particle_sweep", W.single_particle_sweep())):
            dpo, doffo, outo, capo, qo = prepare(wo)
            q_hits[wo.name] = qo["n_hits"]
            tun_o = tune_for(wo, dpo, doffo, outo, capo)
            n_o = max(2, args.steps)
            t_h, _, st_h, _ = batched(wo, dpo, doffo, outo, capo, tun_o, n_o, args.warmup, True,
                                      False)
            t_d, k_d, _, _ = batched(wo, dpo, doffo, outo, capo, tun_o, n_o, args.warmup, False,
                                     True)
            t_d0, _, _, _ = batched(wo, dpo, doffo, outo, capo, tun_o, n_o, args.warmup, False,
                                    False)
            # the sweep's per-event form (10,000 launches, ~0.8 s a step) keeps
            # the batched form's tuning
            if wo.name.startswith("single_particle_sweep"):
                n_pe, tun_pe_o, n_tried_o = 2, tun_o, 1
                t_pe_o = per_event(wo, dpo, doffo, outo, capo, tun_o, steps=n_pe)
            else:
                n_pe = 5
                t_pe_o, tun_pe_o, n_tried_o = per_event_best(wo, dpo, doffo, outo, capo, tun_o, n_pe)
            rec = {"hits_per_step": qo["n_hits"], "ms_per_step": t_h * 1e3,
                   "hits_per_s": qo["n_hits"] / t_h, "events_per_s": wo.n_events / t_h,
                   "outputs": "compact, copied to pinned host buffers",
                   "host_copy_workgroups": host_wgs.get(wo.name),
                   "device_resident": {"ms_per_step": t_d0 * 1e3, "hits_per_s": qo["n_hits"] / t_d0,
                                       "ms_per_step_profiled": t_d * 1e3},
                   "hit_energy_scale_MeV": wo.hit_energy_scale,
                   "tuning": tun_o or "library defaults",
                   "per_event_launch": {"ms_per_step": t_pe_o * 1e3,
                                        "hits_per_s": qo["n_hits"] / t_pe_o,
                                        "events_per_s": wo.n_events / t_pe_o, "steps": n_pe,
                                        "tuning": tun_pe_o or "library defaults",
                                        "tunings_tried": n_tried_o},
                   "batched_over_per_event": t_pe_o / t_d0,
                   "roofline": roofline(qo["n_hits"], k_d, key_o, tun_o)}
            n_pt = 5 if wo.name.startswith("hard") else 500
            rec["per_task_launch"] = run_per_task(torch, sim, prepare, wo, n_pt, qo["n_hits"] / t_d0)
            others[wo.name] = rec
            print(f"bench: {wo.name} {qo['n_hits'] / t_h:.4g} hits/s with the copies "
                  f"({qo['n_hits'] / t_d0:.4g} device lists); per-event {t_pe_o * 1e3:.1f} ms/step "
                  f"-> batched is {t_pe_o / t_d0:.1f}x faster; hit step {k_d:.3f} ms", flush=True)
            if wo.name.startswith("single_particle_sweep"):
                sweep = (wo, dpo, doffo, outo, capo, tun_o, qo["n_hits"] / t_d0)
            else:
                del dpo, doffo, outo
        line["other_workloads"] = others
        line["fwd_bwd"] = run_fwd_bwd(torch, sim, geo, par, dev, args.steps, args.warmup)
        line["gpu_sharing"] = run_sharing(torch, geo, par, dev)
        ws, dps, doffs, outs, caps, tuns, rate_s = sweep
        line["fine_tables"] = run_fine_tables(torch, geo, dev, ws, tuns, args.steps, args.warmup)
        line["placement_fp64"] = run_fp64_placement(torch, sim, ws, dps, doffs, outs, caps, tuns,
                                                    args.steps, args.warmup, rate_s)
        line["hit_energy_fluct"] = run_hit_fluct(torch, sim, ws, dps, doffs, outs, caps, tuns,
                                                 args.steps, args.warmup, rate_s)
        line["ceilings"] = run_ceilings()
        ph = line["ceilings"]["philox"]
        line["roofline"]["frac_at_measured_clock"] = (
            line["roofline"]["achieved"] * 1e12 / ph["valu_peak_at_measured_clock"])
        line["roofline"]["measured_ceiling"] = {
            "philox_only_lane_slots_per_s": ph["lane_slots_per_s"], "clock_hz": ph["clock_hz"]}

    if args.copy_probe_mb:
        # a plain device copy of known size: the HBM counters of the profiled
        # kernels are scaled by what the same counters read for this copy
        n = args.copy_probe_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = n * 4

    # ------------------------------------------------- CPU oracle baseline
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = oracle_baseline(w, geo, par)

    sim.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
