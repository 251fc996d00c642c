"""Benchmark of the batched hit simulation on one MI355X.

One step = one fcs_simulate_events call over the whole batch in batched mode
(per-(particle, layer) setup, work-queue build, persistent hit kernel,
ordered compaction and accumulator reset), inputs and outputs resident in
device memory.  The headline workload is the single-particle sweep: 10,000
events of one e/gamma/pi+- each, E log-uniform 1 GeV - 4 TeV, |eta| < 2.5.

Also reported on the same JSON line: the same batch as synchronous calls;
the per-event launch form (one launch sequence and one host synchronization
per event) and the per-(particle, layer) launch form (on a slice); the
forward+backward throughput of the differentiable workload (64 single
pions); the multi-particle workloads (hard scatter, pile-up) in the batched
and per-event forms; several jobs sharing the GPU (1 to 16 contexts on host
threads); the headline batch on 64 x 64-bin tables, with the FP64
placement variant (with the count of hits that change cell) and with the
per-hit energy fluctuation variant; the device-atomic ceiling (FP32
atomic adds into one event's cells, uniform and at a hot spot); the
roofline of the hit kernel; and the CPU oracle timed on the host (one thread and
threads over event ranges).

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
VALU_LANE_OPS_PEAK = N_CU * 64 * CLOCK_HZ       # 32-bit VALU lane-ops per second
HBM_PEAK = 8.0e12

# Algorithmic 32-bit operations per hit (a 32x32->64 product counts as its two
# 32-bit halves): Philox4x32-10 = 10 rounds x (2 products = 4 + 4 xor) = 80
# (the key schedule is shared by all hits); three 24-bit uniforms (shift,
# convert, scale) = 9; bin choice from the guide table (index + ~2 compares)
# = 3; radial / angular bin split = 2; radius = 4; octant sine and cosine
# (offset, square, 4 + 5 multiply-add steps, final multiply, quadrant select)
# = 24; deta / dphi = 4; eta / phi = 2; phi wrap = 3; region-grid lookup
# (acceptance, region, two floor-and-clamp indices, linear index) = 22;
# deposit = 1.
OPS_PER_HIT = 80 + 9 + 3 + 2 + 4 + 24 + 4 + 2 + 3 + 22 + 1
KERNEL_SOURCES = ("paper_2103_14737_amd/csrc/fcs_math.hpp",
                  "paper_2103_14737_amd/csrc/fcs_kernels.hpp",
                  "paper_2103_14737_amd/csrc/fcs_runtime.hip",
                  "paper_2103_14737_amd/build.py")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_hits_traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, tuning):
    """HBM bytes per launch of the hit kernel from the committed counter
    summaries: the entry taken on the current kernel sources, this workload
    and this tuning, if there is one; else None."""
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


def oracle_baseline(w, geo, par, max_threads=16, budget_one=10.0, budget_all=5.0):
    """The oracle timed on the host: whole passes over the workload on one
    thread (until about `budget_one` s, at most 5 passes), then the same
    workload split into event ranges run by independent threads at once
    (the oracle is re-entrant and releases the interpreter lock while it
    runs; at most `max_threads`, the CPU share of one GPU) until about
    `budget_all` s.  Median passes; returns the cpu_baseline record."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_2103_14737_amd import workloads as W
    oracle.build(force=False)
    go, po = oracle.Geometry(geo), oracle.Param(par)

    def run(sw):
        return oracle.simulate(go, po, sw.particles, sw.event_offsets, sw.seed,
                               event_index_base=sw.notes.get("event_index_base", 0),
                               hit_energy_scale=sw.hit_energy_scale)["n_hits_total"]

    runs = []
    while not runs or (len(runs) < 5 and sum(runs) < budget_one):
        t0 = time.perf_counter()
        total = run(w)
        runs.append(time.perf_counter() - t0)
    dt = sorted(runs)[len(runs) // 2]
    one = {"value": total / dt, "cores": 1,
           "sample": f"the whole {w.name} workload ({w.n_events} events, {total} hits), one "
                     f"thread, median of {len(runs)} passes ({sum(runs):.1f} s in all)"}
    print(f"bench: oracle {one['value']:.4g} hits/s on 1 core", flush=True)
    n_thr = max(1, min(max_threads, len(os.sched_getaffinity(0)), w.n_events))
    bounds = np.linspace(0, w.n_events, n_thr + 1).astype(int)
    parts = [W.subset_events(w, int(a), int(b - a)) for a, b in zip(bounds[:-1], bounds[1:])
             if b > a]
    runs_n = []
    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        while not runs_n or (len(runs_n) < 10 and sum(runs_n) < budget_all):
            t0 = time.perf_counter()
            tot = sum(ex.map(run, parts))
            runs_n.append(time.perf_counter() - t0)
            assert tot == total, (tot, total)
    dt_n = sorted(runs_n)[len(runs_n) // 2]
    print(f"bench: oracle {total / dt_n:.4g} hits/s on {len(parts)} cores", flush=True)
    return {"value": total / dt_n, "unit": "hits/s", "cores": len(parts), "kind": "oracle",
            "sample": f"the whole {w.name} workload ({w.n_events} events, {total} hits) split "
                      f"into {len(parts)} event ranges run by {len(parts)} threads at once, "
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


def run_atomic_ceiling(torch, dev, n_cells=191338, n_ops=1 << 25, reps=5):
    """The device-atomic ceiling of a deposit of one atomic per hit: FP32
    atomic adds into one event's cell array (191,338 cells, 765 KB) through
    torch's index_add_ (one atomic add per element on this GPU), at
    uniformly random cells and at a shower-like hot spot (cells at an
    exponentially distributed distance, mean 8 cells, from one centre).
    Atomic adds per second; the hit kernel's privatized deposit (hits
    counted per cell in LDS) is compared against it."""
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    cells = torch.zeros(n_cells, dtype=torch.float32, device=dev)
    vals = torch.ones(n_ops, dtype=torch.float32, device=dev)
    idx_u = torch.randint(0, n_cells, (n_ops,), device=dev, generator=g)
    dist = torch.empty(n_ops, dtype=torch.float32, device=dev).exponential_(1.0 / 8.0, generator=g)
    sign = torch.randint(0, 2, (n_ops,), device=dev, generator=g) * 2 - 1
    idx_h = (n_cells // 2 + sign * dist.long()).clamp_(0, n_cells - 1)
    res = {"cells": n_cells, "atomics_per_pass": n_ops}
    for name, idx in (("uniform", idx_u), ("hot_spot", idx_h)):
        cells.index_add_(0, idx, vals)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            cells.index_add_(0, idx, vals)
        torch.cuda.synchronize()
        res[f"{name}_per_s"] = n_ops * reps / (time.perf_counter() - t0)
    print(f"bench: FP32 atomic adds into 765 KB: {res['uniform_per_s']:.3g}/s uniform, "
          f"{res['hot_spot_per_s']:.3g}/s at a hot spot", flush=True)
    return res


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
    ap.add_argument("--sharing-only", action="store_true",
                    help="time only the concurrent-jobs study and print its figures")
    ap.add_argument("--only-headline", action="store_true",
                    help="time only the headline batched workload (for profiling)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default tuning instead of the autotuner's")
    ap.add_argument("--tuning", type=str, default="",
                    help="chunk_hits,big_task_hits,tile_hits,wg_per_cu (skips the autotuner)")
    ap.add_argument("--workload", default="single_particle_sweep",
                    choices=["single_particle_sweep", "hard_scatter", "pileup"],
                    help="headline workload to time (the other choices are for profiling)")
    ap.add_argument("--write-tuning", type=str, default="",
                    help="write the tuning used as chunk,big,tile,wg to this file")
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
        tun = None
        if args.tuning:
            c_, b_, t_, w_ = (int(x) for x in args.tuning.split(","))
            tun = dict(chunk_hits=c_, big_task_hits=b_, tile_hits=t_, wg_per_cu=w_)
        print(json.dumps(run_fwd_bwd(torch, sim, geo, par, dev, args.steps, args.warmup, tun)),
              flush=True)
        return 0
    if args.sharing_only:
        print(json.dumps(run_sharing(torch, geo, par, dev)), flush=True)
        return 0
    if args.fine_tables_only:
        w = W.BY_NAME[args.workload]()
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
        w = W.BY_NAME[args.workload]()
        dp, doff, out, cap, q = prepare(w)
        print(json.dumps(run_fp64_placement(torch, sim, w, dp, doff, out, cap, {}, args.steps,
                                            args.warmup, float("nan"))), flush=True)
        print(json.dumps(run_hit_fluct(torch, sim, w, dp, doff, out, cap, {}, args.steps,
                                       args.warmup, float("nan"))), flush=True)
        return 0

    # ------------------------------------------------ headline: batched sweep
    w = W.BY_NAME[args.workload]()
    dp, doff, out, cap, q = prepare(w)
    hits_per_step = q["n_hits"]
    print(f"bench: {w.name}: {w.n_events} events, {hits_per_step} hits per step", flush=True)
    tuning = {}
    if args.tuning:
        c_, b_, t_, w_ = (int(x) for x in args.tuning.split(","))
        tuning = dict(chunk_hits=c_, big_task_hits=b_, tile_hits=t_, wg_per_cu=w_)
    elif not args.no_autotune:
        from paper_2103_14737_amd import autotune
        t0 = time.perf_counter()
        tuning = autotune.tune(sim, dp, doff, w.seed, out=out, cell_capacity=cap,
                               hit_energy_scale=w.hit_energy_scale,
                               verbose=bool(os.environ.get("FCS_TUNE_VERBOSE")))
        print(f"bench: autotuned {tuning} in {time.perf_counter() - t0:.1f} s", flush=True)
    if args.write_tuning:
        with open(args.write_tuning, "w") as f:
            t_ = tuning or {}
            f.write(",".join(str(t_.get(k, 0)) for k in ("chunk_hits", "big_task_hits",
                                                          "tile_hits", "wg_per_cu")))
    stats = []

    # Timed steps: the batch is enqueued K times back to back (asynchronous
    # calls, as a serving loop issues them) between two device
    # synchronizations; the hit kernel of every step is timed with HIP events
    # on the library's stream.  fcs_synchronize returns the steps' totals.
    def step_async():
        sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap, out=out,
                            profile=True, hit_energy_scale=w.hit_energy_scale, async_launch=True,
                            **tuning)

    for _ in range(args.warmup):
        step_async()
    sim.synchronize()
    _sync(torch)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_async()
    st = sim.synchronize()
    _sync(torch)
    t_step = (time.perf_counter() - t0) / args.steps
    assert st["n_calls"] == args.steps and st["n_hits"] == args.steps * hits_per_step, st
    kernel_ms = st["kernel_ms"] / args.steps
    value = hits_per_step / t_step
    print(f"bench: batched {t_step * 1e3:.3f} ms/step, {value:.4g} hits/s, "
          f"hit kernel {kernel_ms:.3f} ms", flush=True)

    # the same batch as synchronous calls (each waits for its results)
    wall = []

    def step_batched(profile=False):
        t0 = time.perf_counter()
        r = sim.simulate_events(dp, doff, w.seed, outputs=("compact",), cell_capacity=cap,
                                out=out, profile=profile, hit_energy_scale=w.hit_energy_scale,
                                **tuning)
        wall.append(time.perf_counter() - t0)
        stats.append(r["stats"])
        return r["stats"]["n_hits"]

    t_sync, _ = _time_steps(torch, step_batched, args.steps, 1)
    timed = stats[-args.steps:]
    assert all(s["n_hits"] == hits_per_step for s in timed)
    call_ms = float(np.mean([s["device_ms"] for s in timed]))
    wall_ms = np.array(wall[-args.steps:]) * 1e3
    print(f"bench: synchronous calls {t_sync * 1e3:.3f} ms/step", flush=True)

    line = {
        "metric": METRIC, "value": value, "unit": "hits/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_events": w.n_events,
                   "n_particles": w.n_particles, "seed": w.seed,
                   "hit_energy_scale_MeV": w.hit_energy_scale, "n_cells": geo["n_cells"],
                   "mode": "batched", "outputs": "compact (cell_id, E) per event",
                   "hits_per_step": hits_per_step, "tuning": tuning or "library defaults"},
        "events_per_s": w.n_events / t_step,
        "synchronous_calls": {"ms_per_step": t_sync * 1e3, "hits_per_s": hits_per_step / t_sync,
                              "device_ms_per_call": call_ms,
                              "median_ms": float(np.median(wall_ms)),
                              "std_ms": float(np.std(wall_ms))},
        "geometry_param_load_ms": load_ms,
    }
    # roofline of the dominant kernel (the persistent hit kernel)
    ops = OPS_PER_HIT * hits_per_step
    achieved = ops / (kernel_ms * 1e-3)
    # context: one device atomic per hit could not reach this rate
    if not args.only_headline:
        ceil = run_atomic_ceiling(torch, dev)
        ceil["hits_per_s_over_uniform"] = value / ceil["uniform_per_s"]
        ceil["hits_per_s_over_hot_spot"] = value / ceil["hot_spot_per_s"]
        line["atomic_ceiling"] = ceil
    line["roofline"] = {"kernel": "k_hits", "bound": "alu", "achieved": achieved / 1e12,
                        "peak": VALU_LANE_OPS_PEAK / 1e12, "unit": "Tops/s",
                        "frac": achieved / VALU_LANE_OPS_PEAK,
                        "traffic": measured_traffic(args.workload, tuning),
                        "kernel_source_hash": kernel_source_hash(),
                        "ops_per_hit": OPS_PER_HIT, "hits_per_launch": hits_per_step,
                        "kernel_ms": kernel_ms}

    if not args.only_headline and args.workload == "single_particle_sweep":
        # -------------------------------------------- per-event launch form
        pe_steps = max(1, min(2, args.steps))
        stats.clear()

        def step_per_event():
            r = sim.simulate_events(dp, doff, w.seed, mode="per_event", outputs=("compact",),
                                    cell_capacity=cap, out=out, **tuning)
            return r["stats"]["n_hits"]

        t_pe, res = _time_steps(torch, step_per_event, pe_steps, 1)
        assert all(h == hits_per_step for h in res)
        line["per_event_launch"] = {"ms_per_step": t_pe * 1e3,
                                    "hits_per_s": hits_per_step / t_pe,
                                    "events_per_s": w.n_events / t_pe, "steps": pe_steps}
        line["batched_over_per_event"] = t_pe / t_step
        print(f"bench: per-event {t_pe * 1e3:.1f} ms/step -> batched is "
              f"{t_pe / t_step:.1f}x faster", flush=True)

        line["per_task_launch"] = run_per_task(torch, sim, prepare, w, 500, value)

        line["fwd_bwd"] = run_fwd_bwd(torch, sim, geo, par, dev, args.steps, args.warmup)

        # ---------------------------------------- multi-particle workloads
        others = {}
        for wo in (W.hard_scatter(), W.pileup()):
            dpo, doffo, outo, capo, qo = prepare(wo)

            tun_o = {}
            if not args.no_autotune:
                from paper_2103_14737_amd import autotune
                tun_o = autotune.tune(sim, dpo, doffo, wo.seed, out=outo, cell_capacity=capo,
                                      hit_energy_scale=wo.hit_energy_scale)

            def step_o():
                sim.simulate_events(dpo, doffo, wo.seed, outputs=("compact",),
                                    cell_capacity=capo, out=outo,
                                    hit_energy_scale=wo.hit_energy_scale, async_launch=True,
                                    **tun_o)

            n_o = max(2, args.steps // 2)
            step_o()
            sim.synchronize()
            _sync(torch)
            t0 = time.perf_counter()
            for _ in range(n_o):
                step_o()
            st_o = sim.synchronize()
            _sync(torch)
            t_o = (time.perf_counter() - t0) / n_o
            assert st_o["n_hits"] == n_o * qo["n_hits"], st_o

            # the per-event launch form of the same batch
            def step_o_pe():
                r = sim.simulate_events(dpo, doffo, wo.seed, mode="per_event", outputs=("compact",),
                                        cell_capacity=capo, out=outo,
                                        hit_energy_scale=wo.hit_energy_scale, **tun_o)
                return r["stats"]["n_hits"]

            t_pe_o, res_o = _time_steps(torch, step_o_pe, 2, 1)
            assert all(h == qo["n_hits"] for h in res_o)
            others[wo.name] = {"hits_per_step": qo["n_hits"], "ms_per_step": t_o * 1e3,
                               "hits_per_s": qo["n_hits"] / t_o,
                               "events_per_s": wo.n_events / t_o,
                               "hit_energy_scale_MeV": wo.hit_energy_scale,
                               "tuning": tun_o or "library defaults",
                               "per_event_launch": {"ms_per_step": t_pe_o * 1e3,
                                                    "hits_per_s": qo["n_hits"] / t_pe_o,
                                                    "events_per_s": wo.n_events / t_pe_o,
                                                    "steps": 2},
                               "batched_over_per_event": t_pe_o / t_o}
            if wo.name.startswith("hard_scatter"):
                others[wo.name]["per_task_launch"] = run_per_task(
                    torch, sim, prepare, wo, 5, qo["n_hits"] / t_o)
            print(f"bench: {wo.name} {qo['n_hits'] / t_o:.4g} hits/s; per-event "
                  f"{t_pe_o * 1e3:.1f} ms/step -> batched is {t_pe_o / t_o:.1f}x faster", flush=True)
            del dpo, doffo, outo
        line["other_workloads"] = others
        line["gpu_sharing"] = run_sharing(torch, geo, par, dev)
        line["fine_tables"] = run_fine_tables(torch, geo, dev, w, tuning, args.steps, args.warmup)
        line["placement_fp64"] = run_fp64_placement(torch, sim, w, dp, doff, out, cap, tuning,
                                                    args.steps, args.warmup, value)
        line["hit_energy_fluct"] = run_hit_fluct(torch, sim, w, dp, doff, out, cap, tuning,
                                                 args.steps, args.warmup, value)

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
