"""Autotuner for the batched launch: picks chunk size, large-task threshold,
tile size (or, for events of many particles, the window pass's particles
per work item) and persistent workgroups per CU for a workload by timing the
candidates on the device, and caches the choice in a JSON file keyed by the
device and a signature of the workload.

The tuning never changes hit counts, hit positions or cell indices (only the
FP32 summation order of cell energies), so any candidate is a valid result.
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "fcs_mi355x_tune.json")

# (chunk_hits, big_task_hits, tile_hits, wg_per_cu, window_particles)
CANDIDATES = [
    (c, b, t, w, 0)
    for c in (1024, 2048, 4096, 8192)
    for b in (32, 64, 128, 256)
    for t in (256, 512)
    for w in (3, 4, 5, 8)
    if b <= t
]
# batches of many particles per event deposit their small tasks by cell
# windows (the tiles are not used): the window pass's particles per work item
# replace the tile size
WINDOW_CANDIDATES = [
    (c, b, 512, w, p)
    for c in (1024, 2048, 4096)
    for b in (64, 128, 256)
    for w in (4, 8)
    for p in (1024, 2048)
]
# the library's rule for the window pass (particles per event on average)
WINDOW_MIN_PARTICLES_PER_EVENT = 64


def signature(n_events, n_particles, n_hits, n_cells, outputs):
    """Workloads with the same event count, particle count, hit count (to
    within a factor of two) and outputs share a tuning."""
    hb = int(max(n_hits, 1)).bit_length()
    return f"ev{n_events}-p{n_particles}-h2^{hb}-c{n_cells}-{'+'.join(sorted(outputs))}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(sim, particles, event_offsets, seed, *, outputs=("compact",), hit_energy_scale=100.0,
         candidates=None, reps=3, finalists=4, final_reps=7, final_calls=8,
         cache_path=DEFAULT_CACHE, force=False, out=None, cell_capacity=None, verbose=False):
    """Return the best tuning dict for this workload (cached).  Every
    candidate is timed `reps` times; the `finalists` fastest are timed again,
    `final_reps` times over `final_calls` back-to-back calls each, and the
    fastest median wins."""
    import torch
    info = sim.info()
    q = sim.query_sizes(particles, event_offsets, seed, hit_energy_scale=hit_energy_scale)
    n_events = int(event_offsets.shape[0]) - 1
    n_particles = int(particles.shape[0])
    key = f"{info['device_name']}-cu{info['compute_units']}/" + signature(
        n_events, n_particles, q["n_hits"], info["n_cells"], outputs)
    cache = _load(cache_path)
    if not force and key in cache:
        return dict(cache[key]["tuning"])
    dense = n_particles >= WINDOW_MIN_PARTICLES_PER_EVENT * n_events
    cands = candidates or (WINDOW_CANDIDATES if dense else CANDIDATES)
    cap = q["max_cells"] if cell_capacity is None else cell_capacity
    results = []
    for (c, b, t, w, p) in cands:
        kw = dict(chunk_hits=c, big_task_hits=b, tile_hits=t, wg_per_cu=w)
        if p:
            kw["window_particles"] = p
        run = lambda: sim.simulate_events(particles, event_offsets, seed, outputs=outputs,  # noqa: E731
                                          hit_energy_scale=hit_energy_scale,
                                          cell_capacity=cap, out=out, **kw)
        run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        results.append((ts[len(ts) // 2], kw))
        if verbose:
            print(f"autotune {kw}: {ts[len(ts) // 2] * 1e3:.3f} ms", flush=True)
    results.sort(key=lambda r: r[0])
    # finalists: back-to-back calls, asynchronous when inputs and outputs are
    # on the device (as a serving loop issues them)
    use_async = out is not None and torch.is_tensor(particles) and particles.is_cuda
    final = []
    for _, kw in results[:finalists]:
        ts = []
        for _ in range(final_reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(final_calls):
                sim.simulate_events(particles, event_offsets, seed, outputs=outputs,
                                    hit_energy_scale=hit_energy_scale, cell_capacity=cap,
                                    out=out, async_launch=use_async, **kw)
            if use_async:
                sim.synchronize()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) / final_calls)
        ts.sort()
        final.append((ts[len(ts) // 2], kw))
        if verbose:
            print(f"autotune final {kw}: {ts[len(ts) // 2] * 1e3:.3f} ms", flush=True)
    final.sort(key=lambda r: r[0])
    best_t, best = final[0]
    cache = _load(cache_path)
    cache[key] = {"tuning": best, "ms": best_t * 1e3, "n_candidates": len(results)}
    _store(cache_path, cache)
    return dict(best)


HOST_COPY_CANDIDATES = (1, 2, 3, 4, 6, 8, 16)


def tune_host_copy(sim, particles, event_offsets, seed, host_sets, cell_capacity, *,
                   hit_energy_scale=100.0, tuning=None, candidates=HOST_COPY_CANDIDATES,
                   calls=8, reps=3):
    """Workgroups of the copy kernel that writes the lists of asynchronous
    calls to pinned host buffers (`host_sets`: two dicts of host_empty
    arrays): each candidate is timed over `calls` back-to-back calls, `reps`
    times, and the fastest median wins.  A batch whose compute outlasts its
    copy wants few (the link's traffic slows the kernels beside it); one
    whose copy dominates wants the link's full rate."""
    import numpy as np
    tuning = dict(tuning or {})

    def run(wgs, n):
        for i in range(n):
            sim.simulate_events(particles, event_offsets, seed, outputs=("compact",),
                                out=host_sets[i % 2], cell_capacity=cell_capacity,
                                hit_energy_scale=hit_energy_scale, async_launch=True,
                                host_outputs=True, host_copy_workgroups=wgs, **tuning)
        sim.synchronize()

    best, best_t = None, None
    for wgs in candidates:
        run(wgs, 2)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            run(wgs, calls)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        if best_t is None or t < best_t:
            best, best_t = wgs, t
    return best
