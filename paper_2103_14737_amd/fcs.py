"""Python binding of the C ABI in include/fcs.h (ctypes; argument marshalling
only -- every step of the simulation runs in the HIP library).

Inputs may be numpy arrays (host) or torch CUDA tensors (device, the call is
ordered after torch's current stream); outputs follow the inputs: numpy for
host inputs, torch CUDA tensors for device inputs.  torch provides device
memory and streams only.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .workloads import PARTICLE_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfcs.so")

FCS_OK = 0
FCS_E_INVALID_ARG = -1
FCS_E_NOT_LOADED = -2
FCS_E_CAPACITY = -3
FCS_E_HIP = -4
FCS_E_NO_DEVICE = -5
FCS_E_NOMEM = -6
FCS_DEVICE_NONE = -1

FCS_MODE_BATCHED = 0
FCS_MODE_PER_EVENT = 1
FCS_MODE_PER_TASK = 2
FCS_OUT_DENSE = 1
FCS_OUT_COMPACT = 2
FCS_OUT_HITS = 4
FCS_OUT_COUNTS = 8
FCS_OUT_ELAYER = 16
_OUT_NAMES = {"dense": FCS_OUT_DENSE, "compact": FCS_OUT_COMPACT, "hits": FCS_OUT_HITS,
              "counts": FCS_OUT_COUNTS, "elayer": FCS_OUT_ELAYER}

# every symbol include/fcs.h declares
EXPORTS = ("fcs_create", "fcs_destroy", "fcs_last_error", "fcs_get_info", "fcs_host_alloc",
           "fcs_host_free", "fcs_load_geometry", "fcs_load_parametrization",
           "fcs_load_parametrization_async", "fcs_default_options",
           "fcs_simulate_events", "fcs_simulate_events_noalloc", "fcs_query_sizes", "fcs_backward",
           "fcs_synchronize")

_vp = C.c_void_p


class FcsInfo(C.Structure):
    _fields_ = [("device_name", C.c_char * 64), ("compute_units", C.c_int32),
                ("device", C.c_int32), ("n_cells", C.c_int64), ("n_layers", C.c_int32),
                ("n_regions", C.c_int32), ("n_histograms", C.c_int64),
                ("device_bytes", C.c_int64)]


class FcsGeometry(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_layers", C.c_int32), ("n_regions", C.c_int32),
                ("cell_id", _vp), ("reg_eta_lo", _vp), ("reg_eta_hi", _vp),
                ("reg_inv_deta", _vp), ("reg_inv_dphi", _vp), ("reg_phi_lo", _vp),
                ("reg_neta", _vp), ("reg_nphi", _vp), ("reg_offset", _vp),
                ("layer_inv_r", _vp)]


class FcsParam(C.Structure):
    _fields_ = [("n_types", C.c_int32), ("n_ebins", C.c_int32), ("n_etabins", C.c_int32),
                ("n_layers", C.c_int32), ("n_rbins", C.c_int32), ("n_abins", C.c_int32),
                ("r_max_mm", C.c_float), ("e_edges", _vp), ("eta_edges", _vp),
                ("dirichlet_alpha", _vp), ("weights", _vp)]


class FcsSimOptions(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("event_index_base", C.c_uint64), ("mode", C.c_int32),
                ("outputs", C.c_uint32), ("hit_energy_scale_mev", C.c_float),
                ("nhit_cap", C.c_int32), ("min_layer_energy_mev", C.c_double),
                ("chunk_hits", C.c_int32), ("big_task_hits", C.c_int32),
                ("tile_hits", C.c_int32), ("wg_per_cu", C.c_int32), ("use_graph", C.c_int32),
                ("inputs_on_device", C.c_int32), ("outputs_on_device", C.c_int32),
                ("profile", C.c_int32), ("elayer_override", _vp), ("stream", _vp),
                ("n_particles", C.c_int64), ("async_launch", C.c_int32),
                ("reuse_forward_queue", C.c_int32), ("placement_fp64", C.c_int32),
                ("hit_energy_fluct", C.c_int32), ("window_pass", C.c_int32),
                ("window_particles", C.c_int32), ("host_copy_workgroups", C.c_int32)]


class FcsSimOutput(C.Structure):
    _fields_ = [("cells", _vp), ("cell_ids", _vp), ("cell_e", _vp),
                ("event_cell_offsets", _vp), ("cell_capacity", C.c_int64),
                ("hit_eta", _vp), ("hit_phi", _vp), ("hit_e", _vp), ("hit_cell", _vp),
                ("task_hit_offsets", _vp), ("hit_capacity", C.c_int64), ("counts", _vp),
                ("elayer", _vp), ("n_hits", C.c_int64), ("n_hits_out_of_acceptance", C.c_int64),
                ("n_tasks", C.c_int64), ("n_cells_nonzero", C.c_int64),
                ("required_cell_capacity", C.c_int64), ("required_hit_capacity", C.c_int64),
                ("n_work_items", C.c_int64), ("device_ms", C.c_double),
                ("kernel_ms", C.c_double), ("setup_ms", C.c_double), ("compact_ms", C.c_double)]


class FcsAsyncStats(C.Structure):
    _fields_ = [("n_calls", C.c_int64), ("n_hits", C.c_int64),
                ("n_hits_out_of_acceptance", C.c_int64), ("n_cells_nonzero", C.c_int64),
                ("kernel_ms", C.c_double)]


class FcsSizes(C.Structure):
    _fields_ = [("n_hits", C.c_int64), ("n_tasks", C.c_int64), ("max_cells", C.c_int64)]


class FcsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fcs error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libfcs.so; raise if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2103_14737_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.fcs_create.argtypes = [C.POINTER(_vp), C.c_int]
        L.fcs_create.restype = C.c_int
        L.fcs_destroy.argtypes = [_vp]
        L.fcs_destroy.restype = None
        L.fcs_last_error.argtypes = [_vp]
        L.fcs_last_error.restype = C.c_char_p
        L.fcs_get_info.argtypes = [_vp, C.POINTER(FcsInfo)]
        L.fcs_host_alloc.argtypes = [_vp, C.c_int64, C.POINTER(_vp)]
        L.fcs_host_free.argtypes = [_vp, _vp]
        L.fcs_load_geometry.argtypes = [_vp, C.POINTER(FcsGeometry)]
        L.fcs_load_parametrization.argtypes = [_vp, C.POINTER(FcsParam)]
        L.fcs_load_parametrization_async.argtypes = [_vp, C.POINTER(FcsParam)]
        L.fcs_default_options.argtypes = [C.POINTER(FcsSimOptions)]
        L.fcs_default_options.restype = None
        L.fcs_simulate_events.argtypes = [_vp, _vp, _vp, C.c_int64, C.POINTER(FcsSimOptions),
                                          C.POINTER(FcsSimOutput)]
        L.fcs_simulate_events_noalloc.argtypes = L.fcs_simulate_events.argtypes
        L.fcs_query_sizes.argtypes = [_vp, _vp, _vp, C.c_int64, C.POINTER(FcsSimOptions),
                                      C.POINTER(FcsSizes)]
        L.fcs_backward.argtypes = [_vp, _vp, _vp, C.c_int64, C.POINTER(FcsSimOptions), _vp, _vp,
                                   _vp]
        L.fcs_synchronize.argtypes = [_vp, C.POINTER(FcsAsyncStats)]
        for f in ("fcs_get_info", "fcs_host_alloc", "fcs_host_free", "fcs_load_geometry",
                  "fcs_load_parametrization", "fcs_load_parametrization_async",
                  "fcs_simulate_events", "fcs_simulate_events_noalloc", "fcs_query_sizes",
                  "fcs_backward", "fcs_synchronize"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x):
    if x is None:
        return None
    if _is_torch(x):
        return x.data_ptr()
    return x.ctypes.data


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Simulator:
    """One library context on one GPU (or FCS_DEVICE_NONE for argument
    checks without a GPU)."""

    def __init__(self, device: int = 0):
        self._L = lib()
        h = _vp()
        rc = self._L.fcs_create(C.byref(h), device)
        if rc != FCS_OK:
            raise FcsError(rc, self._L.fcs_last_error(None).decode())
        self._h = h
        self._pinned = []
        self.device = device
        self.n_cells = 0
        self.n_layers = 0
        self.n_hist = 0

    def close(self):
        if getattr(self, "_h", None):
            for p in self._pinned:
                self._L.fcs_host_free(self._h, p)
            self._pinned = []
            self._L.fcs_destroy(self._h)
            self._h = None

    def host_empty(self, shape, dtype):
        """A numpy array in pinned host memory from fcs_host_alloc (freed with
        the context): the host outputs of asynchronous calls."""
        dt = np.dtype(dtype)
        n = int(np.prod(shape)) * dt.itemsize
        p = _vp()
        self._check(self._L.fcs_host_alloc(self._h, max(n, 16), C.byref(p)))
        self._pinned.append(p.value)
        buf = (C.c_char * max(n, 16)).from_address(p.value)
        return np.frombuffer(buf, dtype=dt, count=int(np.prod(shape))).reshape(shape)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != FCS_OK:
            raise FcsError(rc, self._L.fcs_last_error(self._h).decode())

    def info(self):
        i = FcsInfo()
        self._check(self._L.fcs_get_info(self._h, C.byref(i)))
        return {k: (getattr(i, k).decode() if k == "device_name" else getattr(i, k))
                for k, _ in FcsInfo._fields_}

    # -------------------------------------------------------------- loads
    def load_geometry(self, g: dict):
        arrs = {
            "cell_id": _host(g["cell_id"], np.int64),
            "reg_eta_lo": _host(g["reg_eta_lo"], np.float32),
            "reg_eta_hi": _host(g["reg_eta_hi"], np.float32),
            "reg_inv_deta": _host(g["reg_inv_deta"], np.float32),
            "reg_inv_dphi": _host(g["reg_inv_dphi"], np.float32),
            "reg_phi_lo": _host(g["reg_phi_lo"], np.float32),
            "reg_neta": _host(g["reg_neta"], np.int32),
            "reg_nphi": _host(g["reg_nphi"], np.int32),
            "reg_offset": _host(g["reg_offset"], np.int32),
            "layer_inv_r": _host(g["layer_inv_r"], np.float32),
        }
        s = FcsGeometry(int(g["n_cells"]), int(g["n_layers"]), int(g["n_regions"]),
                        *[_ptr(arrs[k]) for k, _ in FcsGeometry._fields_[3:]])
        self._check(self._L.fcs_load_geometry(self._h, C.byref(s)))
        self.n_cells = int(g["n_cells"])
        self.n_layers = int(g["n_layers"])

    def load_parametrization(self, p: dict, async_load: bool = False):
        """fcs_load_parametrization, or with async_load
        fcs_load_parametrization_async (the next call uses the new tables;
        calls already enqueued keep the old ones)."""
        arrs = [_host(p["e_edges"], np.float32), _host(p["eta_edges"], np.float32),
                _host(p["alpha"], np.float32), _host(p["weights"], np.float32)]
        s = FcsParam(int(p["n_types"]), int(p["n_ebins"]), int(p["n_etabins"]),
                     int(p["n_layers"]), int(p["n_rbins"]), int(p["n_abins"]),
                     float(p["r_max_mm"]), *[_ptr(a) for a in arrs])
        call = (self._L.fcs_load_parametrization_async if async_load
                else self._L.fcs_load_parametrization)
        self._check(call(self._h, C.byref(s)))
        self.n_hist = arrs[3].size // 256

    # ------------------------------------------------------------ options
    def _options(self, seed, event_index_base, mode, outputs, hit_energy_scale, nhit_cap,
                 min_layer_energy, chunk_hits, big_task_hits, tile_hits, wg_per_cu, use_graph,
                 on_device, elayer_override, stream, n_particles=0, async_launch=False):
        o = FcsSimOptions()
        self._L.fcs_default_options(C.byref(o))
        o.seed = seed
        o.event_index_base = event_index_base
        o.mode = {"batched": FCS_MODE_BATCHED, "per_event": FCS_MODE_PER_EVENT,
                  "per_task": FCS_MODE_PER_TASK}[mode]
        flags = 0
        for n in outputs:
            flags |= _OUT_NAMES[n]
        o.outputs = flags
        o.hit_energy_scale_mev = hit_energy_scale
        o.nhit_cap = nhit_cap
        o.min_layer_energy_mev = min_layer_energy
        o.chunk_hits, o.big_task_hits, o.tile_hits, o.wg_per_cu = (chunk_hits, big_task_hits,
                                                                   tile_hits, wg_per_cu)
        o.use_graph = 1 if use_graph else 0
        o.inputs_on_device = 1 if on_device else 0
        o.outputs_on_device = 1 if on_device else 0
        o.elayer_override = _ptr(elayer_override)
        o.stream = stream
        o.n_particles = n_particles
        o.async_launch = 1 if async_launch else 0
        return o

    def _inputs(self, particles, event_offsets, elayer_override):
        if _is_torch(particles):
            import torch
            assert particles.is_cuda and event_offsets.is_cuda
            assert particles.dtype == torch.int32 and particles.dim() == 2 and particles.shape[1] == 4, \
                "device particles: int32 tensor [N, 4] holding (pdg, e, eta, phi) bit patterns"
            assert event_offsets.dtype == torch.int64
            p = particles.contiguous()
            off = event_offsets.contiguous()
            ov = None if elayer_override is None else elayer_override.contiguous().float()
            stream = torch.cuda.current_stream(particles.device).cuda_stream
            return p, off, ov, True, stream, int(off.shape[0]) - 1
        p = np.ascontiguousarray(particles, PARTICLE_DTYPE)
        off = np.ascontiguousarray(event_offsets, np.int64)
        ov = None if elayer_override is None else np.ascontiguousarray(elayer_override, np.float32)
        return p, off, ov, False, None, len(off) - 1

    # ---------------------------------------------------------- simulate
    def simulate_events(self, particles, event_offsets, seed, *, event_index_base=0,
                        mode="batched", outputs=("compact",), hit_energy_scale=100.0,
                        nhit_cap=20000, min_layer_energy=1e-6, chunk_hits=0, big_task_hits=0,
                        tile_hits=0, wg_per_cu=0, use_graph=True, elayer_override=None,
                        cell_capacity=None, hit_capacity=None, n_particles=None, out=None,
                        profile=False, async_launch=False, placement_fp64=False,
                        hit_energy_fluct=False, noalloc=False, window_pass=0,
                        window_particles=0, host_outputs=False, host_copy_workgroups=0):
        """Run fcs_simulate_events.  Returns a dict of the requested outputs
        (numpy for host inputs, torch CUDA tensors for device inputs) and the
        statistics.  Capacities default to the sizes fcs_query_sizes
        reports.  `out` may pass preallocated device buffers (dict).

        async_launch (device inputs): enqueue and return at once; the outputs
        are full-capacity buffers (event_cell_offsets[-1] holds the compacted
        total), "stats" is None, and synchronize() reports errors and totals.

        placement_fp64: place the hits and look up their cells in FP64 (a
        chain variant of the FP32 contract).  hit_energy_fluct: every hit's
        energy is Ehit times an exponential factor of mean 1 (a chain
        variant).

        noalloc: call fcs_simulate_events_noalloc (batched mode, device inputs
        and outputs; pass `out` buffers and capacities so that the binding
        allocates nothing either).

        window_pass: 0 automatic, 1 always, -1 never deposit the small tasks
        by cell windows (see fcs_sim_options); window_particles tunes it.

        host_outputs (device inputs, async_launch, compact output): `out`
        holds pinned host arrays from host_empty(); the lists are copied
        there after the batch, beside the next one, by a copy kernel of
        host_copy_workgroups workgroups (0: the default; -1: the runtime's
        copy of cell_capacity entries)."""
        p, off, ov, dev, stream, n_events = self._inputs(particles, event_offsets, elayer_override)
        N = (int(p.shape[0]) if dev else len(p)) if n_particles is None else n_particles
        o = self._options(seed, event_index_base, mode, outputs, hit_energy_scale, nhit_cap,
                          min_layer_energy, chunk_hits, big_task_hits, tile_hits, wg_per_cu,
                          use_graph, dev, ov, stream, n_particles=N if dev else 0,
                          async_launch=async_launch)
        o.profile = 1 if profile else 0
        o.placement_fp64 = 1 if placement_fp64 else 0
        o.hit_energy_fluct = 1 if hit_energy_fluct else 0
        o.window_pass = int(window_pass)
        o.window_particles = int(window_particles)
        o.host_copy_workgroups = int(host_copy_workgroups)
        if host_outputs:
            o.outputs_on_device = 0
        L = self.n_layers
        need_sizes = (("compact" in outputs and cell_capacity is None) or
                      ("hits" in outputs and hit_capacity is None))
        if need_sizes and not (out and "cell_ids" in out and cell_capacity is not None):
            s = self.query_sizes(particles, event_offsets, seed, event_index_base=event_index_base,
                                 hit_energy_scale=hit_energy_scale, nhit_cap=nhit_cap,
                                 min_layer_energy=min_layer_energy)
            if cell_capacity is None:
                cell_capacity = s["max_cells"]
            if hit_capacity is None:
                hit_capacity = s["n_hits"]
        res = {} if out is None else dict(out)

        def alloc(name, shape, dtype):
            if name in res:
                return res[name]
            if dev:
                import torch
                tdt = {np.float32: torch.float32, np.int64: torch.int64, np.int32: torch.int32}[dtype]
                a = torch.empty(shape, dtype=tdt, device=p.device)
            else:
                a = np.empty(shape, dtype)
            res[name] = a
            return a

        so = FcsSimOutput()
        if "dense" in outputs:
            so.cells = _ptr(alloc("cells", (n_events, self.n_cells), np.float32))
        if "compact" in outputs:
            cap = max(int(cell_capacity), 1)
            so.cell_ids = _ptr(alloc("cell_ids", (cap,), np.int64))
            so.cell_e = _ptr(alloc("cell_e", (cap,), np.float32))
            so.event_cell_offsets = _ptr(alloc("event_cell_offsets", (n_events + 1,), np.int64))
            so.cell_capacity = int(cell_capacity)
        if "hits" in outputs:
            hc = max(int(hit_capacity), 1)
            for k, dt in (("hit_eta", np.float32), ("hit_phi", np.float32),
                          ("hit_e", np.float32), ("hit_cell", np.int32)):
                setattr(so, k, _ptr(alloc(k, (hc,), dt)))
            so.task_hit_offsets = _ptr(alloc("task_hit_offsets", (N * L + 1,), np.int64))
            so.hit_capacity = int(hit_capacity)
        if "counts" in outputs:
            so.counts = _ptr(alloc("counts", (N * L,), np.int32))
        if "elayer" in outputs:
            so.elayer = _ptr(alloc("elayer", (N * L,), np.float32))
        call = self._L.fcs_simulate_events_noalloc if noalloc else self._L.fcs_simulate_events
        rc = call(self._h, _ptr(p), _ptr(off), n_events, C.byref(o), C.byref(so))
        self._check(rc)
        if async_launch:
            res["stats"] = None
            return res
        stats = {k: getattr(so, k) for k in ("n_hits", "n_hits_out_of_acceptance", "n_tasks",
                                             "n_cells_nonzero", "n_work_items", "device_ms",
                                             "kernel_ms", "setup_ms", "compact_ms")}
        nnz = so.n_cells_nonzero
        if "compact" in outputs:
            res["cell_ids"] = res["cell_ids"][:nnz]
            res["cell_e"] = res["cell_e"][:nnz]
        if "hits" in outputs:
            for k in ("hit_eta", "hit_phi", "hit_e", "hit_cell"):
                res[k] = res[k][:so.n_hits]
        res["stats"] = stats
        return res

    def query_sizes(self, particles, event_offsets, seed, *, event_index_base=0,
                    hit_energy_scale=100.0, nhit_cap=20000, min_layer_energy=1e-6):
        p, off, _, dev, stream, n_events = self._inputs(particles, event_offsets, None)
        o = self._options(seed, event_index_base, "batched", (), hit_energy_scale, nhit_cap,
                          min_layer_energy, 0, 0, 0, 0, False, dev, None, stream,
                          n_particles=int(p.shape[0]) if dev else 0)
        s = FcsSizes()
        self._check(self._L.fcs_query_sizes(self._h, _ptr(p), _ptr(off), n_events, C.byref(o),
                                            C.byref(s)))
        return {"n_hits": s.n_hits, "n_tasks": s.n_tasks, "max_cells": s.max_cells}

    def synchronize(self):
        """fcs_synchronize: wait for the context's work; raise the first error
        of the asynchronous calls; return their summed statistics."""
        st = FcsAsyncStats()
        self._check(self._L.fcs_synchronize(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in FcsAsyncStats._fields_}

    def backward(self, particles, event_offsets, seed, grad_cells, *, event_index_base=0,
                 hit_energy_scale=100.0, nhit_cap=20000, min_layer_energy=1e-6,
                 elayer_override=None, grad_elayer=None, grad_weights=None, chunk_hits=0,
                 big_task_hits=0, tile_hits=0, wg_per_cu=0, need_elayer=True, need_weights=True,
                 async_launch=False, reuse_forward_queue=False, hit_energy_fluct=False):
        """fcs_backward on device tensors: returns (grad_elayer [N*L],
        grad_weights [n_hist*256]) as torch CUDA float32 tensors; a gradient
        with need_* False is not computed and returned as None.  With
        async_launch the call returns once enqueued (torch's current stream
        waits for the gradients); errors are raised by synchronize().
        reuse_forward_queue: the inputs are those of the last batched
        simulate_events call on these device tensors, unchanged; its work
        queue is reused when the library can match the call."""
        import torch
        p, off, ov, dev, stream, n_events = self._inputs(particles, event_offsets, elayer_override)
        assert dev and _is_torch(grad_cells) and grad_cells.is_cuda
        N = int(p.shape[0])
        o = self._options(seed, event_index_base, "batched", (), hit_energy_scale, nhit_cap,
                          min_layer_energy, chunk_hits, big_task_hits, tile_hits, wg_per_cu,
                          False, dev, ov, stream, n_particles=N, async_launch=async_launch)
        o.reuse_forward_queue = 1 if reuse_forward_queue else 0
        o.hit_energy_fluct = 1 if hit_energy_fluct else 0
        g = grad_cells.contiguous().float()
        if not need_elayer:
            grad_elayer = None
        elif grad_elayer is None:
            grad_elayer = torch.empty(N * self.n_layers, dtype=torch.float32, device=g.device)
        if not need_weights:
            grad_weights = None
        elif grad_weights is None:
            grad_weights = torch.empty(self.n_hist * 256, dtype=torch.float32, device=g.device)
        self._check(self._L.fcs_backward(self._h, _ptr(p), _ptr(off), n_events, C.byref(o),
                                         _ptr(g), _ptr(grad_elayer), _ptr(grad_weights)))
        return grad_elayer, grad_weights


def particles_to_device(particles, device="cuda"):
    """numpy PARTICLE_DTYPE array -> int32 [N, 4] CUDA tensor of the same
    16-byte records (the layout fcs_particle has)."""
    import torch
    a = np.ascontiguousarray(particles, PARTICLE_DTYPE).view(np.int32).reshape(-1, 4)
    return torch.from_numpy(a.copy()).to(device)
