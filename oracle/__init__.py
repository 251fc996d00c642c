"""ctypes wrapper of the C oracle (fcs_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "fcs_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wno-unused-function"]


def build(force: bool = True, out: str | None = None, extra=()) -> str:
    """Compile the oracle with gcc (contraction off, no fast math) into `out`
    (default liboracle.so), with `extra` flags (the sanitizer test's)."""
    lib = out or LIB
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, *extra, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, lib)
    return lib


class OgGeom(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_layers", C.c_int32), ("n_regions", C.c_int32),
                ("reg_eta_lo", C.c_void_p), ("reg_eta_hi", C.c_void_p),
                ("reg_inv_deta", C.c_void_p), ("reg_inv_dphi", C.c_void_p),
                ("reg_phi_lo", C.c_void_p), ("reg_neta", C.c_void_p),
                ("reg_nphi", C.c_void_p), ("reg_offset", C.c_void_p),
                ("layer_inv_r", C.c_void_p)]


class OgParam(C.Structure):
    _fields_ = [("n_types", C.c_int32), ("n_ebins", C.c_int32), ("n_etabins", C.c_int32),
                ("n_layers", C.c_int32), ("r_max", C.c_float), ("e_edges", C.c_void_p),
                ("eta_edges", C.c_void_p), ("alpha", C.c_void_p), ("cum", C.c_void_p)]


class OgOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("event_index_base", C.c_uint64),
                ("hit_energy_scale", C.c_float), ("nhit_cap", C.c_int32),
                ("min_layer_energy", C.c_double), ("elayer_override", C.c_void_p),
                ("placement_fp64", C.c_int32), ("hit_energy_fluct", C.c_int32)]


class OgOut(C.Structure):
    _fields_ = [("n_hits", C.c_void_p), ("elayer", C.c_void_p), ("ehit", C.c_void_p),
                ("set", C.c_void_p),
                ("cell_cap", C.c_int64), ("ev_cell_off", C.c_void_p), ("cell_idx", C.c_void_p),
                ("cell_e", C.c_void_p), ("cell_cnt", C.c_void_p),
                ("hit_cap", C.c_int64), ("hit_eta", C.c_void_p), ("hit_phi", C.c_void_p),
                ("hit_e", C.c_void_p), ("hit_cell", C.c_void_p), ("hit_bin", C.c_void_p),
                ("n_hits_total", C.c_int64), ("n_out_of_acc", C.c_int64),
                ("n_cells_nonzero", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("FCS_ORACLE_LIB") or LIB  # another build of the same source
        if path == LIB and not os.path.exists(LIB):
            build()
        L = C.CDLL(path)
        vp, i64, u64, f32, f64, i32, u32 = (C.c_void_p, C.c_int64, C.c_uint64, C.c_float,
                                            C.c_double, C.c_int32, C.c_uint32)
        L.oracle_philox.argtypes = [vp, vp, vp]
        L.oracle_philox_batch.argtypes = [vp, vp, i64, vp]
        L.oracle_log.argtypes = [f64]; L.oracle_log.restype = f64
        L.oracle_exp.argtypes = [f64]; L.oracle_exp.restype = f64
        L.oracle_cos_turns.argtypes = [f64]; L.oracle_cos_turns.restype = f64
        L.oracle_lnfact.argtypes = [i64]; L.oracle_lnfact.restype = f64
        L.oracle_gamma.argtypes = [f64, u64, u32, u32, u32]; L.oracle_gamma.restype = f64
        L.oracle_poisson.argtypes = [f64, u64, u32, u32, u32]; L.oracle_poisson.restype = i64
        L.oracle_select_set.argtypes = [vp, i32, f32, f32]; L.oracle_select_set.restype = i32
        L.oracle_build_cum.argtypes = [vp, i64, vp]; L.oracle_build_cum.restype = C.c_int
        L.oracle_find_bin.argtypes = [vp, f32]; L.oracle_find_bin.restype = i32
        L.oracle_sincos_bin.argtypes = [i32, f32, vp, vp]
        L.oracle_lookup.argtypes = [vp, i32, f32, f32]; L.oracle_lookup.restype = i32
        L.oracle_hit.argtypes = [vp, vp, f32, u64, u32, u32, u32, u32, f32, f32, vp, vp, vp]
        L.oracle_hit.restype = i32
        L.oracle_simulate.argtypes = [vp, vp, vp, vp, i64, vp, vp]; L.oracle_simulate.restype = C.c_int
        L.oracle_perturbed_elayer.argtypes = [vp, vp, vp, i64, vp, f64, vp]
        L.oracle_perturbed_elayer.restype = C.c_int
        L.oracle_gradient.argtypes = [vp, vp, vp, i64, vp, vp, i64, vp, vp, vp, vp]
        L.oracle_gradient.restype = C.c_int
        L.oracle_surrogate_loss.argtypes = [vp, vp, vp, vp, i64, vp, vp, i64, vp, vp]
        L.oracle_surrogate_loss.restype = f64
        for name in ("gamma", "poisson"):
            getattr(L, f"oracle_{name}_batch").argtypes = [f64, u64, i64, vp]
        L.oracle_sincos_batch.argtypes = [vp, vp, i64, vp, vp]
        L.oracle_log_batch.argtypes = [vp, i64, vp]
        L.oracle_exp_batch.argtypes = [vp, i64, vp]
        L.oracle_cos_turns_batch.argtypes = [vp, i64, vp]
        L.oracle_lookup_batch.argtypes = [vp, vp, vp, vp, i64, vp]
        L.oracle_find_bin_batch.argtypes = [vp, vp, i64, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class Geometry:
    """Holds the numpy arrays alive and the C view of a geometry dict."""

    def __init__(self, g):
        self.g = {k: (np.ascontiguousarray(v) if isinstance(v, np.ndarray) else v)
                  for k, v in g.items()}
        gg = self.g
        self.c = OgGeom(gg["n_cells"], gg["n_layers"], gg["n_regions"],
                        _p(gg["reg_eta_lo"]), _p(gg["reg_eta_hi"]), _p(gg["reg_inv_deta"]),
                        _p(gg["reg_inv_dphi"]), _p(gg["reg_phi_lo"]), _p(gg["reg_neta"]),
                        _p(gg["reg_nphi"]), _p(gg["reg_offset"]), _p(gg["layer_inv_r"]))

    @property
    def n_cells(self):
        return self.g["n_cells"]


def build_cum(weights):
    w = np.ascontiguousarray(weights, np.float32)
    n_hist = w.size // 256
    cum = np.empty_like(w)
    rc = lib().oracle_build_cum(_p(w), n_hist, _p(cum))
    if rc != 0:
        raise ValueError("invalid histogram weights")
    return cum


class Param:
    def __init__(self, p, cum=None):
        self.p = dict(p)
        self.weights = np.ascontiguousarray(p["weights"], np.float32)
        self.cum = build_cum(self.weights) if cum is None else cum
        self.e_edges = np.ascontiguousarray(p["e_edges"], np.float32)
        self.eta_edges = np.ascontiguousarray(p["eta_edges"], np.float32)
        self.alpha = np.ascontiguousarray(p["alpha"], np.float32)
        self.c = OgParam(p["n_types"], p["n_ebins"], p["n_etabins"], p["n_layers"],
                         p["r_max_mm"], _p(self.e_edges), _p(self.eta_edges), _p(self.alpha),
                         _p(self.cum))

    @property
    def n_layers(self):
        return self.p["n_layers"]

    @property
    def n_hist(self):
        return self.weights.size // 256


def make_opts(seed, event_index_base=0, hit_energy_scale=100.0, nhit_cap=20000,
              min_layer_energy=1e-6, elayer_override=None, placement_fp64=False,
              hit_energy_fluct=False):
    ov = None if elayer_override is None else np.ascontiguousarray(elayer_override, np.float32)
    o = OgOpts(seed, event_index_base, hit_energy_scale, nhit_cap, min_layer_energy, _p(ov),
               1 if placement_fp64 else 0, 1 if hit_energy_fluct else 0)
    o._keep = ov
    return o


def simulate(geom: Geometry, param: Param, particles, event_offsets, seed, event_index_base=0,
             hit_energy_scale=100.0, nhit_cap=20000, min_layer_energy=1e-6,
             elayer_override=None, hit_list=False, cell_cap=None, hit_cap=None,
             placement_fp64=False, hit_energy_fluct=False):
    """Run the oracle.  Returns a dict of numpy arrays: per-task n/elayer/ehit/
    set, per-event sparse cells (ev_cell_off, cell_idx, cell_e, cell_cnt),
    optional hit list, and stats.  placement_fp64: the hits placed and
    looked up in FP64; hit_energy_fluct: an exponential per-hit energy
    factor (chain variants)."""
    parts = np.ascontiguousarray(particles)
    off = np.ascontiguousarray(event_offsets, np.int64)
    n_ev = len(off) - 1
    N = len(parts)
    L = param.n_layers
    opts = make_opts(seed, event_index_base, hit_energy_scale, nhit_cap, min_layer_energy,
                     elayer_override, placement_fp64, hit_energy_fluct)
    res = {"n": np.zeros(N * L, np.int32), "elayer": np.zeros(N * L, np.float64),
           "ehit": np.zeros(N * L, np.float32), "set": np.zeros(N * L, np.int32)}
    while True:
        if hit_cap is None and hit_list:
            hit_cap = max(1024, 40 * N * L)
        if cell_cap is None:
            cell_cap = max(1024, min(n_ev * geom.n_cells, 4 * 24 * 1000 * N))
        out = OgOut()
        out.n_hits = _p(res["n"]); out.elayer = _p(res["elayer"])
        out.ehit = _p(res["ehit"]); out.set = _p(res["set"])
        ev_cell_off = np.zeros(n_ev + 1, np.int64)
        cell_idx = np.zeros(cell_cap, np.int32)
        cell_e = np.zeros(cell_cap, np.float64)
        cell_cnt = np.zeros(cell_cap, np.int32)
        out.cell_cap = cell_cap
        out.ev_cell_off = _p(ev_cell_off); out.cell_idx = _p(cell_idx)
        out.cell_e = _p(cell_e); out.cell_cnt = _p(cell_cnt)
        hits = None
        if hit_list:
            hits = {"eta": np.zeros(hit_cap, np.float32), "phi": np.zeros(hit_cap, np.float32),
                    "e": np.zeros(hit_cap, np.float32), "cell": np.zeros(hit_cap, np.int32),
                    "bin": np.zeros(hit_cap, np.int32)}
            out.hit_cap = hit_cap
            out.hit_eta = _p(hits["eta"]); out.hit_phi = _p(hits["phi"])
            out.hit_e = _p(hits["e"]); out.hit_cell = _p(hits["cell"])
            out.hit_bin = _p(hits["bin"])
        rc = lib().oracle_simulate(C.byref(geom.c), C.byref(param.c), _p(parts), _p(off), n_ev,
                                   C.byref(opts), C.byref(out))
        if rc == -3:
            cell_cap = max(cell_cap, out.n_cells_nonzero)
            if hit_list:
                hit_cap = max(hit_cap, out.n_hits_total)
            continue
        if rc != 0:
            raise ValueError(f"oracle_simulate failed with code {rc}")
        break
    nnz = out.n_cells_nonzero
    res.update(ev_cell_off=ev_cell_off, cell_idx=cell_idx[:nnz].copy(),
               cell_e=cell_e[:nnz].copy(), cell_cnt=cell_cnt[:nnz].copy(),
               n_hits_total=out.n_hits_total, n_out_of_acc=out.n_out_of_acc,
               n_cells_nonzero=nnz)
    if hit_list:
        nh = out.n_hits_total
        res["hits"] = {k: v[:nh].copy() for k, v in hits.items()}
    return res


def perturbed_elayer(param: Param, particles, event_offsets, seed, sigma=0.2,
                     event_index_base=0, hit_energy_scale=100.0, nhit_cap=20000,
                     min_layer_energy=1e-6):
    parts = np.ascontiguousarray(particles)
    off = np.ascontiguousarray(event_offsets, np.int64)
    opts = make_opts(seed, event_index_base, hit_energy_scale, nhit_cap, min_layer_energy)
    out = np.zeros(len(parts) * param.n_layers, np.float32)
    rc = lib().oracle_perturbed_elayer(C.byref(param.c), _p(parts), _p(off), len(off) - 1,
                                       C.byref(opts), sigma, _p(out))
    if rc != 0:
        raise ValueError(rc)
    return out


def gradient(geom: Geometry, param: Param, particles, event_offsets, seed, grad_cells,
             event_index_base=0, hit_energy_scale=100.0, nhit_cap=20000,
             min_layer_energy=1e-6, elayer_override=None, hit_energy_fluct=False):
    parts = np.ascontiguousarray(particles)
    off = np.ascontiguousarray(event_offsets, np.int64)
    opts = make_opts(seed, event_index_base, hit_energy_scale, nhit_cap, min_layer_energy,
                     elayer_override, hit_energy_fluct=hit_energy_fluct)
    g = np.ascontiguousarray(grad_cells, np.float32)
    dE = np.zeros(len(parts) * param.n_layers, np.float64)
    dW = np.zeros(param.weights.size, np.float64)
    rc = lib().oracle_gradient(C.byref(geom.c), C.byref(param.c), _p(param.weights),
                               param.n_hist, _p(parts), _p(off), len(off) - 1, C.byref(opts),
                               _p(g), _p(dE), _p(dW))
    if rc != 0:
        raise ValueError(rc)
    return dE, dW


def surrogate_loss(geom: Geometry, param: Param, w, particles, event_offsets, seed, targets,
                   event_index_base=0, hit_energy_scale=100.0, nhit_cap=20000,
                   min_layer_energy=1e-6, elayer_override=None, hit_energy_fluct=False):
    parts = np.ascontiguousarray(particles)
    off = np.ascontiguousarray(event_offsets, np.int64)
    opts = make_opts(seed, event_index_base, hit_energy_scale, nhit_cap, min_layer_energy,
                     elayer_override, hit_energy_fluct=hit_energy_fluct)
    w = np.ascontiguousarray(w, np.float64)
    T = np.ascontiguousarray(targets, np.float64)
    return lib().oracle_surrogate_loss(C.byref(geom.c), C.byref(param.c), _p(param.weights),
                                       _p(w), param.n_hist, _p(parts), _p(off), len(off) - 1,
                                       C.byref(opts), _p(T))


def philox(ctr, key):
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, np.uint32)
    out = np.zeros_like(ctr)
    lib().oracle_philox_batch(_p(ctr), _p(key), len(ctr), _p(out))
    return out


def _batch(fn, x, dtype_in, dtype_out):
    x = np.ascontiguousarray(x, dtype_in)
    out = np.zeros(x.shape, dtype_out)
    fn(_p(x), x.size, _p(out))
    return out


def log(x):
    return _batch(lib().oracle_log_batch, x, np.float64, np.float64)


def exp(x):
    return _batch(lib().oracle_exp_batch, x, np.float64, np.float64)


def cos_turns(u):
    return _batch(lib().oracle_cos_turns_batch, u, np.float64, np.float64)


def sincos_bin(ia, u):
    ia = np.ascontiguousarray(ia, np.int32)
    u = np.ascontiguousarray(u, np.float32)
    c = np.zeros(u.shape, np.float32)
    s = np.zeros(u.shape, np.float32)
    lib().oracle_sincos_batch(_p(ia), _p(u), u.size, _p(c), _p(s))
    return c, s


def gamma_batch(alpha, seed, n):
    out = np.zeros(n, np.float64)
    lib().oracle_gamma_batch(alpha, seed, n, _p(out))
    return out


def poisson_batch(mu, seed, n):
    out = np.zeros(n, np.int64)
    lib().oracle_poisson_batch(mu, seed, n, _p(out))
    return out


def lookup(geom: Geometry, layer, eta, phi):
    layer = np.ascontiguousarray(layer, np.int32)
    eta = np.ascontiguousarray(eta, np.float32)
    phi = np.ascontiguousarray(phi, np.float32)
    out = np.zeros(eta.shape, np.int32)
    lib().oracle_lookup_batch(C.byref(geom.c), _p(layer), _p(eta), _p(phi), eta.size, _p(out))
    return out


def find_bin(cum256, u):
    cum256 = np.ascontiguousarray(cum256, np.float32)
    u = np.ascontiguousarray(u, np.float32)
    out = np.zeros(u.shape, np.int32)
    lib().oracle_find_bin_batch(_p(cum256), _p(u), u.size, _p(out))
    return out


def select_set(param: Param, pdg, e, eta):
    return lib().oracle_select_set(C.byref(param.c), int(pdg), float(e), float(eta))


def lnfact(k):
    return lib().oracle_lnfact(int(k))
