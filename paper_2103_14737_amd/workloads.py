"""Seeded synthetic inputs: calorimeter geometry, lateral-shape parametrization
family and particle workloads.

The paper simulates with the ATLAS calorimeter description (187,652 cells in
24 samplings, 78 regions; CUDA Implementation section) and FastCaloSim
parametrization files for single e/gamma/pi between 1 GeV and 4 TeV
(Introduction; Test Data section).  Neither is available, so this module
builds stand-ins of the same shape:

* geometry: 24 layers, each cut into 4 eta regions on |eta| < 3.2 with uniform
  eta x phi grids (fine granularity in |eta| < 1.4), 191,338 cells;
* parametrization: one 32(r) x 8(alpha) lateral histogram per
  (particle type, 16 log-E bins, 10 |eta| bins, layer) with exponentially
  falling radial weights, plus Dirichlet concentrations for the per-layer
  energy split;
* particle workloads: the single-particle sweeps and multi-particle events
  (hard scatter, pile-up) described in the benchmark section.

Everything here is input generation only (numpy, PCG64).  None of the
simulation arithmetic lives here, so the oracle and the device path can both
consume these arrays without sharing any method code.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PDG_E = 11
PDG_GAMMA = 22
PDG_PI = 211

N_LAYERS = 24
N_REGIONS = 4
REGION_BOUNDS = (-3.2, -1.4, 0.0, 1.4, 3.2)
# Layer radius (mm) of the cylinder the lateral shape is projected onto.
LAYER_R_MM = [1450.0, 1550.0, 1700.0, 1900.0, 2000.0, 2100.0] + [
    2300.0 + 100.0 * (l - 6) for l in range(6, 24)
]
# (deta, dphi) of the two central regions (|eta| < 1.4) per layer; the outer
# regions are (0.1, 0.1) everywhere.
CENTRAL_GRAN = [(0.025, 0.1), (0.003, 0.1), (0.025, 0.0245), (0.05, 0.05),
                (0.1, 0.1), (0.1, 0.1)] + [(0.1, 0.1)] * 18
OUTER_GRAN = (0.1, 0.1)

N_TYPES = 3
N_EBINS = 16
N_ETABINS = 10
N_RBINS = 32
N_ABINS = 8
N_BINS = N_RBINS * N_ABINS
R_MAX_MM = 300.0


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def _build_geometry(radii, central, outer, bounds=REGION_BOUNDS):
    n_layers = len(radii)
    n_reg = len(bounds) - 1
    reg = {k: [] for k in ("eta_lo", "eta_hi", "inv_deta", "inv_dphi",
                           "phi_lo", "neta", "nphi", "offset")}
    cell_eta, cell_phi, cell_deta, cell_dphi = [], [], [], []
    cell_layer, cell_id = [], []
    off = 0
    for l in range(n_layers):
        for k in range(n_reg):
            lo, hi = bounds[k], bounds[k + 1]
            width = hi - lo
            is_central = abs(lo) < 1.5 and abs(hi) < 1.5
            deta, dphi = central[l] if is_central else outer[l]
            neta = int(round(width / deta))
            nphi = int(round(2.0 * math.pi / dphi))
            deta_eff = width / neta
            dphi_eff = 2.0 * math.pi / nphi
            reg["eta_lo"].append(lo)
            reg["eta_hi"].append(hi)
            reg["inv_deta"].append(1.0 / deta_eff)
            reg["inv_dphi"].append(1.0 / dphi_eff)
            reg["phi_lo"].append(-math.pi)
            reg["neta"].append(neta)
            reg["nphi"].append(nphi)
            reg["offset"].append(off)
            ie, ip = np.meshgrid(np.arange(neta), np.arange(nphi), indexing="ij")
            ie = ie.ravel()
            ip = ip.ravel()
            cell_eta.append(lo + (ie + 0.5) * deta_eff)
            cell_phi.append(-math.pi + (ip + 0.5) * dphi_eff)
            cell_deta.append(np.full(ie.size, deta_eff))
            cell_dphi.append(np.full(ie.size, dphi_eff))
            cell_layer.append(np.full(ie.size, l))
            cell_id.append((np.int64(l) << 40) | (np.int64(k) << 32)
                           | (ie.astype(np.int64) << 16) | ip.astype(np.int64))
            off += neta * nphi
    g = {
        "n_cells": off,
        "n_layers": n_layers,
        "n_regions": n_reg,
        "cell_eta": np.concatenate(cell_eta).astype(np.float32),
        "cell_phi": np.concatenate(cell_phi).astype(np.float32),
        "cell_deta": np.concatenate(cell_deta).astype(np.float32),
        "cell_dphi": np.concatenate(cell_dphi).astype(np.float32),
        "cell_layer": np.concatenate(cell_layer).astype(np.int32),
        "cell_id": np.concatenate(cell_id).astype(np.int64),
        "reg_eta_lo": np.array(reg["eta_lo"], np.float32),
        "reg_eta_hi": np.array(reg["eta_hi"], np.float32),
        "reg_inv_deta": np.array(reg["inv_deta"], np.float32),
        "reg_inv_dphi": np.array(reg["inv_dphi"], np.float32),
        "reg_phi_lo": np.array(reg["phi_lo"], np.float32),
        "reg_neta": np.array(reg["neta"], np.int32),
        "reg_nphi": np.array(reg["nphi"], np.int32),
        "reg_offset": np.array(reg["offset"], np.int32),
        "layer_r": np.array(radii, np.float32),
        "layer_inv_r": np.array([1.0 / r for r in radii], np.float32),
    }
    return g


def make_geometry():
    """Full synthetic calorimeter: 24 layers x 4 regions, 191,338 cells."""
    return _build_geometry(LAYER_R_MM, CENTRAL_GRAN, [OUTER_GRAN] * N_LAYERS)


def make_tiny_geometry():
    """3 layers x 4 regions of coarse cells (a few hundred) for exhaustive
    brute-force cell-search tests.  Radii are small so that a 300 mm lateral
    spread crosses several cells and region edges."""
    radii = [400.0, 600.0, 900.0]
    central = [(0.2, math.pi / 8), (0.4, math.pi / 4), (0.2, math.pi / 4)]
    outer = [(0.4, math.pi / 4), (0.4, math.pi / 8), (0.3, math.pi / 6)]
    return _build_geometry(radii, central, outer)


# --------------------------------------------------------------------------
# parametrization family
# --------------------------------------------------------------------------
def _lambda_base(t, l):
    em = l < 6
    if t == 0:
        return 18.0 if em else 60.0
    if t == 1:
        return 20.0 if em else 60.0
    return 40.0 if em else 90.0


def _dirichlet_alpha(t, l):
    if t in (0, 1):
        return 2.0 if l < 6 else 0.1
    if l < 6:
        return 0.5
    if l < 12:
        return 2.0
    return 0.1


def make_param(n_layers=N_LAYERS, n_ebins=N_EBINS, n_etabins=N_ETABINS):
    """Histogram family: sets = 3 types x 16 log-E bins x 10 |eta| bins, one
    32 x 8 (r, alpha) histogram per (set, layer); bin b = ir * 8 + ia.
    Weights w = exp(-r_c / lambda) / 8 with r_c the bin's radial centre.
    Finer binnings (up to 64 x 64, about 0.3 M histograms, the table volume
    of a full physics sample) cover the same E and |eta| ranges with the
    same lambda(E, |eta|); the default binning is the 16 x 10 family."""
    e_edges = np.array([1000.0 * 4000.0 ** (k / n_ebins) for k in range(n_ebins + 1)],
                       np.float32)
    eta_edges = np.array([(0.32 * N_ETABINS / n_etabins) * k if n_etabins != N_ETABINS
                          else 0.32 * k for k in range(n_etabins + 1)], np.float32)
    alpha = np.array([[_dirichlet_alpha(t, l) for l in range(n_layers)]
                      for t in range(N_TYPES)], np.float32)
    dr = R_MAX_MM / N_RBINS
    r_c = (np.arange(N_RBINS) + 0.5) * dr
    n_sets = N_TYPES * n_ebins * n_etabins
    w = np.empty((n_sets, n_layers, N_RBINS, N_ABINS), np.float64)
    for t in range(N_TYPES):
        for ie in range(n_ebins):
            for ih in range(n_etabins):
                s = (t * n_ebins + ie) * n_etabins + ih
                # bin index in units of the 16 x 10 binning (exact for it)
                xe, xh = ie * N_EBINS / n_ebins, ih * N_ETABINS / n_etabins
                for l in range(n_layers):
                    lam = _lambda_base(t, l) * (1.0 + 0.04 * xe) * (1.0 + 0.03 * xh)
                    w[s, l] = (np.exp(-r_c / lam) / N_ABINS)[:, None]
    return {
        "n_types": N_TYPES,
        "n_ebins": n_ebins,
        "n_etabins": n_etabins,
        "n_layers": n_layers,
        "n_rbins": N_RBINS,
        "n_abins": N_ABINS,
        "r_max_mm": R_MAX_MM,
        "e_edges": e_edges,
        "eta_edges": eta_edges,
        "alpha": alpha.reshape(-1),
        "weights": w.astype(np.float32).reshape(-1),
    }


# --------------------------------------------------------------------------
# particle workloads
# --------------------------------------------------------------------------
PARTICLE_DTYPE = np.dtype([("pdg", np.int32), ("e", np.float32),
                           ("eta", np.float32), ("phi", np.float32)])


@dataclass
class Workload:
    name: str
    seed: int                      # Philox key for the simulation
    particles: np.ndarray          # PARTICLE_DTYPE [N]
    event_offsets: np.ndarray      # int64 [n_events + 1]
    hit_energy_scale: float = 100.0  # MeV of layer energy per expected hit
    notes: dict = field(default_factory=dict)

    @property
    def n_events(self):
        return len(self.event_offsets) - 1

    @property
    def n_particles(self):
        return len(self.particles)


def _pick_types(rng, n, frac_e, frac_g):
    u = rng.random(n)
    pdg = np.where(u < frac_e, PDG_E, np.where(u < frac_e + frac_g, PDG_GAMMA, PDG_PI))
    sign = np.where(rng.random(n) < 0.5, 1, -1)
    return np.where(pdg == PDG_PI, pdg * sign, pdg).astype(np.int32)


def _power_law_m2(rng, n, lo, hi):
    """E with density proportional to E^-2 on [lo, hi] (inverse CDF)."""
    u = rng.random(n)
    return 1.0 / (1.0 / lo - u * (1.0 / lo - 1.0 / hi))


def _pack(pdg, e, eta, phi):
    p = np.empty(len(pdg), PARTICLE_DTYPE)
    p["pdg"] = pdg
    p["e"] = e.astype(np.float32)
    p["eta"] = eta.astype(np.float32)
    phi32 = phi.astype(np.float32)
    # keep phi inside [-pi_f, pi_f) after rounding to float
    phi32 = np.where(phi32 >= np.float32(math.pi), np.float32(-math.pi), phi32)
    p["phi"] = phi32
    return p


def single_electron():
    """One 65 GeV electron at eta = 0.2, phi = 0 (Philox seed 1234)."""
    p = _pack(np.array([PDG_E]), np.array([65000.0]), np.array([0.2]), np.array([0.0]))
    return Workload("single_electron_65GeV", 1234, p, np.array([0, 1], np.int64))


def single_particle_sweep(n_events=10000, seed=7):
    """Single e/gamma/pi+- (40/20/40) per event, E log-uniform 1 GeV - 4 TeV,
    |eta| < 2.5, phi uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pdg = _pick_types(rng, n_events, 0.4, 0.2)
    e = np.exp(rng.uniform(math.log(1.0e3), math.log(4.0e6), n_events))
    eta = rng.uniform(-2.5, 2.5, n_events)
    phi = rng.uniform(-math.pi, math.pi, n_events)
    return Workload(f"single_particle_sweep_{n_events}ev", seed, _pack(pdg, e, eta, phi),
                    np.arange(n_events + 1, dtype=np.int64))


def hard_scatter(n_events=100, seed=42, n_min=500, n_max=2000):
    """Events of U{500..2000} particles, e/gamma/pi 15/15/70, E ~ E^-2 on
    1-500 GeV, |eta| < 3.2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = rng.integers(n_min, n_max + 1, n_events)
    n = int(counts.sum())
    pdg = _pick_types(rng, n, 0.15, 0.15)
    e = _power_law_m2(rng, n, 1.0e3, 5.0e5)
    eta = rng.uniform(-3.2, 3.2, n)
    phi = rng.uniform(-math.pi, math.pi, n)
    off = np.zeros(n_events + 1, np.int64)
    off[1:] = np.cumsum(counts)
    return Workload(f"hard_scatter_{n_events}ev", seed, _pack(pdg, e, eta, phi), off)


def pileup(n_events=20, seed=99, n_hard=1500, n_pu=200, n_per_pu=60,
           hit_energy_scale=3.0):
    """HL-LHC-like events: a 1500-particle hard scatter (as hard_scatter) plus
    200 pile-up vertices of 60 soft particles (E ~ E^-2 on 0.5-20 GeV)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    per = n_hard + n_pu * n_per_pu
    parts = []
    for _ in range(n_events):
        pdg_h = _pick_types(rng, n_hard, 0.15, 0.15)
        e_h = _power_law_m2(rng, n_hard, 1.0e3, 5.0e5)
        m = n_pu * n_per_pu
        pdg_s = _pick_types(rng, m, 0.15, 0.15)
        e_s = _power_law_m2(rng, m, 5.0e2, 2.0e4)
        pdg = np.concatenate([pdg_h, pdg_s])
        e = np.concatenate([e_h, e_s])
        eta = rng.uniform(-3.2, 3.2, per)
        phi = rng.uniform(-math.pi, math.pi, per)
        parts.append(_pack(pdg, e, eta, phi))
    off = np.arange(n_events + 1, dtype=np.int64) * per
    return Workload(f"pileup_{n_events}ev", seed, np.concatenate(parts), off,
                    hit_energy_scale=hit_energy_scale)


def single_pion_diff(n_events=64, seed=2021):
    """Single pi+- per event (50/50 sign), E log-uniform 10-200 GeV, |eta| < 2.5."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sign = np.where(rng.random(n_events) < 0.5, 1, -1)
    pdg = (PDG_PI * sign).astype(np.int32)
    e = np.exp(rng.uniform(math.log(1.0e4), math.log(2.0e5), n_events))
    eta = rng.uniform(-2.5, 2.5, n_events)
    phi = rng.uniform(-math.pi, math.pi, n_events)
    return Workload(f"single_pion_{n_events}ev", seed, _pack(pdg, e, eta, phi),
                    np.arange(n_events + 1, dtype=np.int64))


def subset_events(w: Workload, first: int, count: int) -> Workload:
    """Events [first, first+count) of a workload; returns the slice and keeps
    the global event index of its first event (offset by the parent's own,
    for a slice of a slice) in notes['event_index_base']."""
    a, b = int(w.event_offsets[first]), int(w.event_offsets[first + count])
    off = w.event_offsets[first:first + count + 1] - w.event_offsets[first]
    sub = Workload(f"{w.name}[{first}:{first + count}]", w.seed, w.particles[a:b].copy(),
                   off.astype(np.int64), w.hit_energy_scale, dict(w.notes))
    sub.notes["event_index_base"] = int(w.notes.get("event_index_base", 0)) + first
    return sub


BY_NAME = {
    "single_electron": single_electron,
    "single_particle_sweep": single_particle_sweep,
    "hard_scatter": hard_scatter,
    "pileup": pileup,
    "single_pion_diff": single_pion_diff,
}
