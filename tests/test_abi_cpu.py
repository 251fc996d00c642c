"""The C-ABI library without a GPU: it loads, exports every symbol the
header declares, and checks arguments (device-less context) before any
device work."""
import os
import re

import numpy as np
import pytest

from paper_2103_14737_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    from paper_2103_14737_amd import fcs
    if os.environ.get("FCS_TEST_LIB"):  # another build of the same source
        fcs.LIB_PATH = os.environ["FCS_TEST_LIB"]
    return fcs


def _declared():
    with open(os.path.join(ROOT, "include", "fcs.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fcs_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(F):
    L = F.lib()
    declared = _declared()
    assert set(declared) == set(F.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_create_without_gpu(F):
    import torch
    if torch.cuda.is_available():
        pytest.skip("host has a GPU")
    with pytest.raises(F.FcsError) as e:
        F.Simulator(0)
    assert e.value.code == F.FCS_E_NO_DEVICE


@pytest.fixture()
def dry(F):
    s = F.Simulator(F.FCS_DEVICE_NONE)
    yield s
    s.close()


def test_dry_context_loads_valid_inputs(F, dry):
    dry.load_geometry(W.make_geometry())
    dry.load_parametrization(W.make_param())
    info = dry.info()
    assert info["n_cells"] == 191338 and info["n_histograms"] == 11520 and info["device"] == -1


def _bad_geometry(field, value):
    g = W.make_tiny_geometry()
    g = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    if callable(value):
        value(g)
    else:
        g[field] = value
    return g


@pytest.mark.parametrize("case,needle", [
    ("offset", "reg_offset"),
    ("gap", "does not start"),
    ("ncells", "n_cells"),
    ("layers", "n_layers"),
    ("inv_r", "layer_inv_r"),
    ("neta", "reg_neta"),
])
def test_geometry_validation(F, dry, case, needle):
    if case == "offset":
        g = _bad_geometry(None, lambda g: g["reg_offset"].__setitem__(2, g["reg_offset"][2] + 1))
    elif case == "gap":
        g = _bad_geometry(None, lambda g: g["reg_eta_lo"].__setitem__(1, np.float32(-1.3)))
    elif case == "ncells":
        g = _bad_geometry("n_cells", 5)
    elif case == "layers":
        g = _bad_geometry("n_layers", 0)
    elif case == "inv_r":
        g = _bad_geometry(None, lambda g: g["layer_inv_r"].__setitem__(1, np.float32(np.nan)))
    else:
        g = _bad_geometry(None, lambda g: g["reg_neta"].__setitem__(0, 0))
    with pytest.raises(F.FcsError) as e:
        dry.load_geometry(g)
    assert e.value.code == F.FCS_E_INVALID_ARG
    assert needle in str(e.value)


def test_param_validation(F, dry):
    with pytest.raises(F.FcsError) as e:
        dry.load_parametrization(W.make_param())
    assert e.value.code == F.FCS_E_NOT_LOADED
    dry.load_geometry(W.make_geometry())
    p = W.make_param()
    p["weights"] = p["weights"].copy()
    p["weights"][5] = -1.0
    with pytest.raises(F.FcsError) as e:
        dry.load_parametrization(p)
    assert "weights[5]" in str(e.value)
    p = W.make_param()
    p["weights"] = p["weights"].copy()
    p["weights"][256:512] = 0.0
    with pytest.raises(F.FcsError) as e:
        dry.load_parametrization(p)
    assert "histogram 1 " in str(e.value)
    p = W.make_param(n_layers=3)
    with pytest.raises(F.FcsError) as e:
        dry.load_parametrization(p)
    assert "n_layers" in str(e.value)
    p = W.make_param()
    p["n_rbins"] = 16
    with pytest.raises(F.FcsError):
        dry.load_parametrization(p)


def test_simulate_argument_checks(F, dry):
    dry.load_geometry(W.make_geometry())
    dry.load_parametrization(W.make_param())
    w = W.single_particle_sweep(n_events=5)
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10)
    assert e.value.code == F.FCS_E_NO_DEVICE          # valid arguments reach the device step
    bad = w.particles.copy()
    bad["pdg"][3] = 13
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(bad, w.event_offsets, 1, cell_capacity=10)
    assert e.value.code == F.FCS_E_INVALID_ARG and "particle 3" in str(e.value)
    bad = w.particles.copy()
    bad["e"][1] = -5
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(bad, w.event_offsets, 1, cell_capacity=10)
    assert "energy" in str(e.value)
    off = w.event_offsets.copy()
    off[2], off[3] = off[3], off[2]
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, off, 1, cell_capacity=10)
    assert "decreases" in str(e.value)
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10, tile_hits=300)
    assert "tile_hits" in str(e.value)
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10,
                            hit_energy_scale=0.0)
    assert "hit_energy_scale" in str(e.value)


def test_simulate_needs_loads(F, dry):
    w = W.single_electron()
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10)
    assert e.value.code == F.FCS_E_NOT_LOADED


def test_async_argument_checks(F, dry):
    import ctypes as C
    dry.load_geometry(W.make_geometry())
    dry.load_parametrization(W.make_param())
    w = W.single_particle_sweep(n_events=5)
    # asynchronous calls need device inputs and outputs
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10, async_launch=True)
    assert e.value.code == F.FCS_E_INVALID_ARG and "async_launch" in str(e.value)
    st = F.FcsAsyncStats()
    assert F.lib().fcs_synchronize(dry._h, C.byref(st)) == F.FCS_E_NO_DEVICE
    assert st.n_calls == 0
    o = F.FcsSimOptions()
    F.lib().fcs_default_options(C.byref(o))
    assert o.async_launch == 0 and o.n_particles == 0 and o.reuse_forward_queue == 0
    o.n_particles = -3
    so = F.FcsSimOutput()
    p = np.ascontiguousarray(w.particles)
    off = np.ascontiguousarray(w.event_offsets)
    rc = F.lib().fcs_simulate_events(dry._h, p.ctypes.data, off.ctypes.data, 5, C.byref(o), C.byref(so))
    assert rc == F.FCS_E_INVALID_ARG


def test_async_backward_argument_checks(F, dry):
    import ctypes as C
    dry.load_geometry(W.make_geometry())
    dry.load_parametrization(W.make_param())
    w = W.single_particle_sweep(n_events=5)
    o = F.FcsSimOptions()
    F.lib().fcs_default_options(C.byref(o))
    o.async_launch = 1  # host inputs: refused before any device work
    p = np.ascontiguousarray(w.particles)
    off = np.ascontiguousarray(w.event_offsets)
    g = np.zeros(5 * 191338, np.float32)
    rc = F.lib().fcs_backward(dry._h, p.ctypes.data, off.ctypes.data, 5, C.byref(o), g.ctypes.data,
                              None, None)
    assert rc == F.FCS_E_INVALID_ARG
    assert "async_launch" in F.lib().fcs_last_error(dry._h).decode()


def test_launch_modes(F, dry):
    """The three launch forms are accepted (valid arguments reach the device
    step); other mode numbers are refused before any device work."""
    import ctypes as C
    dry.load_geometry(W.make_geometry())
    dry.load_parametrization(W.make_param())
    w = W.single_particle_sweep(n_events=5)
    for mode in ("batched", "per_event", "per_task"):
        with pytest.raises(F.FcsError) as e:
            dry.simulate_events(w.particles, w.event_offsets, 1, mode=mode, cell_capacity=10)
        assert e.value.code == F.FCS_E_NO_DEVICE, mode
    assert (F.FCS_MODE_BATCHED, F.FCS_MODE_PER_EVENT, F.FCS_MODE_PER_TASK) == (0, 1, 2)
    o = F.FcsSimOptions()
    F.lib().fcs_default_options(C.byref(o))
    o.mode = 3
    o.outputs = 8  # counts only
    so = F.FcsSimOutput()
    cnt = np.zeros(5 * 24, np.int32)
    so.counts = cnt.ctypes.data
    p = np.ascontiguousarray(w.particles)
    off = np.ascontiguousarray(w.event_offsets)
    rc = F.lib().fcs_simulate_events(dry._h, p.ctypes.data, off.ctypes.data, 5, C.byref(o), C.byref(so))
    assert rc == F.FCS_E_INVALID_ARG
    assert "mode" in F.lib().fcs_last_error(dry._h).decode()


def test_backward_refuses_fp64_placement(F, dry):
    import ctypes as C
    dry.load_geometry(W.make_geometry())
    dry.load_parametrization(W.make_param())
    w = W.single_particle_sweep(n_events=5)
    o = F.FcsSimOptions()
    F.lib().fcs_default_options(C.byref(o))
    assert o.placement_fp64 == 0
    o.placement_fp64 = 1
    p = np.ascontiguousarray(w.particles)
    off = np.ascontiguousarray(w.event_offsets)
    g = np.zeros(5 * 191338, np.float32)
    rc = F.lib().fcs_backward(dry._h, p.ctypes.data, off.ctypes.data, 5, C.byref(o), g.ctypes.data,
                              None, None)
    assert rc == F.FCS_E_INVALID_ARG
    assert "placement_fp64" in F.lib().fcs_last_error(dry._h).decode()


def test_chain_variant_options(F, dry):
    """The two chain variants exclude each other; the adjoint takes the
    energy fluctuation (valid arguments reach the device step)."""
    import ctypes as C
    dry.load_geometry(W.make_geometry())
    dry.load_parametrization(W.make_param())
    w = W.single_particle_sweep(n_events=5)
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10, placement_fp64=True,
                            hit_energy_fluct=True)
    assert e.value.code == F.FCS_E_INVALID_ARG and "exclusive" in str(e.value)
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10, hit_energy_fluct=True)
    assert e.value.code == F.FCS_E_NO_DEVICE  # valid: reaches the device step
    o = F.FcsSimOptions()
    F.lib().fcs_default_options(C.byref(o))
    assert o.hit_energy_fluct == 0
    o.hit_energy_fluct = 1
    p = np.ascontiguousarray(w.particles)
    off = np.ascontiguousarray(w.event_offsets)
    g = np.zeros(5 * 191338, np.float32)
    rc = F.lib().fcs_backward(dry._h, p.ctypes.data, off.ctypes.data, 5, C.byref(o), g.ctypes.data,
                              None, None)
    assert rc == F.FCS_E_NO_DEVICE, F.lib().fcs_last_error(dry._h).decode()


def test_min_layer_energy_keeps_hit_energies_normal(F, dry):
    """min_layer_energy_mev must be at least FLT_MIN x nhit_cap (x 2^26 with
    the energy fluctuation): with at most nhit_cap hits no hit energy of a
    layer above the bound is a subnormal FP32 number."""
    dry.load_geometry(W.make_geometry())
    dry.load_parametrization(W.make_param())
    w = W.single_particle_sweep(n_events=3)
    flt_min = float(np.finfo(np.float32).tiny)
    ok = flt_min * 20000 * 1.0001
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10,
                            min_layer_energy=ok)
    assert e.value.code == F.FCS_E_NO_DEVICE         # valid: reaches the device step
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10,
                            min_layer_energy=flt_min * 20000 * 0.999)
    assert e.value.code == F.FCS_E_INVALID_ARG and "min_layer_energy" in str(e.value)
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10,
                            min_layer_energy=ok, hit_energy_fluct=True)
    assert e.value.code == F.FCS_E_INVALID_ARG and "2^26" in str(e.value)
    with pytest.raises(F.FcsError) as e:
        dry.simulate_events(w.particles, w.event_offsets, 1, cell_capacity=10,
                            min_layer_energy=ok * 2 ** 26, hit_energy_fluct=True)
    assert e.value.code == F.FCS_E_NO_DEVICE


def test_noalloc_entry_point_argument_checks(F, dry):
    """fcs_simulate_events_noalloc takes batched mode with device inputs and
    outputs only; valid arguments reach the device step (a device-less
    context never reads the pointers)."""
    import ctypes as C
    dry.load_geometry(W.make_geometry())
    dry.load_parametrization(W.make_param())
    L = F.lib()
    dummy = C.c_void_p(0x1000)

    def call(**kw):
        o = F.FcsSimOptions()
        L.fcs_default_options(C.byref(o))
        o.inputs_on_device = o.outputs_on_device = 1
        o.n_particles = 3
        for k, v in kw.items():
            setattr(o, k, v)
        so = F.FcsSimOutput()
        so.cell_ids = so.cell_e = so.event_cell_offsets = dummy
        so.cell_capacity = 10
        return L.fcs_simulate_events_noalloc(dry._h, dummy, dummy, 3, C.byref(o), C.byref(so))

    assert call() == F.FCS_E_NO_DEVICE
    assert call(mode=F.FCS_MODE_PER_EVENT) == F.FCS_E_INVALID_ARG
    assert "batched mode" in L.fcs_last_error(dry._h).decode()
    assert call(inputs_on_device=0) == F.FCS_E_INVALID_ARG
    assert call(outputs_on_device=0) == F.FCS_E_INVALID_ARG
