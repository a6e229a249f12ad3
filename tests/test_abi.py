"""CPU checks of the C-ABI library: it loads, exports every function that
include/tslb.h declares, its parameter struct matches the binding, and the
host-side validation and sizing work without touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2403_15773_amd import tslb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(tslb_\w+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tslb.LIB_PATH):
        from paper_2403_15773_amd import build
        build.build()
    return tslb.load_library()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(lib, name), name
    assert declared <= set(tslb.EXPORTS)


def test_params_struct_layout(lib):
    assert lib.tslb_params_size() == ctypes.sizeof(tslb.Params)


def test_defaults_and_required_bytes(lib):
    p = tslb.Params()
    lib.tslb_params_init(ctypes.byref(p))
    assert p.abi_version == tslb.ABI_VERSION and (p.nx, p.ny, p.nz) == (32, 32, 32)
    # FP32: ten moment planes + phi, two buffers, planes padded to 64 elements
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 2 * 11 * 4 * 32 ** 3
    p.storage = tslb.STORE_FP16
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 2 * (10 * 2 + 4) * 32 ** 3
    p.storage = tslb.STORE_FP16Q  # rho', ubar binary32 + six binary16 stress planes + phi
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 2 * (4 * 4 + 6 * 2 + 4) * 32 ** 3
    p.storage = tslb.STORE_FP32
    p.components = 1  # one component: the ten moment planes only
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 2 * 10 * 4 * 32 ** 3
    p.components = 2
    p.nx = 33  # 33*32*32 = 33792 = 528 * 64: still aligned
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 2 * 11 * 4 * 33792
    p.nx, p.ny, p.nz = 5, 3, 3  # 45 -> padded to 64
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 2 * (((10 * 4 * 64 + 255) // 256) * 256 + 4 * 64)


@pytest.mark.parametrize("field,value", [
    ("nu", 0.0), ("nu", -1.0), ("width", 0.0), ("sigma", -1e-3), ("storage", 7), ("abi_version", 99), ("components", 3), ("components", 0),
    ("nx", 0), ("check_interval", -1), ("eps", 0.0), ("eps", 1e-40), ("eps", float("nan")),
    ("max_mass_drift", -1e-6), ("max_mass_drift", float("inf"))])
def test_invalid_parameters_rejected_on_host(lib, field, value):
    p = tslb.Params()
    lib.tslb_params_init(ctypes.byref(p))
    setattr(p, field, value)
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 0
    h = ctypes.c_void_p()
    assert lib.tslb_create(ctypes.byref(p), ctypes.byref(h)) == tslb.E_INVAL
    assert h.value is None
    assert len(lib.tslb_last_error(None)) > 0


def _vd_params(lib, **over):
    p = tslb.Params()
    lib.tslb_params_init(ctypes.byref(p))
    p.variable_density, p.density_a, p.density_b, p.nu_a, p.nu_b = 1, 10.0, 1.0, 0.05, 0.02
    for k, v in over.items():
        if k == "gravity":
            for c in range(3):
                p.gravity[c] = v[c]
        else:
            setattr(p, k, v)
    return p


def test_noalloc_diagnostics_rejects_bad_arguments_on_host(lib):
    """The allocation-free diagnostics entry point checks its arguments before
    any device call."""
    p = tslb.Params()
    lib.tslb_params_init(ctypes.byref(p))
    assert lib.tslb_diagnostics_noalloc(None, 256, None, 256) == tslb.E_INVAL
    assert lib.tslb_diagnostics_noalloc(ctypes.byref(p), None, None, 256) == tslb.E_INVAL
    assert lib.tslb_diagnostics_noalloc(ctypes.byref(p), 256, None, None) == tslb.E_INVAL
    assert lib.tslb_diagnostics_noalloc(ctypes.byref(p), 258, None, 256) == tslb.E_INVAL  # state not 4-byte aligned
    assert lib.tslb_diagnostics_noalloc(ctypes.byref(p), 256, None, 260) == tslb.E_INVAL  # out not 8-byte aligned
    p.nu = -1.0
    assert lib.tslb_diagnostics_noalloc(ctypes.byref(p), 256, None, 256) == tslb.E_INVAL
    p.nu, p.device = 0.1, 4096
    assert lib.tslb_diagnostics_noalloc(ctypes.byref(p), 256, None, 256) == tslb.E_INVAL
    assert len(lib.tslb_last_error(None)) > 0


def test_variable_density_parameters(lib):
    assert lib.tslb_required_bytes(ctypes.byref(_vd_params(lib))) == 2 * 11 * 4 * 32 ** 3
    assert lib.tslb_required_bytes(ctypes.byref(_vd_params(lib, gravity=(0.0, 0.0, -1e-5)))) > 0
    bad = [dict(density_a=0.0), dict(density_b=-1.0), dict(nu_a=0.0), dict(nu_b=-1.0), dict(components=1),
           dict(storage=tslb.STORE_FP16), dict(variable_density=2), dict(gravity=(float("nan"), 0.0, 0.0)),
           dict(density_a=float("inf"))]
    for over in bad:
        p = _vd_params(lib, **over)
        assert lib.tslb_required_bytes(ctypes.byref(p)) == 0, over
        h = ctypes.c_void_p()
        assert lib.tslb_create(ctypes.byref(p), ctypes.byref(h)) == tslb.E_INVAL, over
    # gravity belongs to the variable-density step
    p = _vd_params(lib, variable_density=0, gravity=(0.0, 1e-6, 0.0))
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 0


@pytest.mark.parametrize("bc", [(1, 0, 0, 0, 0, 0), (2, 1, 0, 0, 0, 0), (0, 0, 0, 0, 1, 2), (9, 9, 0, 0, 0, 0)])
def test_invalid_boundary_sets_rejected(lib, bc):
    p = tslb.Params()
    lib.tslb_params_init(ctypes.byref(p))
    for s in range(6):
        p.bc[s] = bc[s]
    p.inlet_d = 4.0
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 0


def test_size_limits(lib):
    """N = nx ny nz < 2^33 and nx ny < 2^30 (the inlet noise counter): the largest
    lattices inside the limits are accepted with exact byte counts, the first
    ones outside are rejected."""
    p = tslb.Params()
    lib.tslb_params_init(ctypes.byref(p))
    p.nx, p.ny, p.nz = 1024, 1024, 8191  # N = 2^33 - 2^20, a multiple of 64
    n = 1024 * 1024 * 8191
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 2 * 11 * 4 * n
    p.nz = 8192  # N = 2^33
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 0
    h = ctypes.c_void_p()
    assert lib.tslb_create(ctypes.byref(p), ctypes.byref(h)) == tslb.E_INVAL and h.value is None
    p.nx, p.ny, p.nz = 32768, 32767, 4  # nx ny = 2^30 - 2^15
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 2 * 11 * 4 * (32768 * 32767 * 4)
    p.ny = 32768  # nx ny = 2^30
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 0


def test_inlet_needs_a_positive_diameter(lib):
    p = tslb.Params()
    lib.tslb_params_init(ctypes.byref(p))
    p.bc[:] = [tslb.BC_FREESLIP, tslb.BC_FREESLIP, tslb.BC_FREESLIP, tslb.BC_FREESLIP, tslb.BC_INLET, tslb.BC_OUTFLOW]
    p.inlet_u = 0.05
    for d in (0.0, -3.0, float("nan")):
        p.inlet_d = d
        assert lib.tslb_required_bytes(ctypes.byref(p)) == 0
    p.inlet_d = 8.0
    assert lib.tslb_required_bytes(ctypes.byref(p)) > 0


def test_thin_axis_with_walls_rejected(lib):
    p = tslb.Params()
    lib.tslb_params_init(ctypes.byref(p))
    p.nx = 3
    p.bc[0] = p.bc[1] = tslb.BC_FREESLIP
    assert lib.tslb_required_bytes(ctypes.byref(p)) == 0


def test_null_context_calls_fail_cleanly(lib):
    assert lib.tslb_step(None, 1) == tslb.E_INVAL
    assert lib.tslb_sync(None) == tslb.E_INVAL
    assert lib.tslb_set_state_rest(None, 0) == tslb.E_INVAL
    assert lib.tslb_step_index(None) == -1
    assert lib.tslb_state_bytes(None) == 0
    assert lib.tslb_device_bytes(None) == 0
    n = ctypes.c_int64(5)
    assert lib.tslb_step_kernel_times(None, None, 0, ctypes.byref(n)) == tslb.E_INVAL
    assert lib.tslb_group_busy(None, None, None) == tslb.E_INVAL
    f, t = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.tslb_device_memory(0, None, ctypes.byref(t)) == tslb.E_INVAL
    lib.tslb_destroy(None)


@pytest.mark.parametrize("kind,nodes,reps", [(2, 64, 1), (0, 100, 1), (1, 0, 1), (0, 64, 0)])
def test_projection_probe_rejects_bad_arguments_on_host(lib, kind, nodes, reps):
    import numpy as np
    coef = np.zeros((16, max(nodes, 1)), np.float32)
    ms = ctypes.c_double()
    rc = lib.tslb_probe_projection(kind, coef.ctypes.data, nodes, reps, 1, 0, None, ctypes.byref(ms))
    assert rc == tslb.E_INVAL and len(lib.tslb_last_error(None)) > 0
