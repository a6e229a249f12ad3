"""The allocation-free diagnostics entry point (tslb_diagnostics_noalloc)
against tslb_diagnostics on the same state, through the C-ABI: two calls in a
row, the second on a smaller lattice, then a non-finite buffer and argument
checks.  Its partial sums live in the library's static device scratch."""
import ctypes

import numpy as np
import pytest

from paper_2403_15773_amd import inputs

pytestmark = pytest.mark.gpu

EPS = 1e-4


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


def _droplet():
    nx, ny, nz = 40, 36, 44
    x, y, z = inputs.grid_coords(nx, ny, nz)
    st = inputs.quiescent(nx, ny, nz)
    st["phi"] = 0.5 * (1 - np.tanh(2 * (np.sqrt((x - 18.2) ** 2 + (y - 19.5) ** 2 + (z - 22.0) ** 2) - 7.0) / 3.0))
    node = np.arange(nx * ny * nz, dtype=np.uint64)
    st["u"] = 0.01 * np.stack([inputs.noise(11, 0, 0, node, a).reshape(nz, ny, nx) for a in range(3)])
    p = dict(nx=nx, ny=ny, nz=nz, nu=0.03, sigma=0.02, width=3.0, bc=(0,) * 6, eps=EPS)
    f = {"rho_dev": np.full((nz, ny, nx), 1e-3, np.float32), "u": st["u"].astype(np.float32),
         "P": st["P"].astype(np.float32), "phi": st["phi"].astype(np.float32)}
    return p, f


def _upload(raw):
    """(device copy of a raw state, device output of three doubles)."""
    from hip_runtime import DeviceBuffer
    dev = DeviceBuffer(raw.nbytes)
    dev.upload(raw)
    out = DeviceBuffer(3 * 8)
    out.upload(np.full(3, -7.0))
    return dev, out


def _run(sim, dev, out, stream):
    """The allocation-free entry point on an uploaded state; waits for it."""
    from paper_2403_15773_amd.tslb import diagnostics_noalloc
    diagnostics_noalloc(sim.params, dev.ptr, stream.handle, out.ptr)
    stream.synchronize()


def _result(out):
    o = out.download(24, dtype=np.float64)
    return float(o[0]), float(o[1]), bool(o[2] == 1.0), o[2]


def _noalloc(sim, raw, stream):
    """Upload a raw state and run the allocation-free entry point on it;
    returns (mass, phase, finite, finite flag)."""
    dev, out = _upload(raw)
    try:
        _run(sim, dev, out, stream)
        return _result(out)
    finally:
        dev.free()
        out.free()


def test_noalloc_diagnostics_match_tslb_diagnostics():
    from hip_runtime import Stream
    from paper_2403_15773_amd.tslb import Simulation, device_memory
    stream = Stream()
    # first call: a 40 x 36 x 44 droplet in binary32 after 6 steps
    _say("noalloc diagnostics: droplet 40x36x44 fp32")
    p, f = _droplet()
    with Simulation(**p) as s:
        s.set_state(**f)
        s.step(6)
        d = s.diagnostics()
        raw = s.get_state_raw()
        mass, phase, finite, flag = _noalloc(s, raw, stream)
    assert mass == d["mass"] and phase == d["phase"] and finite == d["finite"] and flag == 1.0
    assert abs(mass - (40 * 36 * 44) * (1 + 1e-3)) < 1e-6 * mass
    # second call: a smaller jet (boundary layers, 16-bit stress) after 9 steps
    _say("noalloc diagnostics: jet 24x20x32 fp16q")
    q = inputs.jet_params(24, 20, 32, d=6.0, u=0.05, re=600.0, we=40.0, seed=4) | {"eps": EPS}
    with Simulation(**q, storage="fp16q", u_scale=0.05) as s:
        s.set_state_rest()
        s.step(9)
        d = s.diagnostics()
        raw = s.get_state_raw()
        dev, out = _upload(raw)
        free0, _ = device_memory(0)
        _run(s, dev, out, stream)
        free1, _ = device_memory(0)
        mass, phase, finite, flag = _result(out)
        dev.free()
        out.free()
    stream.destroy()
    assert mass == d["mass"] and phase == d["phase"] and finite == d["finite"] and flag == 1.0
    assert phase > 0  # the inlet has brought phase in
    # the call itself allocated no device memory
    assert free1 == free0


def test_noalloc_reports_non_finite_and_rejects_bad_arguments():
    from hip_runtime import Stream, device_synchronize
    from paper_2403_15773_amd import tslb
    _say("noalloc diagnostics: NaN word, bad arguments")
    p, f = _droplet()
    stream = Stream()
    with tslb.Simulation(**p) as s:
        s.set_state(**f)
        raw = s.get_state_raw()
        d = s.diagnostics()
        bad = raw.copy()
        bad.view(np.float32)[3 * (40 * 36 * 44) + 123] = np.nan  # one u_z word
        mass, phase, finite, flag = _noalloc(s, bad, stream)
        assert not finite and flag == 0.0 and phase == d["phase"]
        lib = tslb.load_library()
        dev, out = _upload(raw)
        assert lib.tslb_diagnostics_noalloc(ctypes.byref(s.params), None, None, out.ptr) == tslb.E_INVAL
        assert lib.tslb_diagnostics_noalloc(ctypes.byref(s.params), dev.ptr, None, None) == tslb.E_INVAL
        assert lib.tslb_diagnostics_noalloc(ctypes.byref(s.params), dev.ptr + 2, None, out.ptr) == tslb.E_INVAL
        q = tslb.make_params(**p)
        q.nu = -1.0
        assert lib.tslb_diagnostics_noalloc(ctypes.byref(q), dev.ptr, None, out.ptr) == tslb.E_INVAL
        # the null stream works too
        assert lib.tslb_diagnostics_noalloc(ctypes.byref(s.params), dev.ptr, None, out.ptr) == tslb.OK
        device_synchronize()
        o = out.download(24, dtype=np.float64)
        assert o[0] == d["mass"] and o[1] == d["phase"] and o[2] == 1.0
        dev.free()
        out.free()
    stream.destroy()
